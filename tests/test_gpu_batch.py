"""Batched path: many uneven grids advanced by one launch per sweep, each with
its own dt.  Checked per grid against the FP64 oracle, against single-grid
handles (bitwise: same kernels), under graph replay and under the autotuner's
launch shapes."""
import numpy as np
import pytest

from paper_2106_13465_amd import inputs
from test_gpu_parity import TOL64, rel_err

pytestmark = pytest.mark.gpu

GRIDS = [  # (nx, ny, bc, generator seed)
    (70, 33, 1, 1), (2, 5, 3, 2), (128, 128, 2, 3), (61, 190, 3, 4), (300, 7, 1, 5),
    (64, 64, 3, 6), (17, 121, 2, 7),
]


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def batch_inputs():
    return [inputs.random_states(nx, ny, seed=100 + s, rough=0.6) for nx, ny, _, s in GRIDS]


def make_batch(torch, states, dtype=None, **opts):
    from paper_2106_13465_amd.hydro import HydroBatch

    b = HydroBatch([(nx, ny) for nx, ny, _, _ in GRIDS], 1.4, 0.8, [g[2] for g in GRIDS],
                   dtype=dtype or torch.float64)
    if opts:
        b.set_options(**opts)
    b.set_states(states)
    return b


def test_batch_matches_oracle_per_grid(torch_cuda, orc):
    states = batch_inputs()
    b = make_batch(torch_cuda, states)
    dts = b.compute_dt()
    for g, U in enumerate(states):
        ref_dt = orc.compute_dt(U, orc.cfg(bc=GRIDS[g][2]))
        assert abs(dts[g] - ref_dt) <= 1e-13 * ref_dt
    b.step(6)
    got = b.get_states()
    t, n, _ = b.clock()
    for g, U in enumerate(states):
        c = orc.cfg(bc=GRIDS[g][2])
        ref = U.copy()
        t_or = sum(orc.step(ref, c) for _ in range(6))
        assert n[g] == 6 and abs(t[g] - t_or) <= 1e-13 * t_or
        assert rel_err(got[g], ref) <= TOL64, g
    T = b.totals()
    assert T.shape == (len(GRIDS), 4)
    for g in range(len(GRIDS)):
        R = orc.totals(np.ascontiguousarray(got[g]))
        A = np.abs(got[g]).sum(axis=(1, 2)) / max(got[g].shape[1:]) ** 2
        assert np.all(np.abs(T[g] - R) <= 1e-14 * A), g


def test_batch_equals_single_handles_bitwise(torch_cuda, orc):
    from paper_2106_13465_amd.hydro import Hydro

    states = batch_inputs()
    b = make_batch(torch_cuda, states)
    b.step(4)
    got = b.get_states()
    for g, U in enumerate(states):
        nx, ny, bc, _ = GRIDS[g]
        h = Hydro(nx, ny, 1.4, 0.8, bc)
        h.set_state(U)
        h.step(4)
        assert np.array_equal(h.get_state(), got[g]), g


def test_batch_graph_replay(torch_cuda):
    states = batch_inputs()
    a = make_batch(torch_cuda, states)
    e = make_batch(torch_cuda, states)
    for rep in range(3):
        a.graph_steps(2)
        e.step(2)
        for x, y in zip(a.get_states(), e.get_states()):
            assert np.array_equal(x, y), rep
        a.step(1)
        e.step(1)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_autotune_does_not_change_results(torch_cuda, dtype_name):
    dtype = torch_cuda.float64 if dtype_name == "f64" else torch_cuda.float32
    states = batch_inputs()
    a = make_batch(torch_cuda, states, dtype)
    b = make_batch(torch_cuda, states, dtype)
    tune = b.autotune(use_cache=False)
    assert tune["candidates"] > 4 and tune["ms_x"] > 0 and tune["ms_y"] > 0
    # the tuner's timing sweeps left the bound state untouched
    for x, y in zip(b.get_states(), states):
        assert np.array_equal(x, y.astype(x.dtype))
    again = b.autotune(use_cache=True)
    assert again["cached"] == 1 and again["seg_x"] == tune["seg_x"]
    a.step(3)
    b.step(3)
    for x, y in zip(a.get_states(), b.get_states()):
        assert np.array_equal(x, y)


def test_single_grid_autotune(torch_cuda, orc):
    from paper_2106_13465_amd.hydro import Hydro

    U = inputs.random_states(333, 257, seed=9, rough=0.5)
    a = Hydro(333, 257, 1.4, 0.8, 3)
    a.set_state(U)
    b = Hydro(333, 257, 1.4, 0.8, 3)
    b.set_state(U)
    print("tune", b.autotune(use_cache=False))
    a.step(2)
    b.step(2)
    assert np.array_equal(a.get_state(), b.get_state())


def test_batch_totals_and_fp32(torch_cuda, orc):
    states = batch_inputs()
    b = make_batch(torch_cuda, states, torch_cuda.float32)
    b.step(5)
    got = b.get_states()
    T = b.totals()
    for g, U in enumerate(states):
        c = orc.cfg(bc=GRIDS[g][2])
        ref = U.copy()
        for _ in range(5):
            orc.step(ref, c)
        G = got[g].astype(np.float64)
        for k in range(4):
            l1 = np.abs(G[k] - ref[k]).sum() / max(np.abs(ref[k]).sum(), 1e-300)
            assert l1 < 1e-5, (g, k, l1)
        tot = orc.totals(np.ascontiguousarray(G))
        A = np.abs(G).sum(axis=(1, 2)) / max(G.shape[1:]) ** 2
        assert np.all(np.abs(T[g] - tot) <= 1e-13 * A + 1e-300), g


def test_many_tiny_grids(torch_cuda, orc):
    """300 grids of 2..17 cells a side with all three boundary types: the work
    list's grid search and the per-grid dt over many small entries."""
    from paper_2106_13465_amd.hydro import HydroBatch

    rng = np.random.Generator(np.random.PCG64(77))
    shapes = [(int(rng.integers(2, 18)), int(rng.integers(2, 18))) for _ in range(300)]
    bcs = [int(b) for b in rng.integers(1, 4, size=300)]
    states = [inputs.random_states(nx, ny, seed=1000 + g, rough=0.6)
              for g, (nx, ny) in enumerate(shapes)]
    b = HydroBatch(shapes, 1.4, 0.8, bcs, dtype=torch_cuda.float64)
    b.set_states(states)
    b.step(3)
    got = b.get_states()
    for g, U in enumerate(states):
        ref = U.copy()
        c = orc.cfg(bc=bcs[g])
        for _ in range(3):
            orc.step(ref, c)
        assert rel_err(got[g], ref) <= TOL64, (g, shapes[g], bcs[g])


@pytest.mark.parametrize("shape", [(4096, 2), (2, 4096), (3001, 3)])
def test_extreme_aspect_ratios(torch_cuda, orc, shape):
    from paper_2106_13465_amd.hydro import Hydro

    nx, ny = shape
    U = inputs.random_states(nx, ny, seed=nx + ny, rough=0.6)
    h = Hydro(nx, ny, 1.4, 0.8, "periodic", dtype=torch_cuda.float64)
    h.set_state(U)
    h.step(4)
    ref = U.copy()
    c = orc.cfg(bc=3)
    for _ in range(4):
        orc.step(ref, c)
    assert rel_err(h.get_state(), ref) <= TOL64
