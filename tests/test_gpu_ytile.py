"""The tiled y-sweep (options.ysweep = tile: 16 x 64 tiles transposed through
LDS, swept one cell per lane with the x-sweep's code) against the FP64 oracle
and against the default column march: single sweeps for every boundary type,
steps, the other limiters and solvers, a passive scalar, batches, statistics,
launch shapes and the autotuner."""
import numpy as np
import pytest

from paper_2106_13465_amd import inputs
from test_gpu_parity import CASES, TOL64, make, rel_err

pytestmark = pytest.mark.gpu

TILE = 1


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name,gen", CASES + [
    ("ragged", lambda: inputs.random_states(37, 130, seed=24)),
    ("tall", lambda: inputs.random_smooth(3, 250, seed=25, amp=0.5))])
@pytest.mark.parametrize("bc", [1, 2, 3])
def test_tile_single_y_sweep_fp64(torch_cuda, orc, name, gen, bc):
    U = gen()
    print(f"tile y-sweep {name} bc={bc} shape={U.shape}", flush=True)
    h = make(torch_cuda, U, bc, ysweep=TILE)
    c = orc.cfg(bc=bc)
    dt = h.compute_dt()
    h.sweep(1)
    ref = U.copy()
    orc.sweep(ref, 1, dt, c)
    assert rel_err(h.get_state(), ref) <= TOL64


@pytest.mark.parametrize("bc", [1, 2, 3])
def test_tile_steps_fp64_and_fp32(torch_cuda, orc, bc):
    U = inputs.random_states(97, 131, seed=60 + bc, rough=0.5)
    print(f"tile steps bc={bc}", flush=True)
    c = orc.cfg(bc=bc)
    ref = U.copy()
    t_or = sum(orc.step(ref, c) for _ in range(8))
    h = make(torch_cuda, U, bc, ysweep=TILE)
    h.step(8)
    t, n, _ = h.clock()
    assert n == 8 and abs(t - t_or) <= 1e-13 * t_or
    assert rel_err(h.get_state(), ref) <= TOL64
    h32 = make(torch_cuda, U, bc, dtype=torch_cuda.float32, ysweep=TILE)
    h32.step(8)
    got = h32.get_state().astype(np.float64)
    for k in range(4):
        assert np.abs(got[k] - ref[k]).sum() < 1e-5 * np.abs(ref[k]).sum(), k


@pytest.mark.parametrize("opts", [dict(limiter=1), dict(limiter=2), dict(riemann=1),
                                  dict(riemann=2), dict(order=1)])
def test_tile_with_options(torch_cuda, orc, opts):
    U = inputs.random_states(70, 121, seed=71, rough=0.6)
    print(f"tile options {opts}", flush=True)
    c = orc.cfg(bc=3, **opts)
    ref = U.copy()
    for s in range(5):
        orc.step(ref, c, step_index=s)  # odd steps y first with the alternating order
    h = make(torch_cuda, U, 3, ysweep=TILE, **opts)
    h.step(5)
    assert rel_err(h.get_state(), ref) <= TOL64


def test_tile_passive_scalar(torch_cuda, orc):
    from paper_2106_13465_amd.hydro import Hydro

    nx, ny = 66, 140
    U = inputs.with_scalars(inputs.random_states(nx, ny, seed=72, rough=0.6),
                            inputs.random_scalars(nx, ny, seed=73, k=1))
    c = orc.cfg(bc=1, nscalars=1)
    ref = U.copy()
    for _ in range(4):
        orc.step(ref, c)
    h = Hydro(nx, ny, 1.4, 0.8, 1, dtype=torch_cuda.float64, nscalars=1)
    h.set_options(ysweep=TILE)
    h.set_state(U)
    h.step(4)
    assert rel_err(h.get_state(), ref) <= TOL64


def test_tile_matches_march_and_launch_shapes(torch_cuda, orc):
    """Tiles and march agree to the parity bar; the autotuner's choice of
    persistent block counts for the tiled sweep gives the bitwise same state as
    one block per tile."""
    U = inputs.random_smooth(150, 260, seed=74, amp=0.5)
    a = make(torch_cuda, U, 3)
    a.step(4)
    march = a.get_state()
    h = make(torch_cuda, U, 3, ysweep=TILE)
    h.step(4)
    tile = h.get_state()
    assert rel_err(tile, march) <= TOL64
    h = make(torch_cuda, U, 3, ysweep=TILE)
    tune = h.autotune(use_cache=False)
    print("tile autotune", tune)
    h.set_state(U)
    h.step(4)
    assert np.array_equal(h.get_state(), tile)


def test_tile_stats_match_oracle_histogram(torch_cuda, orc):
    U = inputs.random_states(130, 70, seed=42)
    h = make(torch_cuda, U, 2, stats=1, ysweep=TILE)
    h.step(1)
    s = h.stats()
    assert s["interfaces"] == (130 + 1) * 70 + (70 + 1) * 130
    hist = np.zeros(11, dtype=np.int64)
    ref = U.copy()
    orc.step(ref, orc.cfg(bc=2), hist)
    g = np.array(s["hist"][:11])
    assert g.sum() == hist.sum()
    assert np.abs(g - hist).sum() <= 0.01 * hist.sum()
    # per-wave groups: x-sweep 3 segments per row; tiled y-sweep one
    # 60-row segment per tile column (130 columns x 2 tiles of rows)
    w = np.array(s["wave_hist"][:11])
    assert w.sum() == 70 * 3 + 130 * 2
    assert rel_err(h.get_state(), ref) <= TOL64


def test_tile_batch(torch_cuda, orc):
    from paper_2106_13465_amd.hydro import HydroBatch

    grids = [(70, 33, 1, 1), (2, 5, 3, 2), (128, 128, 2, 3), (61, 190, 3, 4), (17, 121, 2, 7)]
    states = [inputs.random_states(nx, ny, seed=100 + s, rough=0.6) for nx, ny, _, s in grids]
    b = HydroBatch([(nx, ny) for nx, ny, _, _ in grids], 1.4, 0.8, [g[2] for g in grids],
                   dtype=torch_cuda.float64)
    b.set_options(ysweep=TILE)
    b.set_states(states)
    b.step(5)
    got = b.get_states()
    for g, U in enumerate(states):
        c = orc.cfg(bc=grids[g][2])
        ref = U.copy()
        for _ in range(5):
            orc.step(ref, c)
        assert rel_err(got[g], ref) <= TOL64, g


def test_tile_graph_replay(torch_cuda, orc):
    U = inputs.random_states(90, 77, seed=75, rough=0.5)
    a = make(torch_cuda, U, 3, ysweep=TILE)
    a.step(6)
    b = make(torch_cuda, U, 3, ysweep=TILE)
    b.graph_steps(3)
    b.graph_steps(3)
    assert np.array_equal(a.get_state(), b.get_state())
