"""Options beyond the default method: the MC and van Leer limiters, the
alternating sweep order and the exact / HLLC interface solvers, each against
the FP64 oracle with the same option, including graph replay (whose captured
sweep order depends on the starting step's parity) and the batched path."""
import numpy as np
import pytest

from paper_2106_13465_amd import inputs
from test_gpu_parity import TOL64, make, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("bc", [1, 3])
@pytest.mark.parametrize("limiter", [1, 2])
def test_limiters_fp64(torch_cuda, orc, limiter, bc):
    U = inputs.random_states(130, 75, seed=60 + limiter, rough=0.6)
    h = make(torch_cuda, U, bc, limiter=limiter)
    h.step(5)
    ref = U.copy()
    c = orc.cfg(bc=bc, limiter=limiter)
    for _ in range(5):
        orc.step(ref, c)
    assert rel_err(h.get_state(), ref) <= TOL64


@pytest.mark.parametrize("limiter", [0, 1, 2])
def test_limiters_fp32_l1(torch_cuda, orc, limiter):
    U = inputs.random_smooth(160, 120, seed=70, amp=0.5)
    h = make(torch_cuda, U, 3, dtype=torch_cuda.float32, limiter=limiter)
    h.step(10)
    ref = U.copy()
    c = orc.cfg(bc=3, limiter=limiter)
    for _ in range(10):
        orc.step(ref, c)
    got = h.get_state().astype(np.float64)
    for k in range(4):
        assert np.abs(got[k] - ref[k]).sum() / np.abs(ref[k]).sum() < 1e-5


@pytest.mark.parametrize("bc", [1, 2, 3])
def test_alternating_order_fp64(torch_cuda, orc, bc):
    U = inputs.random_states(110, 90, seed=80 + bc, rough=0.6)
    h = make(torch_cuda, U, bc, order=1)
    h.step(6)
    t, step, _ = h.clock()
    ref = U.copy()
    c = orc.cfg(bc=bc, order=1)
    t_or = sum(orc.step(ref, c, step_index=s) for s in range(6))
    assert step == 6 and abs(t - t_or) <= 1e-13 * t_or
    assert rel_err(h.get_state(), ref) <= TOL64


def test_alternating_order_graph_parity(torch_cuda, orc):
    """Graph replays of 3 steps start on alternating parities (the graph is
    recaptured for each); the result equals 6 eager steps bitwise and the
    oracle's 6 steps with the same order."""
    U = inputs.random_states(96, 70, seed=91, rough=0.6)
    a = make(torch_cuda, U, 3, order=1)
    b = make(torch_cuda, U, 3, order=1)
    a.step(6)
    b.graph_steps(3)
    b.graph_steps(3)
    np.testing.assert_array_equal(b.get_state(), a.get_state())
    ref = U.copy()
    c = orc.cfg(bc=3, order=1)
    for s in range(6):
        orc.step(ref, c, step_index=s)
    assert rel_err(b.get_state(), ref) <= TOL64


def test_alternating_order_restart(torch_cuda, orc):
    """A restart at an odd step count resumes with the y-first order."""
    U = inputs.random_states(64, 48, seed=92, rough=0.6)
    a = make(torch_cuda, U, 2, order=1)
    a.step(3)
    mid = a.get_state()
    t, step, _ = a.clock()
    a.step(2)
    b = make(torch_cuda, mid, 2, order=1)
    b.set_clock(t, step)
    b.step(2)
    np.testing.assert_array_equal(b.get_state(), a.get_state())


def test_batch_options(torch_cuda, orc):
    from paper_2106_13465_amd.hydro import HydroBatch

    shapes = [(70, 33), (45, 91), (128, 64)]
    bcs = [1, 3, 2]
    states = [inputs.random_states(nx, ny, seed=200 + g, rough=0.6)
              for g, (nx, ny) in enumerate(shapes)]
    b = HydroBatch(shapes, 1.4, 0.8, bcs, dtype=torch_cuda.float64)
    b.set_options(limiter=2, order=1)
    b.set_states(states)
    b.graph_steps(2)
    b.step(3)
    got = b.get_states()
    for g, U in enumerate(states):
        ref = U.copy()
        c = orc.cfg(bc=bcs[g], limiter=2, order=1)
        for s in range(5):
            orc.step(ref, c, step_index=s)
        assert rel_err(got[g], ref) <= TOL64, g


def test_option_validation(torch_cuda):
    from paper_2106_13465_amd.hydro import Hydro, HydroError

    h = Hydro(16, 16, 1.4, 0.8, "periodic")
    with pytest.raises(HydroError):
        h.set_options(limiter=3)
    with pytest.raises(HydroError):
        h.set_options(order=2)
    o = h.options()
    assert o["limiter"] == 0 and o["order"] == 0 and o["riemann"] == 0


# ------------------------------------------------------------------ solvers
@pytest.mark.parametrize("bc", [1, 2, 3])
@pytest.mark.parametrize("riemann", [1, 2])
def test_solvers_fp64(torch_cuda, orc, riemann, bc):
    U = inputs.random_states(130, 75, seed=300 + 10 * riemann + bc, rough=0.6)
    h = make(torch_cuda, U, bc, riemann=riemann)
    h.step(5)
    t, _, _ = h.clock()
    ref = U.copy()
    c = orc.cfg(bc=bc, riemann=riemann)
    t_or = sum(orc.step(ref, c) for _ in range(5))
    assert abs(t - t_or) <= 1e-13 * t_or
    assert rel_err(h.get_state(), ref) <= TOL64


@pytest.mark.parametrize("riemann", [1, 2])
def test_solvers_single_sweeps_fp64(torch_cuda, orc, riemann):
    """One x- and one y-sweep of a rough state, each against the oracle's."""
    U = inputs.random_states(97, 66, seed=320 + riemann, rough=0.9)
    for direction in (0, 1):
        h = make(torch_cuda, U, 3, riemann=riemann)
        dt = h.compute_dt()
        h.sweep(direction)
        ref = U.copy()
        orc.sweep(ref, direction, dt, orc.cfg(bc=3, riemann=riemann))
        assert rel_err(h.get_state(), ref) <= TOL64, direction


@pytest.mark.parametrize("riemann", [1, 2])
def test_solvers_fp32_l1(torch_cuda, orc, riemann):
    U = inputs.random_smooth(160, 120, seed=330, amp=0.5)
    h = make(torch_cuda, U, 3, dtype=torch_cuda.float32, riemann=riemann)
    h.step(10)
    ref = U.copy()
    c = orc.cfg(bc=3, riemann=riemann)
    for _ in range(10):
        orc.step(ref, c)
    got = h.get_state().astype(np.float64)
    for k in range(4):
        assert np.abs(got[k] - ref[k]).sum() / np.abs(ref[k]).sum() < 1e-5


def test_exact_solver_iteration_histogram(torch_cuda, orc):
    """Newton iteration counts of the exact solver against the oracle's
    (an integer decided in floating point: within 1% of interfaces)."""
    U = inputs.random_states(120, 80, seed=340, rough=0.8)
    h = make(torch_cuda, U, 3, riemann=1, stats=1)
    h.step(1)
    s = h.stats()
    ref = U.copy()
    hist = np.zeros(11, dtype=np.int64)
    orc.step(ref, orc.cfg(bc=3, riemann=1), hist)
    g = np.array(s["hist"][:11])
    assert g.sum() == hist.sum() > 0
    assert np.abs(g - hist).sum() <= 0.01 * hist.sum()


def test_hllc_counts_nothing(torch_cuda, orc):
    U = inputs.random_states(64, 40, seed=341, rough=0.5)
    h = make(torch_cuda, U, 3, riemann=2, stats=1)
    h.step(2)
    s = h.stats()
    assert s["interfaces"] == 0 and sum(s["hist"]) == 0


@pytest.mark.parametrize("riemann", [1, 2])
def test_solvers_with_other_options(torch_cuda, orc, riemann):
    """Each solver with the MC / van Leer limiters and the alternating
    order, through graph replays (bitwise equal to eager steps)."""
    lim = 1 if riemann == 1 else 2
    U = inputs.random_states(90, 70, seed=350 + riemann, rough=0.6)
    a = make(torch_cuda, U, 1, riemann=riemann, limiter=lim, order=1)
    b = make(torch_cuda, U, 1, riemann=riemann, limiter=lim, order=1)
    a.step(5)
    b.graph_steps(2)
    b.graph_steps(3)
    np.testing.assert_array_equal(b.get_state(), a.get_state())
    ref = U.copy()
    c = orc.cfg(bc=1, riemann=riemann, limiter=lim, order=1)
    for s in range(5):
        orc.step(ref, c, step_index=s)
    assert rel_err(a.get_state(), ref) <= TOL64


def test_batch_solvers(torch_cuda, orc):
    from paper_2106_13465_amd.hydro import HydroBatch

    shapes = [(70, 33), (45, 91), (128, 64)]
    bcs = [2, 3, 1]
    states = [inputs.random_states(nx, ny, seed=360 + g, rough=0.6)
              for g, (nx, ny) in enumerate(shapes)]
    for riemann in (1, 2):
        b = HydroBatch(shapes, 1.4, 0.8, bcs, dtype=torch_cuda.float64)
        b.set_options(riemann=riemann)
        b.set_states(states)
        b.graph_steps(3)
        got = b.get_states()
        for g, U in enumerate(states):
            ref = U.copy()
            c = orc.cfg(bc=bcs[g], riemann=riemann)
            for _ in range(3):
                orc.step(ref, c)
            assert rel_err(got[g], ref) <= TOL64, (riemann, g)


def test_solver_option_validation(torch_cuda):
    from paper_2106_13465_amd.hydro import Hydro, HydroError

    h = Hydro(16, 16, 1.4, 0.8, "periodic")
    with pytest.raises(HydroError):
        h.set_options(riemann=3)
    with pytest.raises(HydroError):
        h.set_options(riemann=2, guess=1)
    assert h.options()["riemann"] == 0


# ------------------------------------------------------------------ passive scalars
def with_scalar(U, seed):
    _, ny, nx = U.shape
    return inputs.with_scalars(U, inputs.random_scalars(nx, ny, seed=seed))


def make_s(torch_cuda, V, bc, dtype=None, **opts):
    from paper_2106_13465_amd.hydro import Hydro

    dtype = dtype or torch_cuda.float64
    _, ny, nx = V.shape
    h = Hydro(nx, ny, 1.4, 0.8, bc, dtype=dtype, nscalars=V.shape[0] - 4)
    if opts:
        h.set_options(**opts)
    h.set_state(V)
    return h


@pytest.mark.parametrize("bc", [1, 2, 3])
@pytest.mark.parametrize("riemann", [0, 1, 2])
def test_scalar_steps_fp64(torch_cuda, orc, riemann, bc):
    V = with_scalar(inputs.random_states(110, 70, seed=400 + bc, rough=0.6), 10 + riemann)
    h = make_s(torch_cuda, V, bc, riemann=riemann)
    h.step(5)
    ref = V.copy()
    c = orc.cfg(bc=bc, riemann=riemann, nscalars=1)
    for _ in range(5):
        orc.step(ref, c)
    assert rel_err(h.get_state(), ref) <= TOL64


@pytest.mark.parametrize("riemann", [0, 2])
def test_scalar_single_sweeps_fp64(torch_cuda, orc, riemann):
    V = with_scalar(inputs.random_states(97, 66, seed=410, rough=0.9), 11)
    for direction in (0, 1):
        h = make_s(torch_cuda, V, 1, riemann=riemann)
        dt = h.compute_dt()
        h.sweep(direction)
        ref = V.copy()
        orc.sweep(ref, direction, dt, orc.cfg(bc=1, riemann=riemann, nscalars=1))
        assert rel_err(h.get_state(), ref) <= TOL64, direction


def test_scalar_uniform_follows_density(torch_cuda):
    U = inputs.random_states(90, 60, seed=411, rough=0.7)
    V = inputs.with_scalars(U, np.full((60, 90), 0.5))
    h = make_s(torch_cuda, V, 1, limiter=1, order=1)
    h.step(6)
    S = h.get_state()
    np.testing.assert_allclose(S[4], 0.5 * S[0], rtol=1e-14, atol=0)


def test_scalar_with_options_graph_and_stats(torch_cuda, orc):
    """MC limiter, alternating order and statistics with a scalar, through
    graph replays (bitwise equal to eager steps) and against the oracle."""
    V = with_scalar(inputs.random_states(96, 72, seed=412, rough=0.6), 12)
    a = make_s(torch_cuda, V, 3, limiter=1, order=1, stats=1)
    b = make_s(torch_cuda, V, 3, limiter=1, order=1)
    a.step(4)
    b.graph_steps(1)
    b.graph_steps(3)
    np.testing.assert_array_equal(b.get_state(), a.get_state())
    ref = V.copy()
    hist = np.zeros(11, dtype=np.int64)
    c = orc.cfg(bc=3, limiter=1, order=1, nscalars=1)
    for s in range(4):
        orc.step(ref, c, hist, step_index=s)
    assert rel_err(a.get_state(), ref) <= TOL64
    g = np.array(a.stats()["hist"][:11])
    assert g.sum() == hist.sum() and np.abs(g - hist).sum() <= 0.01 * hist.sum()


def test_scalar_totals(torch_cuda, orc):
    V = with_scalar(inputs.random_states(80, 50, seed=413, rough=0.6), 13)
    h = make_s(torch_cuda, V, 3)
    T0 = h.totals()
    assert len(T0) == 5
    np.testing.assert_allclose(T0, orc.totals(V), rtol=1e-14, atol=1e-16)
    h.step(5)
    T1 = h.totals()
    assert abs(T1[4] - T0[4]) <= 1e-13 * np.abs(V[4]).mean()


@pytest.mark.parametrize("riemann", [0, 2])
def test_scalar_fp32_l1(torch_cuda, orc, riemann):
    U = inputs.random_smooth(150, 110, seed=414, amp=0.5)
    X = 2.0 + np.sin(np.linspace(0.0, 6.0, 150))[None, :] * np.cos(np.linspace(0.0, 4.0, 110))[:, None]
    V = inputs.with_scalars(U, X)
    h = make_s(torch_cuda, V, 3, dtype=torch_cuda.float32, riemann=riemann)
    h.step(10)
    ref = V.copy()
    c = orc.cfg(bc=3, riemann=riemann, nscalars=1)
    for _ in range(10):
        orc.step(ref, c)
    got = h.get_state().astype(np.float64)
    for k in range(5):
        assert np.abs(got[k] - ref[k]).sum() / np.abs(ref[k]).sum() < 1e-5, k


def test_scalar_batch(torch_cuda, orc):
    from paper_2106_13465_amd.hydro import HydroBatch

    shapes = [(70, 33), (45, 91), (128, 64)]
    bcs = [3, 1, 2]
    states = [with_scalar(inputs.random_states(nx, ny, seed=420 + g, rough=0.6), 20 + g)
              for g, (nx, ny) in enumerate(shapes)]
    b = HydroBatch(shapes, 1.4, 0.8, bcs, dtype=torch_cuda.float64, nscalars=1)
    b.set_options(riemann=1)
    b.set_states(states)
    b.graph_steps(2)
    b.step(1)
    got = b.get_states()
    tot = b.totals()
    assert tot.shape == (3, 5)
    for g, V in enumerate(states):
        ref = V.copy()
        c = orc.cfg(bc=bcs[g], riemann=1, nscalars=1)
        for _ in range(3):
            orc.step(ref, c)
        assert rel_err(got[g], ref) <= TOL64, g
        np.testing.assert_allclose(tot[g], orc.totals(ref), rtol=1e-12, atol=1e-14)


def test_scalar_count_checks(torch_cuda):
    from paper_2106_13465_amd import _lib
    from paper_2106_13465_amd.hydro import Hydro, HydroError

    with pytest.raises(HydroError):
        Hydro(16, 16, 1.4, 0.8, "periodic", nscalars=2)
    h = Hydro(16, 16, 1.4, 0.8, "periodic", nscalars=1)
    assert h.lib.hydro_set_scalars(h.handle, 0) == _lib.HYDRO_ESTATE
    with pytest.raises(ValueError):
        h.set_state(np.ones((4, 16, 16)))
