"""Parity at the full benchmark size (8192^2 Fourier modes + blasts, periodic),
in the launch configuration bench.py times: dt over the whole grid, then one
full step checked on sampled columns.  The oracle reproduces a column after a
step from the input alone: the x-swept value of cell (x, y) needs only cells
x-4..x+4 of row y (two 5-cell stencils), and the y-sweep of column x needs only
that column."""
import numpy as np
import pytest

from paper_2106_13465_amd import inputs

pytestmark = pytest.mark.gpu

N = 8192


@pytest.fixture(scope="module")
def state():
    return inputs.fourier_blasts(N)


def oracle_column_after_step(orc, U, x, dt, c):
    nv, ny, n = U.shape
    h = 1.0 / n
    lam = dt / h
    cols = np.arange(x - 4, x + 5) % n
    xs = np.empty((nv, ny))
    for y in range(ny):
        w = np.ascontiguousarray(U[:, y, cols])  # (rho, rho u, rho v, E, rho X): normal = x
        w1 = orc.pencil(w, lam, c)
        xs[:, y] = w1[:, 4]
    # y-sweep of the column: pencil order (rho, rho v, rho u, E, rho X), periodic ghosts
    order = [0, 2, 1, 3] + list(range(4, nv))
    w = np.empty((nv, ny + 4))
    col = xs[order]
    w[:, 2:-2] = col
    w[:, :2] = col[:, -2:]
    w[:, -2:] = col[:, :2]
    w1 = orc.pencil(w, lam, c)
    return w1[order, 2:-2]


def sample_columns(U):
    # columns through the blasts plus seeded ordinary ones (incl. the edges)
    blast_cols = np.nonzero(np.any(U[3] > 1e6, axis=0))[0]
    rng = np.random.Generator(np.random.PCG64(77))
    cols = list(blast_cols[:4]) + [0, N - 1] + list(rng.integers(0, N, 4))
    return sorted(set(int(c) for c in cols))


@pytest.mark.parametrize("dtype_name,riemann,ns,ysweep", [
    ("f64", 0, 0, 0), ("f32", 0, 0, 0), ("f64", 1, 0, 0), ("f64", 2, 0, 0), ("f64", 0, 1, 0),
    ("f64", 0, 0, 1), ("f32", 0, 0, 1)])
def test_fullsize_step(torch_cuda_fs, orc, state, dtype_name, riemann, ns, ysweep):
    torch = torch_cuda_fs
    from paper_2106_13465_amd.hydro import Hydro

    U = state
    if ns:
        U = inputs.with_scalars(U, inputs.random_scalars(N, N, seed=7, k=ns))
    print(f"fullsize {dtype_name} solver {riemann} scalars {ns} ysweep {ysweep}: 8192^2 one step",
          flush=True)
    c = orc.cfg(bc=orc.BC_PERIODIC, riemann=riemann, nscalars=ns)
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    h = Hydro(N, N, 1.4, 0.8, "periodic", dtype=dtype, nscalars=ns)
    h.set_options(riemann=riemann, ysweep=ysweep)
    h.set_state(U)
    if riemann == 0 and ns == 0:
        h.autotune(use_cache=True)  # the launch shape bench.py times
    dt_or = orc.compute_dt(U, c)
    if dtype_name == "f64":
        assert abs(h.compute_dt() - dt_or) <= 1e-13 * dt_or
    h.step(1)
    t, n, dt_gpu = h.clock()
    assert n == 1
    if dtype_name == "f64":
        assert abs(dt_gpu - dt_or) <= 1e-13 * dt_or
    G = h.get_state()
    h.close()
    from test_gpu_parity import momentum_err_away_from_blasts, var_scales

    for x in sample_columns(U):
        ref = oracle_column_after_step(orc, U, x, dt_or, c)
        got = G[:, :, x].astype(np.float64)
        scales = var_scales(ref)
        if dtype_name == "f64":
            away = momentum_err_away_from_blasts(got, ref)
            print(f"column {x} momentum away from blasts / max|m| {away:.2e}")
            assert away <= 1e-12, (x, away)
        for k in range(4 + ns):
            if dtype_name == "f64":
                err = np.max(np.abs(got[k] - ref[k]) / scales[k])
                print(f"column {x} var {k} rel err {err:.2e}")
                assert err <= 1e-12, (x, k, err)
            else:
                l1 = np.abs(got[k] - ref[k]).sum() / max(np.abs(ref[k]).sum(), 1e-300)
                assert l1 < 1e-5, (x, k, l1)


@pytest.fixture(scope="module")
def torch_cuda_fs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch
