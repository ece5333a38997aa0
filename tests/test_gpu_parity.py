"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on the
same seeded inputs.  FP64 bar: per variable max|U_gpu - U_oracle| / scale <= 1e-12
(dt <= 1e-13 relative), where the scale of rho and E is their max magnitude and
the scale of a momentum component is, cell by cell, max(max|m|, sqrt(2 rho_i E_i)):
the larger of the component's max magnitude and the cell's own momentum scale
(|m| <= sqrt(2 rho E) in every cell).  A cell's momentum update is the difference
of the pressure impulses through its two faces (Figure 5, incoming fluxes); at a
point blast those impulses exceed the cell's momentum by orders of magnitude, so
there its rounding error lives on the cell's sqrt(2 rho E).  Away from blasts
sqrt(2 rho E) is within a small factor of max|m|, so the bar there stays 1e-12
of the momentum itself."""
import math

import numpy as np
import pytest

from paper_2106_13465_amd import inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def var_scales(b):
    """Scale of each conserved variable of the reference state b [4 + ns, ...]:
    max |.| for rho, E and the passive scalars' rho X (scalars); for each
    momentum component an array of per-cell scales max(max|m|, sqrt(2 rho E))."""
    cell = np.sqrt(2.0 * np.abs(b[0]) * np.abs(b[3]))
    scales = [np.max(np.abs(b[0])), np.maximum(np.max(np.abs(b[1])), cell),
              np.maximum(np.max(np.abs(b[2])), cell), np.max(np.abs(b[3]))]
    scales += [np.max(np.abs(b[k])) for k in range(4, b.shape[0])]
    return [np.where(s > 0, s, 1.0) if np.ndim(s) else (s if s > 0 else 1.0) for s in scales]


def rel_err(a, b):
    """Per-variable relative error (momenta per cell), max over every plane."""
    assert a.shape == b.shape
    return max(np.max(np.abs(a[k] - b[k]) / s) for k, s in enumerate(var_scales(b)))


def momentum_err_away_from_blasts(a, b, factor=10.0):
    """Momentum error over max|m| alone, in the cells whose own momentum scale
    sqrt(2 rho E) is within `factor` of max|m| (every cell but the blasts and
    their immediate neighbourhood); 0 if no cell qualifies."""
    cell = np.sqrt(2.0 * np.abs(b[0]) * np.abs(b[3]))
    err = 0.0
    for k in (1, 2):
        m = np.max(np.abs(b[k]))
        mask = cell <= factor * max(m, 1e-300)
        if m > 0 and np.any(mask):
            err = max(err, np.max(np.abs(a[k] - b[k])[mask]) / m)
    return err


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make(torch_cuda, U, bc, dtype=None, **opts):
    from paper_2106_13465_amd.hydro import Hydro

    dtype = dtype or torch_cuda.float64
    _, ny, nx = U.shape
    h = Hydro(nx, ny, 1.4, 0.8, bc, dtype=dtype)
    if opts:
        h.set_options(**opts)
    h.set_state(U)
    return h


CASES = [
    ("random", lambda: inputs.random_states(133, 70, seed=21)),
    ("smooth", lambda: inputs.random_smooth(70, 133, seed=22, amp=0.5)),
    ("tiny", lambda: inputs.random_states(2, 3, seed=23)),
    ("blast", lambda: inputs.blast_corner(64)),
]


@pytest.mark.parametrize("name,gen", CASES)
@pytest.mark.parametrize("bc", [1, 2, 3])
@pytest.mark.parametrize("direction", [0, 1])
def test_single_sweep_fp64(torch_cuda, orc, name, gen, bc, direction):
    U = gen()
    print(f"case {name} bc={bc} dir={direction} shape={U.shape}", flush=True)
    h = make(torch_cuda, U, bc)
    c = orc.cfg(bc=bc)
    dt_gpu = h.compute_dt()
    dt_or = orc.compute_dt(U, c)
    assert abs(dt_gpu - dt_or) <= 1e-13 * dt_or
    h.sweep(direction)
    ref = U.copy()
    orc.sweep(ref, direction, dt_gpu, c)
    assert rel_err(h.get_state(), ref) <= TOL64


@pytest.mark.parametrize("bc", [1, 2, 3])
def test_steps_fp64(torch_cuda, orc, bc):
    U = inputs.random_states(97, 61, seed=30 + bc, rough=0.5)
    print(f"steps bc={bc}", flush=True)
    h = make(torch_cuda, U, bc)
    c = orc.cfg(bc=bc)
    ref = U.copy()
    t_or = 0.0
    for _ in range(10):
        t_or += orc.step(ref, c)
    h.step(10)
    t, n, dt = h.clock()
    assert n == 10
    assert abs(t - t_or) <= 1e-13 * t_or
    assert rel_err(h.get_state(), ref) <= TOL64


def test_blast_corner_100_steps_fp64(torch_cuda, orc):
    """The 128^2 corner point explosion, reflective walls, 100 steps."""
    U = inputs.blast_corner(128)
    print("blast128 100 steps", flush=True)
    h = make(torch_cuda, U, 1)
    c = orc.cfg(bc=1)
    ref = U.copy()
    for _ in range(100):
        orc.step(ref, c)
    h.step(100)
    got = h.get_state()
    err = rel_err(got, ref)
    away = momentum_err_away_from_blasts(got, ref)
    print("blast128 rel err", err, "momentum away from the blast / max|m|", away)
    assert err <= TOL64
    assert away <= TOL64


def test_totals_fp64(torch_cuda, orc):
    U = inputs.random_states(300, 211, seed=40)
    h = make(torch_cuda, U, 3)
    T = h.totals()
    R = orc.totals(U)
    A = np.abs(U).sum(axis=(1, 2)) / 300**2
    assert np.all(np.abs(T - R) <= 1e-14 * A)


def test_uniform_unchanged(torch_cuda, orc):
    U = inputs.uniform(150, 77, 1.3, 0.37, -0.61, 0.8)
    h = make(torch_cuda, U, 3)
    h.step(5)
    assert np.array_equal(h.get_state(), U)


def test_segments_do_not_change_results(torch_cuda, orc):
    """Launch shape (segments per wave, marching length) leaves results
    bitwise unchanged."""
    U = inputs.random_states(250, 190, seed=41, rough=0.5)
    outs = []
    for sx, sy in [(1, 128), (3, 7), (5, 190), (2, 64)]:
        h = make(torch_cuda, U, 3, seg_x=sx, seg_y=sy)
        h.step(3)
        outs.append(h.get_state())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("pitch", [1001, 1013])
@pytest.mark.parametrize("dtype_name", ["float64", "float32"])
def test_staged_stores_any_row_alignment(torch_cuda, orc, dtype_name, pitch):
    """The x-sweep parks updated cells in LDS and stores whole 64-cell blocks
    aligned to the output address.  Rows of 1001 cells (16 whole segments and
    a partial one) at a pitch that gives every row another alignment, and work
    items of 1, 2, 7 and 16 segments (item ends inside a block, a last item
    running past the row's end): one x-sweep gives the same bits for every
    segment count and matches the oracle (FP64 to the bar, FP32 by relative
    L1).  With the pitch equal to the row length a store past a row's end
    would land in the next row; with padding, the padding stays untouched."""
    from paper_2106_13465_amd.hydro import Hydro

    dt = getattr(torch_cuda, dtype_name)
    nx, ny = 1001, 23
    U = inputs.random_states(nx, ny, seed=57, rough=0.5)
    c = orc.cfg(bc=3)
    outs = []
    for sx in (1, 2, 7, 16):
        print(f"staged stores {dtype_name} seg_x={sx} nx={nx} pitch={pitch}", flush=True)
        h = Hydro(nx, ny, 1.4, 0.8, 3, dtype=dt, pitch=pitch)
        h.set_options(seg_x=sx)
        h.set_state(U)
        h.U[:, :, nx:] = -7.0
        torch_cuda.cuda.synchronize()
        dt_gpu = h.compute_dt()
        h.sweep(0)
        h.stream.synchronize()
        full = h.U.cpu().numpy()
        assert np.all(full[:, :, nx:] == -7.0)
        outs.append(full)
        h.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ref = U.copy()
    orc.sweep(ref, 0, dt_gpu, c)
    got = outs[0][:, :, :nx].astype(np.float64)
    if dtype_name == "float64":
        assert rel_err(got, ref) <= TOL64
    else:
        for k in range(4):
            assert np.sum(np.abs(got[k] - ref[k])) <= 1e-5 * np.sum(np.abs(ref[k]))


def test_stats_counts(torch_cuda, orc):
    U = inputs.random_states(130, 70, seed=42)
    h = make(torch_cuda, U, 2, stats=1)
    c = orc.cfg(bc=2)
    h.step(1)
    s = h.stats()
    assert s["interfaces"] == (130 + 1) * 70 + (70 + 1) * 130
    hist = np.zeros(11, dtype=np.int64)
    ref = U.copy()
    orc.step(ref, c, hist)
    g = np.array(s["hist"][:11])
    assert g.sum() == hist.sum()
    # iteration counts may differ where rounding decides a convergence test
    assert np.abs(g - hist).sum() <= 0.01 * hist.sum()
    # per-wave maxima: one group per x-sweep segment (3 per row of 130 cells)
    # and per y-sweep interface row of each 64-column group (71 x 3)
    w = np.array(s["wave_hist"][:11])
    assert w.sum() == 70 * 3 + 71 * 3
    assert w[0] == 0
    top = 10 if g[0] else int(np.nonzero(g)[0].max())
    assert int(np.nonzero(w)[0].max()) == top
    assert 64 * (w * np.arange(11)).sum() >= (g * np.arange(11)).sum() + 10 * g[0]


@pytest.mark.parametrize("amp", [1e-3, 3e-2])
def test_smooth_guess_iterations_and_parity(torch_cuda, orc, amp):
    """Smooth fields, FP64: at amplitude 1e-3 every x-sweep wave has its
    face-pressure ratios within 2^-10 of 1, where the kernel takes the
    two-rarefaction guess's power from its binomial series; at 3e-2 waves of
    both kinds occur.  The guess must be as good as the oracle's: the same
    iteration histogram (a wrong series term would cost a second iteration
    almost everywhere) and the state to the FP64 bar."""
    U = inputs.random_smooth(190, 70, seed=24, amp=amp)
    print(f"smooth amp={amp}", flush=True)
    h = make(torch_cuda, U, 3, stats=1)
    c = orc.cfg(bc=3)
    hist = np.zeros(11, dtype=np.int64)
    ref = U.copy()
    for _ in range(3):
        orc.step(ref, c, hist)
    h.step(3)
    g = np.array(h.stats()["hist"][:11])
    assert g.sum() == hist.sum()
    assert np.abs(g - hist).sum() <= 0.001 * hist.sum()
    assert rel_err(h.get_state(), ref) <= TOL64


@pytest.mark.parametrize("bc", [1, 3])
def test_fp32_l1(torch_cuda, orc, bc):
    U = inputs.random_smooth(160, 120, seed=43, amp=0.5)
    h = make(torch_cuda, U, bc, dtype=torch_cuda.float32)
    c = orc.cfg(bc=bc)
    ref = U.copy()
    for _ in range(10):
        orc.step(ref, c)
    h.step(10)
    got = h.get_state().astype(np.float64)
    for k in range(4):
        l1 = np.abs(got[k] - ref[k]).sum() / max(np.abs(ref[k]).sum(), 1e-300)
        print("fp32 L1", k, l1)
        assert l1 < 1e-5


@pytest.mark.parametrize("fam", [dict(p_decades=2.0, rho_decades=1.0, speed=2.0),
                                 dict(p_decades=4.0, rho_decades=2.0, speed=3.0)])
def test_fp32_strong_jumps_all_converge(torch_cuda, orc, fam):
    """FP32 on strong jumps: the Newton loop stops once its residual is at
    rounding level, so no interface runs to the cap, and the step stays
    within the FP32 L1 bound of the oracle's FP64 step."""
    U = inputs.strong_jumps(256, 192, 41, **fam)
    h = make(torch_cuda, U, 3, dtype=torch_cuda.float32, stats=1)
    h.step(1)
    s = h.stats()
    print("fp32 strong jumps", fam, "unconverged", s["hist"][0], "interfaces", s["interfaces"])
    assert s["interfaces"] == 257 * 192 + 193 * 256
    assert s["hist"][0] == 0
    ref = U.copy()
    orc.step(ref, orc.cfg(bc=3))
    got = h.get_state().astype(np.float64)
    for k in range(4):
        l1 = np.abs(got[k] - ref[k]).sum() / np.abs(ref[k]).sum()
        assert l1 < 1e-5, (k, l1)


@pytest.mark.parametrize("n", [128, 256])
def test_fp32_error_below_truncation(torch_cuda, orc, n):
    """Equal accuracy: a density wave rho = 1 + 0.2 sin(2 pi (x + y)) carried
    by (u, v) = (1, 1) at p = 1 on a periodic grid has the exact solution
    rho(x - t, y - t).  After 100 steps the FP32 state's L1 distance from the
    FP64 state is at least ten times below the FP64 scheme's own error
    against the exact solution (its truncation error)."""
    h_ = 1.0 / n
    x = (np.arange(n) + 0.5) * h_
    X, Y = np.meshgrid(x, x)
    U = inputs.conservative(1.0 + 0.2 * np.sin(2 * np.pi * (X + Y)), 1.0, 1.0, 1.0)
    a = make(torch_cuda, U, 3)
    b = make(torch_cuda, U, 3, dtype=torch_cuda.float32)
    a.step(100)
    b.step(100)
    t, _, _ = a.clock()
    exact = 1.0 + 0.2 * np.sin(2 * np.pi * (X + Y - 2 * t))
    r64 = a.get_state()[0]
    r32 = b.get_state()[0].astype(np.float64)
    trunc = np.abs(r64 - exact).sum() / np.abs(exact).sum()
    fp32 = np.abs(r32 - r64).sum() / np.abs(r64).sum()
    print(f"n={n} t={t:.4f} truncation L1 {trunc:.2e} FP32 L1 {fp32:.2e}")
    assert fp32 <= 0.1 * trunc


def test_graph_replay_matches_eager(torch_cuda, orc):
    """A captured multi-step graph, replayed several times with eager steps and
    host synchronisation in between, matches eager stepping bitwise after
    every replay."""
    U = inputs.random_states(200, 150, seed=44, rough=0.5)
    a = make(torch_cuda, U, 3)
    b = make(torch_cuda, U, 3)
    for rep in range(4):
        a.graph_steps(3)
        b.step(3)
        ga, gb = a.get_state(), b.get_state()
        assert np.array_equal(ga, gb), f"replay {rep}"
        assert a.clock()[1] == b.clock()[1] == 3 * (rep + 1) + rep
        a.step(1)
        b.step(1)
    ref = U.copy()
    c = orc.cfg(bc=3)
    for _ in range(16):
        orc.step(ref, c)
    assert a.clock()[1] == 16
    assert rel_err(a.get_state(), ref) <= TOL64


@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.3])
def test_other_gamma_steps(torch_cuda, orc, gamma):
    """gamma = 5/3 (integer exponent 2 gamma/(gamma-1) = 5 in the guess) and
    gamma = 1.3 (non-integer exponent): 5 steps of a random state against the
    oracle."""
    from paper_2106_13465_amd.hydro import Hydro

    U = inputs.random_states(140, 90, seed=31, gamma=gamma, rough=0.8)
    h = Hydro(140, 90, gamma, 0.8, 2)
    h.set_state(U)
    h.set_options(stats=1)
    h.step(5)
    ref = U.copy()
    c = orc.cfg(gamma=gamma, bc=2)
    hist = np.zeros(11, dtype=np.int64)  # Newton cap 10
    for _ in range(5):
        orc.step(ref, c, hist)
    assert rel_err(h.get_state(), ref) <= TOL64
    s = h.stats()
    # Newton iteration counts: the guesses differ in their last bits, so a
    # count may differ on a few interfaces; the unconverged ones must agree
    g = np.array(s["hist"][:11])
    assert g[0] == hist[0]
    assert g.sum() == hist.sum() > 0
    gpu_mean = sum(k * v for k, v in enumerate(g)) / hist.sum()
    orc_mean = sum(k * v for k, v in enumerate(hist)) / hist.sum()
    assert abs(gpu_mean - orc_mean) <= 0.01 * orc_mean


@pytest.mark.parametrize("bc", [1, 2])
def test_near_vacuum_floors(torch_cuda, orc, bc):
    """Cells receding from each other at several sound speeds with p down to
    1e-9: star pressures fall to the floor, densities to near the floor;
    every floor of the reading applies and must match the oracle's."""
    from paper_2106_13465_amd.hydro import Hydro

    rng = np.random.Generator(np.random.PCG64(55))
    nx, ny = 96, 40
    rho = np.exp(rng.uniform(np.log(1e-6), 0.0, (ny, nx)))
    p = np.exp(rng.uniform(np.log(1e-9), 0.0, (ny, nx)))
    u = np.where(np.arange(nx)[None, :] % 2 == 0, -4.0, 4.0) * np.ones((ny, 1))
    v = np.where(np.arange(ny)[:, None] % 3 == 0, -4.0, 4.0) * np.ones((1, nx))
    U = inputs.conservative(rho, u, v, p)
    h = Hydro(nx, ny, 1.4, 0.8, bc)
    h.set_state(U)
    h.set_options(stats=1)
    h.step(3)
    ref = U.copy()
    c = orc.cfg(bc=bc)
    hist = np.zeros(11, dtype=np.int64)
    for _ in range(3):
        orc.step(ref, c, hist)
    got = h.get_state()
    assert np.all(np.isfinite(got)) and np.all(got[0] > 0)
    assert rel_err(got, ref) <= TOL64
    # interfaces whose root lies under the floor stop on it instead of
    # running to the cap: the iteration counts follow the oracle's, and only
    # a few hundredths of the interfaces stay unconverged
    g = np.array(h.stats()["hist"][:11])
    assert g.sum() == hist.sum() and np.abs(g - hist).sum() <= 0.01 * hist.sum()
    assert hist[0] < 0.01 * hist.sum()


def test_error_paths(torch_cuda):
    """Invalid arguments come back as error codes with a message."""
    from paper_2106_13465_amd import _lib
    from paper_2106_13465_amd.hydro import Hydro, HydroError

    lib = _lib.load()
    assert not lib.hydro_create(1, 5, 1.4, 0.8, 3)
    assert "must be >= 2" in _lib.last_error()
    assert not lib.hydro_create(8, 8, 1.0, 0.8, 3)
    assert not lib.hydro_create(8, 8, 1.4, 1.5, 3)
    assert not lib.hydro_create(8, 8, 1.4, 0.8, 7)
    h = lib.hydro_create(8, 8, 1.4, 0.8, 3)
    assert h
    assert lib.hydro_step(h) == _lib.HYDRO_ESTATE
    assert lib.hydro_sweep(h, 0) == _lib.HYDRO_ESTATE
    assert lib.hydro_compute_dt(h) == _lib.HYDRO_ESTATE
    lib.hydro_destroy(h)
    g = Hydro(16, 16, 1.4, 0.8, "periodic")
    with pytest.raises(HydroError):
        g.sweep(5)
    with pytest.raises(HydroError):
        g.set_options(niter=0)
    with pytest.raises(HydroError):
        g.set_options(tol=-1.0)
    with pytest.raises(HydroError):
        g.set_options(learned_gate=float("nan"))
    with pytest.raises(HydroError):
        g.set_options(learned_gate=51.0)
    assert g.options()["learned_gate"] == _lib.HYDRO_LEARNED_GATE_DEFAULT
    with pytest.raises(HydroError):
        g.graph_steps(0)
    # a non-finite state is latched and reported at the next synchronising call
    U = inputs.uniform(16, 16)
    U[3, 5, 5] = np.nan
    g.set_state(U)
    g.step(1)
    with pytest.raises(HydroError) as ei:
        g.totals()
    assert ei.value.code == _lib.HYDRO_ENONPHYS
    g.set_state(inputs.uniform(16, 16))
    g.step(1)
    assert np.all(np.isfinite(g.totals()))


def test_checkpoint_restart_bitwise(torch_cuda, orc):
    """2N steps equal N steps, a save of (state, clock), a fresh handle and N
    more steps, bitwise."""
    U = inputs.random_smooth(96, 80, seed=45, amp=0.5)
    a = make(torch_cuda, U, 1)
    a.step(8)
    full = a.get_state()
    b = make(torch_cuda, U, 1)
    b.step(4)
    saved, (t, n, _) = b.get_state(), b.clock()
    c = make(torch_cuda, saved, 1)
    c.set_clock(t, n)
    c.step(4)
    assert np.array_equal(c.get_state(), full)
    assert c.clock()[1] == 8 and abs(c.clock()[0] - a.clock()[0]) <= 1e-15 * a.clock()[0]


def transonic_fans(n_along, n_across, axis):
    """Rows (axis 0: the jump along x) or columns (axis 1: along y) each
    holding one Riemann problem whose left wave is a transonic rarefaction:
    strength eps = 1 - p*/p_L from 0.005 to 0.3 and the sonic point at a
    fraction theta of the fan from 0.1 to 0.9 (the right state is the star
    state, so there is no right wave).  Uniform states on either side of the
    jump, so the limited slopes vanish there and the interface at the jump
    sees exactly (L, R): every pencil exercises the fan sampling."""
    g = 1.4
    z = (g - 1) / (2 * g)
    cL = math.sqrt(g)
    U = np.empty((4, n_across, n_along) if axis == 0 else (4, n_along, n_across))
    for k, (eps, theta) in enumerate(zip(np.geomspace(0.005, 0.3, n_across),
                                         np.linspace(0.1, 0.9, n_across))):
        ps = 1.0 - eps
        cs = cL * ps**z
        w = (g + 1) / (g - 1) * (cL - cs)
        uL = cL - theta * w
        us = uL + 2.0 / (g - 1) * (cL - cs)
        left = inputs.conservative(1.0, uL, 0.1, 1.0)
        right = inputs.conservative(0.5, us, -0.2, ps)
        half = n_along // 2
        pencil = np.empty((4, n_along))
        pencil[:, :half] = np.asarray(left).reshape(4, 1)
        pencil[:, half:] = np.asarray(right).reshape(4, 1)
        if axis == 0:
            U[:, k, :] = pencil
        else:  # normal momentum is the y component
            U[:, :, k] = pencil[[0, 2, 1, 3]]
    return U


@pytest.mark.parametrize("direction", [0, 1])
def test_transonic_fans_fp64(torch_cuda, orc, direction):
    """Every pencil's middle interface is a transonic rarefaction (the
    sampling's fan branch, pinned on the oracle against the exact fan): one
    sweep in either direction matches the oracle to the FP64 bar, and a
    second-order step of each precision stays close to it."""
    U = transonic_fans(130, 64, direction)
    print(f"transonic fans dir={direction} shape={U.shape}", flush=True)
    h = make(torch_cuda, U, 2)
    c = orc.cfg(bc=2)
    dt = h.compute_dt()
    h.sweep(direction)
    ref = U.copy()
    orc.sweep(ref, direction, dt, c)
    assert rel_err(h.get_state(), ref) <= TOL64
    h32 = make(torch_cuda, U, 2, dtype=torch_cuda.float32)
    h32.compute_dt()
    h32.sweep(direction)
    got = h32.get_state().astype(np.float64)
    for k in range(4):
        assert np.abs(got[k] - ref[k]).sum() <= 1e-5 * np.abs(ref[k]).sum(), k
