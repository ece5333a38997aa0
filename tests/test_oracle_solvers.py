"""Pins of the oracle's other interface solvers: the exact Riemann solver and
the HLLC flux.  Checked against the independent bracketing solver and exact
sampler in ``exact_riemann.py``, against the two-shock solver where both are
exact, and against properties of the HLLC construction.  CPU only."""
import math

import numpy as np
import pytest

import exact_riemann as ex
from paper_2106_13465_amd import inputs
from test_oracle_sweep import run_until

G = 1.4


def prim(rho, u, ut, p):
    return np.array([rho, u, ut, p], dtype=np.float64)


def random_problem(rng, pdec=3.0):
    """Random left/right primitive states (with transverse velocities) that do
    not generate vacuum, nor a star pressure near the floor, and their exact
    (p*, u*)."""
    while True:
        rL, rR = np.exp(rng.uniform(-2, 2, 2))
        pL, pR = np.exp(rng.uniform(-pdec, pdec, 2))
        uL, uR = rng.uniform(-3, 3, 2)
        try:
            ps, us = ex.star((rL, uL, pL), (rR, uR, pR), G)
        except ValueError:
            continue
        if ps < 1e-9 * min(pL, pR):
            continue
        return prim(rL, uL, rng.uniform(-1, 1), pL), prim(rR, uR, rng.uniform(-1, 1), pR), ps, us


def pattern(L, R, ps):
    return ("s" if ps > L[3] else "r") + ("s" if ps > R[3] else "r")


# ------------------------------------------------------------------ exact solver
def test_exact_wave_function_matches(orc):
    rng = np.random.Generator(np.random.PCG64(21))
    for _ in range(300):
        L, R, ps, _ = random_problem(rng)
        for p in ps * np.exp(rng.uniform(-3, 3, 4)):
            a = orc.exact_f(L, R, G, p)
            b = ex.wave_function(p, (L[0], L[1], L[3]), (R[0], R[1], R[3]), G)
            scale = abs(L[1]) + abs(R[1]) + math.sqrt(G * L[3] / L[0]) + math.sqrt(G * R[3] / R[0])
            assert abs(a - b) <= 1e-13 * (scale + abs(b) + p), (L, R, p, a, b)


def test_exact_star_matches_bracketing(orc):
    """p* and u* equal the bracketing root for every wave pattern (a raised
    cap: from a poor guess above a strong shock's p*, Newton's first step
    lands far below it, and the climb back can take more than 10 steps)."""
    rng = np.random.Generator(np.random.PCG64(22))
    seen = set()
    for _ in range(600):
        L, R, ps, us = random_problem(rng, pdec=5.0)
        seen.add(pattern(L, R, ps))
        _, p, u, it, conv = orc.riemann_exact(L, R, G, niter=60)
        assert conv
        assert math.isclose(p, ps, rel_tol=1e-12), (L, R, p, ps)
        cs = math.sqrt(G * L[3] / L[0]) + math.sqrt(G * R[3] / R[0])
        assert abs(u - us) <= 1e-12 * (cs + abs(us)), (L, R, u, us)
    assert seen == {"ss", "sr", "rs", "rr"}


def test_exact_godunov_state_matches_sampling(orc):
    """The state at x/t = 0 equals the exact sampler's, including transonic
    rarefactions (where the two-shock solver's linear fan is only a reading)."""
    rng = np.random.Generator(np.random.PCG64(23))
    transonic = 0
    for _ in range(800):
        L, R, ps, us = random_problem(rng)
        qg, _, _, _, _ = orc.riemann_exact(L, R, G, niter=60)
        rho, u, p = ex.sample((L[0], L[1], L[3]), (R[0], R[1], R[3]), 0.0, G, (ps, us))
        side = L if us >= 0 else R
        cK = math.sqrt(G * side[3] / side[0])
        head = side[1] - cK if us >= 0 else side[1] + cK
        in_fan = ps <= side[3] and head * (1 if us >= 0 else -1) < 0 and not (
            (rho, u, p) == (side[0], side[1], side[3]))
        if in_fan and abs(p - ps) > 1e-9 * ps:
            transonic += 1
        assert math.isclose(qg[0], rho, rel_tol=1e-11), (L, R, qg, rho)
        assert abs(qg[1] - u) <= 1e-11 * (abs(u) + cK)
        assert math.isclose(qg[3], p, rel_tol=1e-11), (L, R, qg, p)
        assert qg[2] == side[2]
    assert transonic >= 20


def test_exact_two_rarefactions_converge_at_once(orc):
    """For two rarefactions the starting guess is the exact p*: one Newton
    step meets the test."""
    rng = np.random.Generator(np.random.PCG64(24))
    n = 0
    while n < 200:
        L, R, ps, _ = random_problem(rng)
        if pattern(L, R, ps) != "rr":
            continue
        n += 1
        _, p, _, it, conv = orc.riemann_exact(L, R, G)
        assert conv and it == 1 and math.isclose(p, ps, rel_tol=1e-12)


def test_exact_equals_two_shock_for_two_shocks(orc):
    """When both waves are shocks the two-shock solver is exact too: the same
    p*, u* and Godunov state."""
    rng = np.random.Generator(np.random.PCG64(25))
    n = 0
    while n < 200:
        L, R, ps, _ = random_problem(rng)
        if pattern(L, R, ps) != "ss":
            continue
        n += 1
        ga, pa, ua, _, _ = orc.riemann_exact(L, R, G, niter=60)
        gb, pb, ub, _, _ = orc.riemann(L, R, G, niter=60)
        assert math.isclose(pa, pb, rel_tol=1e-12)
        np.testing.assert_allclose(ga, gb, rtol=1e-11, atol=1e-12 * (abs(ua) + 1))


def test_exact_newton_converges_quadratically(orc):
    """On moderate jumps every interface meets the test within the default
    cap in a few steps (a wrong derivative would leave Newton linear)."""
    rng = np.random.Generator(np.random.PCG64(26))
    its = []
    for _ in range(400):
        L, R, ps, _ = random_problem(rng, pdec=1.0)
        _, p, _, it, conv = orc.riemann_exact(L, R, G)
        assert conv
        its.append(it)
    assert np.mean(its) < 3.0 and max(its) <= 8, (np.mean(its), max(its))


def test_exact_wall_and_identical_states(orc):
    q = prim(0.7, 0.3, -0.2, 2.0)
    qg, p, u, _, _ = orc.riemann_exact(q, q, G)
    np.testing.assert_allclose(qg, q, rtol=1e-14)
    m = prim(0.7, -0.3, -0.2, 2.0)
    _, p, u, _, _ = orc.riemann_exact(q, m, G)  # mirrored: a wall
    assert abs(u) <= 1e-15 and p > q[3]


# ------------------------------------------------------------------ HLLC
def test_hllc_speeds_hand_evaluated(orc):
    """(rho, u, p) = (1, 0, 1) | (4, 0.3, 0.01): sqrt-density weights 1 and 2
    give u~ = 0.6/3 = 0.2, H_R = (3.5 * 0.01 + 0.5 * 4 * 0.09)/4 = 0.05375,
    H~ = (3.5 + 2 * 0.05375)/3 = 1.2025, c~ = sqrt(0.4 * (1.2025 - 0.02)) =
    0.687750, so S_R = u~ + c~ = 0.887750 (above u_R + c_R = 0.359161) and
    S_L = u_L - c_L = -1.183216; S* = (0.01 - 1 - 0.3 * 4 * (0.88775 - 0.3)) /
    (-1.183216 - 4 * (0.88775 - 0.3)) = 0.479683."""
    S = orc.hllc_speeds(prim(1.0, 0.0, 0.0, 1.0), prim(4.0, 0.3, 0.0, 0.01), G)
    np.testing.assert_allclose(S, [-1.183216, 0.479683, 0.887750], rtol=2e-6)


@pytest.mark.parametrize("riemann", [0, 1, 2])
def test_pencil_uses_the_chosen_solver(orc, riemann):
    """Piecewise-constant data has zero limited slopes, so the first update
    next to a single jump is U_L - lam (F* - F(U_L)) with F* the chosen
    solver's interface flux."""
    L, R = prim(1.0, 0.2, 0.1, 1.0), prim(0.25, -0.4, -0.3, 0.2)
    n = 8
    w = np.zeros((4, n + 4))
    for j in range(n + 4):
        q = L if j < 6 else R
        w[:, j] = [q[0], q[0] * q[1], q[0] * q[2], q[3] / (G - 1) + 0.5 * q[0] * (q[1] ** 2 + q[2] ** 2)]
    lam = 0.1
    out = orc.pencil(w, lam, orc.cfg(riemann=riemann))
    if riemann == 2:
        Fs = orc.hllc_flux(L, R, G)
    else:
        solve = orc.riemann_exact if riemann == 1 else orc.riemann
        Fs = orc.flux(solve(L, R, G)[0], G)
    np.testing.assert_allclose(out[:, 5], w[:, 5] - lam * (Fs - orc.flux(L, G)), rtol=1e-14,
                               atol=1e-15)
    np.testing.assert_allclose(out[:, 6], w[:, 6] - lam * (orc.flux(R, G) - Fs), rtol=1e-14,
                               atol=1e-15)


def test_hllc_consistency(orc):
    rng = np.random.Generator(np.random.PCG64(31))
    for _ in range(300):
        q = prim(math.exp(rng.uniform(-3, 3)), rng.uniform(-5, 5), rng.uniform(-2, 2),
                 math.exp(rng.uniform(-4, 4)))
        np.testing.assert_allclose(orc.hllc_flux(q, q, G), orc.flux(q, G), rtol=1e-13,
                                   atol=1e-15 * np.abs(orc.flux(q, G)).max())


@pytest.mark.parametrize("u", [0.7, -0.7, 0.0])
def test_hllc_resolves_contact_and_shear_exactly(orc, u):
    """An isolated contact with a shear jump (equal u and p, different rho and
    v) gets the exact flux: the upwind state's, and at u = 0 no mass, energy
    or transverse momentum crosses."""
    L, R = prim(1.3, u, 0.4, 0.8), prim(0.2, u, -0.9, 0.8)
    F = orc.hllc_flux(L, R, G)
    S = orc.hllc_speeds(L, R, G)
    assert abs(S[1] - u) <= 1e-14
    up = L if u >= 0 else R
    np.testing.assert_allclose(F, orc.flux(up, G), rtol=1e-13, atol=1e-14)
    if u == 0.0:
        assert F[0] == pytest.approx(0.0, abs=1e-15) and F[1] == pytest.approx(0.8, rel=1e-14)


def test_hllc_supersonic_upwinding(orc):
    rng = np.random.Generator(np.random.PCG64(32))
    for _ in range(100):
        rL, rR, pL, pR = np.exp(rng.uniform(-1, 1, 4))
        cL, cR = math.sqrt(G * pL / rL), math.sqrt(G * pR / rR)
        m = 3.0 * max(cL, cR)
        L, R = prim(rL, m + rng.uniform(0, 1), 0.3, pL), prim(rR, m + rng.uniform(0, 1), -0.1, pR)
        np.testing.assert_array_equal(orc.hllc_flux(L, R, G), orc.flux(L, G))
        Lm, Rm = L * [1, -1, 1, 1], R * [1, -1, 1, 1]
        np.testing.assert_array_equal(orc.hllc_flux(Rm, Lm, G), orc.flux(Lm, G))


def test_hllc_mirror_symmetry(orc):
    """Swapping the sides and reversing the normal velocity reverses the
    mass, transverse-momentum and energy fluxes and keeps the normal one."""
    rng = np.random.Generator(np.random.PCG64(33))
    for _ in range(300):
        L, R, _, _ = random_problem(rng)
        F = orc.hllc_flux(L, R, G)
        Fm = orc.hllc_flux(R * [1, -1, 1, 1], L * [1, -1, 1, 1], G)
        scale = np.abs(F).max() + 1e-300
        np.testing.assert_allclose(Fm, F * [-1, 1, -1, -1], rtol=0, atol=1e-13 * scale)


def test_hllc_is_godunov_to_second_order_in_weak_jumps(orc):
    """For jumps of size eps about a state, the HLLC flux and contact speed
    differ from the exact Godunov flux and u* by O(eps^2): halving eps
    divides the differences by 4."""
    rng = np.random.Generator(np.random.PCG64(34))
    for _ in range(20):
        base = prim(math.exp(rng.uniform(-1, 1)), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5),
                    math.exp(rng.uniform(-1, 1)))
        d = rng.normal(size=4) * [base[0], 1, 1, base[3]] * 0.5
        errs = []
        for eps in (1e-2, 5e-3, 2.5e-3):
            L, R = base + eps * d, base - eps * d
            ps, us = ex.star((L[0], L[1], L[3]), (R[0], R[1], R[3]), G)
            rho, u, p = ex.sample((L[0], L[1], L[3]), (R[0], R[1], R[3]), 0.0, G, (ps, us))
            Fg = orc.flux(prim(rho, u, L[2] if us >= 0 else R[2], p), G)
            errs.append((np.abs(orc.hllc_flux(L, R, G) - Fg).max(),
                         abs(orc.hllc_speeds(L, R, G)[1] - us)))
        for a, b in zip(errs, errs[1:]):
            assert 3.6 < a[0] / b[0] < 4.4 and 3.6 < a[1] / b[1] < 4.4, errs


# ------------------------------------------------------------------ whole scheme
@pytest.mark.parametrize("riemann", [1, 2])
def test_sod_converges_with_other_solvers(orc, riemann):
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    errs = []
    for n in (100, 200, 400):
        U = inputs.shock_tube(n, 2, (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1))
        c = orc.cfg(bc=orc.BC_OUTFLOW, riemann=riemann)
        t, _ = run_until(orc, U, c, 0.2)
        ref = ex.cell_averages(L, R, np.arange(n + 1) / n, t)
        errs.append(np.abs(U[0, 0, :] - ref[0]).sum() / n)
    assert errs[-1] < 4e-3
    assert math.log2(errs[0] / errs[-1]) / 2 > 0.6, errs


def test_transonic_rarefaction_with_exact_solver(orc):
    """A left-moving rarefaction crossing x/t = 0 (Sod-type data with u_L
    chosen so the fan is transonic): the exact solver's scheme converges."""
    L, R = (1.0, 0.75, 1.0), (0.125, 0.0, 0.1)
    errs = []
    for n in (100, 200, 400):
        U = inputs.shock_tube(n, 2, (1.0, 0.75, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1), x0=0.3)
        c = orc.cfg(bc=orc.BC_OUTFLOW, riemann=1)
        t, _ = run_until(orc, U, c, 0.2)
        ref = ex.cell_averages(L, R, np.arange(n + 1) / n, t, x0=0.3)
        errs.append(np.abs(U[0, 0, :] - ref[0]).sum() / n)
    assert math.log2(errs[0] / errs[-1]) / 2 > 0.6, errs


@pytest.mark.parametrize("riemann", [1, 2])
def test_periodic_conservation_other_solvers(orc, riemann):
    U = inputs.random_states(24, 17, seed=9, rough=0.6)
    T0 = orc.totals(U)
    c = orc.cfg(bc=3, riemann=riemann)
    for _ in range(5):
        orc.step(U, c)
    np.testing.assert_allclose(orc.totals(U), T0, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("riemann", [1, 2])
def test_uniform_flow_unchanged_other_solvers(orc, riemann):
    U = inputs.conservative(np.full((6, 9), 0.8), np.full((6, 9), 0.3), np.full((6, 9), -0.2),
                            np.full((6, 9), 1.7))
    V = U.copy()
    orc.step(V, orc.cfg(bc=3, riemann=riemann))
    np.testing.assert_allclose(V, U, rtol=1e-14, atol=1e-15)
