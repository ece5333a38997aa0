"""Pins of the test tool exact_riemann.py (the independent exact Riemann
solver that several oracle pins compare with), against the gas-dynamics
identities its solution must satisfy: the Rankine-Hugoniot jump conditions
across each shock in the shock's frame, constant entropy and Riemann
invariant across each rarefaction, the characteristic condition u -+ c = x/t
inside a fan, and f(p*) = 0.  CPU only."""
import math

import numpy as np

import exact_riemann as ex

G = 1.4


def problems(seed, n):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < n:
        rL, rR, pL, pR = np.exp(rng.uniform(-2, 2, 4))
        uL, uR = rng.uniform(-3, 3, 2)
        try:
            ps, us = ex.star((rL, uL, pL), (rR, uR, pR), G)
        except ValueError:
            continue
        out.append(((rL, uL, pL), (rR, uR, pR), ps, us))
    return out


def energy(rho, u, p):
    return p / (G - 1) + 0.5 * rho * u * u


def test_root():
    for L, R, ps, _ in problems(1, 300):
        scale = abs(L[1]) + abs(R[1]) + math.sqrt(G * L[2] / L[0]) + math.sqrt(G * R[2] / R[0])
        assert abs(ex.wave_function(ps, L, R, G)) <= 1e-12 * scale


def test_shocks_satisfy_rankine_hugoniot():
    """Across a shock moving at S, the fluxes of mass, momentum and energy in
    the shock frame are continuous."""
    n = 0
    for L, R, ps, us in problems(2, 400):
        for side, K, s in ((0, L, -1.0), (1, R, 1.0)):
            rho, u, p = K
            if ps <= p:
                continue
            c = math.sqrt(G * p / rho)
            S = u + s * c * math.sqrt((G + 1) / (2 * G) * ps / p + (G - 1) / (2 * G))
            xi = S - s * 1e-9 * (abs(S) + 1)  # just inside the star region
            rs, ust, pst = ex.sample(L, R, xi, G, (ps, us))
            assert math.isclose(ust, us, rel_tol=1e-12, abs_tol=1e-12)
            m1, m2 = rho * (u - S), rs * (us - S)
            assert abs(m1 - m2) <= 1e-10 * (abs(m1) + rho * c)
            f1, f2 = m1 * u + p, m2 * us + ps
            assert abs(f1 - f2) <= 1e-10 * (abs(f1) + ps)
            e1 = (energy(rho, u, p) * (u - S) + p * u)
            e2 = (energy(rs, us, ps) * (us - S) + ps * us)
            assert abs(e1 - e2) <= 1e-10 * (abs(e1) + ps * (abs(us) + c))
            n += 1
    assert n > 100


def test_rarefactions_are_isentropic_with_constant_invariant():
    """Across a rarefaction p / rho^gamma and u -+ 2c/(gamma-1) are constant,
    and inside the fan the state satisfies u -+ c = x/t."""
    n = 0
    for L, R, ps, us in problems(3, 400):
        for K, s in ((L, -1.0), (R, 1.0)):
            rho, u, p = K
            if ps > p:
                continue
            c = math.sqrt(G * p / rho)
            head = u + s * c
            cs = c * (ps / p) ** ((G - 1) / (2 * G))
            tail = us + s * cs
            for f in (0.1, 0.5, 0.9, 1.0 + 1e-9):
                xi = head + f * (tail - head)
                if f > 1.0:
                    xi = tail - s * 1e-9 * (abs(tail) + 1)
                r2, u2, p2 = ex.sample(L, R, xi, G, (ps, us))
                c2 = math.sqrt(G * p2 / r2)
                assert math.isclose(p2 / r2 ** G, p / rho ** G, rel_tol=1e-11)
                inv, inv2 = u - s * 2 * c / (G - 1), u2 - s * 2 * c2 / (G - 1)
                assert abs(inv - inv2) <= 1e-11 * (abs(inv) + c)
                if f < 1.0:
                    assert abs(u2 + s * c2 - xi) <= 1e-11 * (abs(xi) + c)
            n += 1
    assert n > 100


def test_contact_carries_u_and_p():
    for L, R, ps, us in problems(4, 200):
        a = ex.sample(L, R, us - 1e-9, G, (ps, us))
        b = ex.sample(L, R, us + 1e-9, G, (ps, us))
        if a[2] == ps and b[2] == ps:
            assert a[1] == b[1] == us
