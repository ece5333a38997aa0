"""Seeded synthetic initial states for the 2D Euler sweep.

This module is shared by the oracle tests, the GPU tests and the benchmark.  It
holds no step of the method: it only builds initial conditions, each given by
primitive fields (rho, u, v, p) and stored in conservative form U = (rho, rho u,
rho v, E) with the ideal-gas total energy E = p/(gamma-1) + rho (u^2+v^2)/2, as
float64 arrays of shape [4, ny, nx] (x fastest).  Cells are square with
h = 1/max(nx, ny); cell centres sit at ((i+1/2) h, (j+1/2) h).

The paper's own test case is a point-explosion problem (Section 7); the
workloads here are synthetic stand-ins of that type and of other standard flows
(shear layers, random Riemann quadrants, strong jumps), generated from numpy's
PCG64 with a fixed seed per workload.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4
SEED_BASE = 2106


def conservative(rho, u, v, p, gamma: float = GAMMA) -> np.ndarray:
    """Stack primitive fields into a conservative [4, ny, nx] float64 array."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), shape)
    v = np.broadcast_to(np.asarray(v, dtype=np.float64), shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), shape)
    U = np.empty((4,) + shape, dtype=np.float64)
    U[0] = rho
    U[1] = rho * u
    U[2] = rho * v
    U[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return U


def cell_size(nx: int, ny: int) -> float:
    return 1.0 / max(nx, ny)


def uniform(nx: int, ny: int, rho=1.0, u=0.0, v=0.0, p=1.0, gamma=GAMMA) -> np.ndarray:
    return conservative(np.full((ny, nx), rho), u, v, p, gamma)


def shock_tube(nx: int, ny: int, left, right, x0: float = 0.5, axis: int = 0,
               gamma=GAMMA) -> np.ndarray:
    """Two constant states (rho, u_n, u_t, p) separated at x0 (fraction of the
    domain) along x (axis 0) or y (axis 1); normal velocity along that axis."""
    h = cell_size(nx, ny)
    n = nx if axis == 0 else ny
    xc = (np.arange(n) + 0.5) * h / (n * h)
    side = xc < x0
    prim = np.where(side[None, :], np.asarray(left, float)[:, None],
                    np.asarray(right, float)[:, None])  # [4, n]
    if axis == 0:
        rho = np.broadcast_to(prim[0][None, :], (ny, nx))
        un = np.broadcast_to(prim[1][None, :], (ny, nx))
        ut = np.broadcast_to(prim[2][None, :], (ny, nx))
        p = np.broadcast_to(prim[3][None, :], (ny, nx))
        return conservative(rho, un, ut, p, gamma)
    rho = np.broadcast_to(prim[0][:, None], (ny, nx))
    un = np.broadcast_to(prim[1][:, None], (ny, nx))
    ut = np.broadcast_to(prim[2][:, None], (ny, nx))
    p = np.broadcast_to(prim[3][:, None], (ny, nx))
    return conservative(rho, ut, un, p, gamma)


def random_smooth(nx: int, ny: int, seed: int, amp: float = 0.2, gamma=GAMMA) -> np.ndarray:
    """Cheap smooth random field (a few Fourier modes), for small tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = cell_size(nx, ny)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    fields = []
    for _ in range(4):
        f = np.zeros((ny, nx))
        for _ in range(3):
            kx, ky = rng.integers(-2, 3, size=2)
            f += rng.uniform(0, 1) * np.cos(2 * np.pi * (kx * X + ky * Y) + rng.uniform(0, 2 * np.pi))
        fields.append(f / max(np.abs(f).max(), 1e-12))
    rho = 1.0 + 0.5 * amp * fields[0]
    u = amp * fields[1]
    v = amp * fields[2]
    p = 1.0 + 0.5 * amp * fields[3]
    return conservative(rho, u, v, p, gamma)


def random_states(nx: int, ny: int, seed: int, gamma=GAMMA, rough: float = 1.0) -> np.ndarray:
    """Cell-wise independent random states (rho, p log-uniform over a decade,
    velocities of order the sound speed): every interface is a generic
    Riemann problem (shocks, rarefactions, contacts, sonic points)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = np.exp(rng.uniform(np.log(0.1), np.log(1.0), size=(ny, nx)) * rough)
    p = np.exp(rng.uniform(np.log(0.1), np.log(1.0), size=(ny, nx)) * rough)
    u = rng.uniform(-1.0, 1.0, size=(ny, nx)) * rough
    v = rng.uniform(-1.0, 1.0, size=(ny, nx)) * rough
    return conservative(rho, u, v, p, gamma)


def strong_jumps(nx: int, ny: int, seed: int, gamma=GAMMA, p_decades: float = 4.0,
                 rho_decades: float = 2.0, speed: float = 3.0) -> np.ndarray:
    """Cell-wise independent random states with strong jumps: rho log-uniform
    over rho_decades, p log-uniform over p_decades (both centred on 1),
    velocities uniform in [-speed, speed].  Most interfaces carry a strong
    shock or rarefaction, the regime where the two-rarefaction guess is
    poor."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ln10 = np.log(10.0)
    rho = np.exp(rng.uniform(-0.5, 0.5, size=(ny, nx)) * rho_decades * ln10)
    p = np.exp(rng.uniform(-0.5, 0.5, size=(ny, nx)) * p_decades * ln10)
    u = rng.uniform(-speed, speed, size=(ny, nx))
    v = rng.uniform(-speed, speed, size=(ny, nx))
    return conservative(rho, u, v, p, gamma)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
def blast_corner(n: int = 128, p0: float = 1e-5, gamma=GAMMA) -> np.ndarray:
    """Point explosion in the corner cell (the paper's test-case type, Section 7):
    rho = 1, u = v = 0, p = p0 everywhere; the total energy of cell (0, 0) is set
    to 1/h^2, i.e. a unit energy deposit.  Used with reflective walls."""
    U = uniform(n, n, 1.0, 0.0, 0.0, p0, gamma)
    h = cell_size(n, n)
    U[3, 0, 0] = 1.0 / (h * h)
    return U


def _fourier_modes(rng, nmodes: int, kmax: int):
    ks = []
    while len(ks) < nmodes:
        kx, ky = rng.integers(-kmax, kmax + 1, size=2)
        if max(abs(kx), abs(ky)) >= 1:
            ks.append((int(kx), int(ky)))
    return ks


def _fourier_field(nx, ny, ks, amps, phases) -> np.ndarray:
    """sum_m a_m cos(2 pi (kx x + ky y) + phi_m), as a sum of two rank-16 outer
    products (cos(A+B) = cos A cos B - sin A sin B)."""
    h = cell_size(nx, ny)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    kx = np.array([k[0] for k in ks], dtype=np.float64)
    ky = np.array([k[1] for k in ks], dtype=np.float64)
    A = 2 * np.pi * kx[:, None] * x[None, :] + phases[:, None]  # [m, nx]
    B = 2 * np.pi * ky[:, None] * y[None, :]                    # [m, ny]
    cA, sA = np.cos(A), np.sin(A)
    cB, sB = np.cos(B) * amps[:, None], np.sin(B) * amps[:, None]
    return cB.T @ cA - sB.T @ sA


def fourier_blasts(n: int = 8192, seed: int = SEED_BASE + 1, nblasts: int = 8,
                   nmodes: int = 16, kmax: int = 8, gamma=GAMMA) -> np.ndarray:
    """Smooth periodic flow plus point blasts.  rho = 1 + 0.3 S/max|S| with S a
    sum of 16 seeded Fourier modes (1 <= max(|kx|,|ky|) <= 8, amplitudes U[0,1],
    phases U[0,2pi)); u, v = 0.5 S_u/max|S_u|, 0.5 S_v/max|S_v| from the same
    wave vectors with independent phases and amplitudes; p = 1; then nblasts
    seeded cells get E = 1/h^2.  Periodic boundaries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = _fourier_modes(rng, nmodes, kmax)
    fields = []
    for _ in range(3):
        amps = rng.uniform(0.0, 1.0, size=nmodes)
        phases = rng.uniform(0.0, 2 * np.pi, size=nmodes)
        f = _fourier_field(n, n, ks, amps, phases)
        fields.append(f / np.abs(f).max())
    rho = 1.0 + 0.3 * fields[0]
    u = 0.5 * fields[1]
    v = 0.5 * fields[2]
    del fields
    U = conservative(rho, u, v, 1.0, gamma)
    del rho, u, v
    h = cell_size(n, n)
    cells = rng.integers(0, n, size=(nblasts, 2))
    for (j, i) in cells:
        U[3, j, i] = 1.0 / (h * h)
    return U


def shear_layer(n: int = 4096, seed: int = SEED_BASE + 2, gamma=GAMMA) -> np.ndarray:
    """Kelvin-Helmholtz shear layer on [0,1]^2: |y - 1/2| < 1/4 -> rho = 2,
    u = +0.5; elsewhere rho = 1, u = -0.5; p = 2.5; v = 0.01 U[-1,1] per cell.
    Periodic boundaries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = cell_size(n, n)
    y = (np.arange(n) + 0.5) * h
    inner = (np.abs(y - 0.5) < 0.25)[:, None]
    rho = np.where(inner, 2.0, 1.0) * np.ones((1, n))
    u = np.where(inner, 0.5, -0.5) * np.ones((1, n))
    v = 0.01 * rng.uniform(-1.0, 1.0, size=(n, n))
    return conservative(rho, u, v, 2.5, gamma)


def multiblast_batch(ngrids: int = 256, seed: int = SEED_BASE + 3, nmin: int = 64,
                     nmax: int = 1024, gamma=GAMMA):
    """Independent square grids, side log-uniform in [nmin, nmax]; background
    rho = 1, u = v = 0, p log-uniform in [1e-5, 1]; 1-8 blasts at seeded cells,
    each depositing an energy log-uniform in [1e-2, 1e2] (E += e/h^2).
    Reflective boundaries.  Returns a list of [4, n, n] arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grids = []
    for _ in range(ngrids):
        n = int(np.rint(nmin * (nmax / nmin) ** rng.uniform(0.0, 1.0)))
        p0 = float(np.exp(rng.uniform(np.log(1e-5), np.log(1.0))))
        U = uniform(n, n, 1.0, 0.0, 0.0, p0, gamma)
        h = cell_size(n, n)
        nb = int(rng.integers(1, 9))
        for _ in range(nb):
            j, i = rng.integers(0, n, size=2)
            e = float(np.exp(rng.uniform(np.log(1e-2), np.log(1e2))))
            U[3, j, i] += e / (h * h)
        grids.append(U)
    return grids


def quadrant_batch(ngrids: int = 64, seed: int = SEED_BASE + 4, nmin: int = 512,
                   nmax: int = 2048, strong_frac: float = 0.1, gamma=GAMMA):
    """2D Riemann problems: four constant states split at the grid centre, with
    rho, p log-uniform in [0.1, 2] per quadrant (p log-uniform in [2e-5, 2] in
    a seeded 10% of the grids, so pressure ratios reach 1e5) and u, v uniform in
    [-1, 1].  Outflow boundaries.  Returns a list of [4, n, n] arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grids = []
    for _ in range(ngrids):
        n = int(np.rint(nmin * (nmax / nmin) ** rng.uniform(0.0, 1.0)))
        strong = rng.uniform(0.0, 1.0) < strong_frac
        plo = 2e-5 if strong else 0.1
        rho_q = np.exp(rng.uniform(np.log(0.1), np.log(2.0), size=4))
        p_q = np.exp(rng.uniform(np.log(plo), np.log(2.0), size=4))
        u_q = rng.uniform(-1.0, 1.0, size=4)
        v_q = rng.uniform(-1.0, 1.0, size=4)
        half = n // 2
        quad = np.zeros((n, n), dtype=np.int64)
        quad[:half, half:] = 1
        quad[half:, :half] = 2
        quad[half:, half:] = 3
        grids.append(conservative(rho_q[quad], u_q[quad], v_q[quad], p_q[quad], gamma))
    return grids


def with_scalars(U: np.ndarray, X) -> np.ndarray:
    """Append passive-scalar planes rho * X_k to a conservative state
    [4, ny, nx]; X is one field [ny, nx] or a stack [k, ny, nx]."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 2:
        X = X[None]
    return np.ascontiguousarray(np.concatenate([U, U[0][None] * X], axis=0))


def random_scalars(nx: int, ny: int, seed: int, k: int = 1) -> np.ndarray:
    """k seeded scalar fields [k, ny, nx]: a smooth part plus cell noise, with
    values of both signs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = cell_size(nx, ny)
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    Xg, Yg = np.meshgrid(x, y)
    out = np.empty((k, ny, nx))
    for s in range(k):
        kx, ky = rng.integers(1, 4, size=2)
        out[s] = (np.sin(2 * np.pi * (kx * Xg + ky * Yg) + rng.uniform(0, 2 * np.pi))
                  + 0.3 * rng.uniform(-1, 1, size=(ny, nx)))
    return out
