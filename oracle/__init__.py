"""Plain FP64 CPU oracle of the split second-order Godunov sweep.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library: the C source here (``hydro_oracle.c``, ``mlp_oracle.c``) is
compiled by ``oracle/build.py`` with gcc into ``liboracle.so`` and reached through
ctypes on host numpy arrays.

The method follows the paper's statement (Section 1; Figures 1, 2 and 5): a
directionally split, second-order Godunov scheme for the 2D compressible Euler
equations on a fixed rectangular grid, with a Riemann problem at every interface.
The readings taken where the paper is silent are listed in ``hydro_oracle.h``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC_REFLECT, BC_OUTFLOW, BC_PERIODIC = 1, 2, 3
LIMITER_MINMOD, LIMITER_MC, LIMITER_VANLEER = 0, 1, 2
ORDER_XY, ORDER_ALTERNATE = 0, 1
RIEMANN_TWO_SHOCK, RIEMANN_EXACT, RIEMANN_HLLC = 0, 1, 2
SCHEME_FINE, SCHEME_COARSE, SCHEME_TASKS = 0, 1, 2
DIR_X, DIR_Y = 0, 1
RHO_MIN = 1e-10
C_MIN = 1e-10


class Cfg(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("bc", ctypes.c_int),
        ("niter", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("limiter", ctypes.c_int),
        ("order", ctypes.c_int),
        ("riemann", ctypes.c_int),
        ("nscalars", ctypes.c_int),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_LL = ctypes.POINTER(ctypes.c_longlong)
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "oracle_cons_to_prim": (None, [_D, ctypes.c_double, _D]),
        "oracle_p_floor": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
        "oracle_sound_speed": (ctypes.c_double, [_D, ctypes.c_double]),
        "oracle_minmod": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
        "oracle_limit": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, ctypes.c_int]),
        "oracle_trace": (None, [_D, _D, ctypes.c_double, ctypes.c_double, _D, _D]),
        "oracle_ptr_guess": (ctypes.c_double, [_D, _D, ctypes.c_double]),
        "oracle_two_shock_f": (ctypes.c_double, [_D, _D, ctypes.c_double, ctypes.c_double]),
        "oracle_riemann": (
            ctypes.c_int,
            [_D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_double, _D, _D, _D,
             ctypes.POINTER(ctypes.c_int)],
        ),
        "oracle_exact_f": (ctypes.c_double, [_D, _D, ctypes.c_double, ctypes.c_double]),
        "oracle_riemann_exact": (
            ctypes.c_int,
            [_D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_double, _D, _D, _D,
             ctypes.POINTER(ctypes.c_int)]),
        "oracle_hllc_speeds": (None, [_D, _D, ctypes.c_double, _D]),
        "oracle_hllc_flux": (None, [_D, _D, ctypes.c_double, _D]),
        "oracle_hllc_left": (ctypes.c_int, [_D, _D, ctypes.c_double]),
        "oracle_load_pencil_n": (
            None, [_D, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                   ctypes.c_int, _D]),
        "oracle_totals_n": (None, [_D, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]),
        "oracle_flux": (None, [_D, ctypes.c_double, _D]),
        "oracle_pencil": (None, [_D, ctypes.c_int, ctypes.c_double, ctypes.POINTER(Cfg), _LL]),
        "oracle_load_pencil": (
            None,
            [_D, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D],
        ),
        "oracle_sweep": (
            None,
            [_D, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
             ctypes.POINTER(Cfg), _LL],
        ),
        "oracle_max_speed": (ctypes.c_double, [_D, ctypes.c_int, ctypes.c_int, ctypes.c_double]),
        "oracle_compute_dt": (
            ctypes.c_double, [_D, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Cfg)]),
        "oracle_step": (
            ctypes.c_double, [_D, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Cfg), _LL]),
        "oracle_step_n": (
            ctypes.c_double,
            [_D, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Cfg), ctypes.c_long, _LL]),
        "oracle_totals": (None, [_D, ctypes.c_int, ctypes.c_int, _D]),
        "oracle_threads": (ctypes.c_int, []),
        "oracle_set_threads": (None, [ctypes.c_int]),
        "oracle_step_scheme": (ctypes.c_double, [_D, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Cfg),
                                                 ctypes.c_int, ctypes.c_int]),
        "oracle_scheme_decomposition": (None, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_int)]),
        "mlp_oracle_nparams": (ctypes.c_int, []),
        "mlp_oracle_bf16": (ctypes.c_double, [ctypes.c_double]),
        "mlp_oracle_forward": (ctypes.c_double, [_D, _D, ctypes.c_int, _D]),
        "mlp_oracle_loss_grad": (None, [_D, _D, _D, ctypes.c_long, ctypes.c_int, _D, _D]),
        "mlp_oracle_features": (None, [_D, ctypes.c_double, _D, _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _vec(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(4))


def cfg(gamma=1.4, cfl=0.8, bc=BC_PERIODIC, niter=10, tol=1e-8, limiter=LIMITER_MINMOD,
        order=ORDER_XY, riemann=RIEMANN_TWO_SHOCK, nscalars=0) -> Cfg:
    return Cfg(float(gamma), float(cfl), int(bc), int(niter), float(tol), int(limiter),
               int(order), int(riemann), int(nscalars))


# ---------------------------------------------------------------- single steps
def cons_to_prim(u, gamma=1.4) -> np.ndarray:
    u = _vec(u)
    q = np.zeros(4)
    _load().oracle_cons_to_prim(_dptr(u), gamma, _dptr(q))
    return q


def p_floor(rho, gamma=1.4) -> float:
    return _load().oracle_p_floor(float(rho), float(gamma))


def sound_speed(q, gamma=1.4) -> float:
    q = _vec(q)
    return _load().oracle_sound_speed(_dptr(q), gamma)


def minmod(a, b) -> float:
    return _load().oracle_minmod(float(a), float(b))


def limit(a, b, limiter) -> float:
    return _load().oracle_limit(float(a), float(b), int(limiter))


def trace(q, dq, gamma, lam):
    q, dq = _vec(q), _vec(dq)
    qm, qp = np.zeros(4), np.zeros(4)
    _load().oracle_trace(_dptr(q), _dptr(dq), gamma, lam, _dptr(qm), _dptr(qp))
    return qm, qp


def ptr_guess(qL, qR, gamma=1.4) -> float:
    qL, qR = _vec(qL), _vec(qR)
    return _load().oracle_ptr_guess(_dptr(qL), _dptr(qR), gamma)


def two_shock_f(qL, qR, gamma, p) -> float:
    qL, qR = _vec(qL), _vec(qR)
    return _load().oracle_two_shock_f(_dptr(qL), _dptr(qR), gamma, float(p))


def riemann(qL, qR, gamma=1.4, niter=10, tol=1e-8):
    """Returns (godunov_state[4], pstar, ustar, iterations, converged)."""
    qL, qR = _vec(qL), _vec(qR)
    qg = np.zeros(4)
    ps, us = ctypes.c_double(), ctypes.c_double()
    conv = ctypes.c_int()
    it = _load().oracle_riemann(_dptr(qL), _dptr(qR), gamma, niter, tol, _dptr(qg),
                                ctypes.byref(ps), ctypes.byref(us), ctypes.byref(conv))
    return qg, ps.value, us.value, it, bool(conv.value)


def exact_f(qL, qR, gamma, p) -> float:
    qL, qR = _vec(qL), _vec(qR)
    return _load().oracle_exact_f(_dptr(qL), _dptr(qR), gamma, float(p))


def riemann_exact(qL, qR, gamma=1.4, niter=10, tol=1e-8):
    """Exact solver; returns (godunov_state[4], pstar, ustar, iterations, converged)."""
    qL, qR = _vec(qL), _vec(qR)
    qg = np.zeros(4)
    ps, us = ctypes.c_double(), ctypes.c_double()
    conv = ctypes.c_int()
    it = _load().oracle_riemann_exact(_dptr(qL), _dptr(qR), gamma, niter, tol, _dptr(qg),
                                      ctypes.byref(ps), ctypes.byref(us), ctypes.byref(conv))
    return qg, ps.value, us.value, it, bool(conv.value)


def hllc_speeds(qL, qR, gamma=1.4) -> np.ndarray:
    """(S_L, S*, S_R) of the HLLC flux."""
    qL, qR = _vec(qL), _vec(qR)
    S = np.zeros(3)
    _load().oracle_hllc_speeds(_dptr(qL), _dptr(qR), gamma, S.ctypes.data_as(_D))
    return S


def hllc_left(qL, qR, gamma=1.4) -> bool:
    qL, qR = _vec(qL), _vec(qR)
    return bool(_load().oracle_hllc_left(_dptr(qL), _dptr(qR), gamma))


def hllc_flux(qL, qR, gamma=1.4) -> np.ndarray:
    qL, qR = _vec(qL), _vec(qR)
    F = np.zeros(4)
    _load().oracle_hllc_flux(_dptr(qL), _dptr(qR), gamma, _dptr(F))
    return F


def flux(qg, gamma=1.4) -> np.ndarray:
    qg = _vec(qg)
    F = np.zeros(4)
    _load().oracle_flux(_dptr(qg), gamma, _dptr(F))
    return F


# ---------------------------------------------------------------- pencils, grids
def pencil(w: np.ndarray, lam: float, c: Cfg, hist: np.ndarray | None = None) -> np.ndarray:
    """1D update of a pencil held with its ghosts, w of shape [4 + c.nscalars,
    n+4]; returns the updated copy."""
    w = np.ascontiguousarray(w, dtype=np.float64).copy()
    if w.shape[0] != 4 + c.nscalars:
        raise ValueError("pencil rows must be 4 + nscalars")
    n = w.shape[1] - 4
    hp = hist.ctypes.data_as(_LL) if hist is not None else None
    _load().oracle_pencil(_dptr(w), n, lam, ctypes.byref(c), hp)
    return w


def load_pencil(U: np.ndarray, direction: int, line: int, bc: int) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    nv, ny, nx = U.shape
    n = nx if direction == DIR_X else ny
    w = np.zeros((nv, n + 4))
    _load().oracle_load_pencil_n(_dptr(U), nx, ny, nv, direction, line, bc, _dptr(w))
    return w


def _grid(U: np.ndarray, c: Cfg | None = None) -> np.ndarray:
    nv = 4 + (c.nscalars if c is not None else 0)
    ok = U.dtype == np.float64 and U.flags.c_contiguous and U.ndim == 3
    if not ok or (U.shape[0] != nv if c is not None else U.shape[0] < 4):
        raise ValueError("oracle grids are contiguous float64 arrays [4 + nscalars, ny, nx]")
    return U


def sweep(U: np.ndarray, direction: int, dt: float, c: Cfg,
          hist: np.ndarray | None = None) -> None:
    """In-place directional sweep of U [4 + c.nscalars, ny, nx]."""
    _grid(U, c)
    _, ny, nx = U.shape
    hp = hist.ctypes.data_as(_LL) if hist is not None else None
    _load().oracle_sweep(_dptr(U), nx, ny, direction, dt, ctypes.byref(c), hp)


def max_speed(U: np.ndarray, gamma=1.4) -> float:
    _grid(U)
    _, ny, nx = U.shape
    return _load().oracle_max_speed(_dptr(U), nx, ny, gamma)


def compute_dt(U: np.ndarray, c: Cfg) -> float:
    _grid(U)
    _, ny, nx = U.shape
    return _load().oracle_compute_dt(_dptr(U), nx, ny, ctypes.byref(c))


def step(U: np.ndarray, c: Cfg, hist: np.ndarray | None = None, step_index: int = 0) -> float:
    """In-place time step (dt, then the two sweeps in the order c.order gives
    for step number step_index); returns dt."""
    _grid(U, c)
    _, ny, nx = U.shape
    hp = hist.ctypes.data_as(_LL) if hist is not None else None
    return _load().oracle_step_n(_dptr(U), nx, ny, ctypes.byref(c), int(step_index), hp)


def totals(U: np.ndarray) -> np.ndarray:
    """Totals of every plane of U (4 conserved variables, then the scalars)."""
    _grid(U)
    nv, ny, nx = U.shape
    out = np.zeros(nv)
    _load().oracle_totals_n(_dptr(U), nx, ny, nv, _dptr(out))
    return out


def threads() -> int:
    return _load().oracle_threads()


def step_scheme(U: np.ndarray, c: Cfg, scheme: int, threads: int) -> float:
    """One time step parallelised by one of the paper's OpenMP schemes
    (SCHEME_FINE, SCHEME_COARSE, SCHEME_TASKS) on `threads` threads; the
    result equals step(U, c) bitwise.  Returns dt."""
    _grid(U, c)
    _, ny, nx = U.shape
    return _load().oracle_step_scheme(_dptr(U), nx, ny, ctypes.byref(c), int(scheme), int(threads))


def scheme_decomposition(threads: int, nx: int, ny: int):
    px, py = ctypes.c_int(), ctypes.c_int()
    _load().oracle_scheme_decomposition(int(threads), int(nx), int(ny), ctypes.byref(px),
                                        ctypes.byref(py))
    return px.value, py.value


def set_threads(n: int) -> None:
    """OpenMP threads of the sweeps (results do not depend on it)."""
    _load().oracle_set_threads(int(n))


# ---------------------------------------------------------------- learned-guess network
MLP_PARAMS = 1313


def mlp_bf16(v: float) -> float:
    return _load().mlp_oracle_bf16(float(v))


def mlp_forward(params, X, emulate=True) -> np.ndarray:
    """Network outputs for X [n, 6] (FP64; emulate = BF16 rounding points)."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 6)
    lib = _load()
    return np.array([lib.mlp_oracle_forward(_dptr(P), _dptr(np.ascontiguousarray(x)),
                                            int(emulate), None) for x in X])


def mlp_loss_grad(params, X, T, emulate=True):
    """(grad [1313], loss) of the mean squared error."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 6)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
    g = np.zeros(MLP_PARAMS)
    loss = ctypes.c_double()
    _load().mlp_oracle_loss_grad(_dptr(P), _dptr(X), _dptr(T), len(T), int(emulate), _dptr(g),
                                 ctypes.byref(loss))
    return g, loss.value


def mlp_features(record, gamma=1.4):
    """(x [6], target) of one interface record (rho_L, u_L, p_L, rho_R, u_R, p_R, p*, .)."""
    rec = np.ascontiguousarray(np.asarray(record, dtype=np.float64).reshape(-1)[:8])
    if rec.size < 8:
        rec = np.concatenate([rec, np.zeros(8 - rec.size)])
    x = np.zeros(6)
    t = ctypes.c_double()
    _load().mlp_oracle_features(_dptr(rec), gamma, _dptr(x), ctypes.byref(t))
    return x, t.value
