"""Python face of libhydro.so: a handle bound to a torch device tensor.

PyTorch provides the device memory (the state tensor [4, ny, pitch]) and the
stream; every computation runs in the library's HIP kernels through the C ABI.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (HYDRO_BC_OUTFLOW, HYDRO_BC_PERIODIC, HYDRO_BC_REFLECT, HYDRO_DIR_X,
                   HYDRO_DIR_Y, HYDRO_F32, HYDRO_F64, HydroError, check)

__all__ = ["Hydro", "HydroBatch", "HydroError", "BC", "DIR_X", "DIR_Y", "step_noalloc"]

BC = {"reflect": HYDRO_BC_REFLECT, "outflow": HYDRO_BC_OUTFLOW, "periodic": HYDRO_BC_PERIODIC}
DIR_X, DIR_Y = HYDRO_DIR_X, HYDRO_DIR_Y
_DTYPE = {torch.float64: HYDRO_F64, torch.float32: HYDRO_F32}


def _bc_code(bc) -> int:
    return BC[bc] if isinstance(bc, str) else int(bc)


def _padded_pitch(nx: int, dtype: torch.dtype) -> int:
    # rows start on a 256-byte boundary
    per = 256 // torch.tensor([], dtype=dtype).element_size()
    return (nx + per - 1) // per * per


class Hydro:
    """One grid: ``Hydro(nx, ny, gamma, cfl, bc, dtype)``.

    The state lives in ``self.U`` (a torch tensor [4 + nscalars, ny, pitch] on
    the current HIP device; planes rho, rho u, rho v, E, then rho X for each
    passive scalar X); ``self.state`` is its [4 + nscalars, ny, nx] view.  Work runs on a stream of the handle's own (a new torch stream at the
    default priority unless one is given), so the step can be graph-captured.
    """

    def __init__(self, nx: int, ny: int, gamma: float = 1.4, cfl: float = 0.8,
                 bc="periodic", dtype: torch.dtype = torch.float64, device="cuda",
                 pitch: int | None = None, stream: torch.cuda.Stream | None = None,
                 nscalars: int = 0):
        self.lib = _lib.load()
        if dtype not in _DTYPE:
            raise ValueError(f"dtype {dtype}: float64 or float32")
        self.nx, self.ny, self.gamma, self.cfl = int(nx), int(ny), float(gamma), float(cfl)
        self.bc = _bc_code(bc)
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.handle = self.lib.hydro_create(self.nx, self.ny, self.gamma, self.cfl, self.bc)
            if not self.handle:
                raise HydroError(_lib.HYDRO_EINVAL, _lib.last_error())
            check(self.lib.hydro_set_scalars(self.handle, int(nscalars)))
            self.nv = 4 + int(nscalars)
            self.pitch = int(pitch) if pitch is not None else _padded_pitch(self.nx, dtype)
            self.U = torch.zeros((self.nv, self.ny, self.pitch), dtype=dtype, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self._bind()

    # ------------------------------------------------------------ plumbing
    def _bind(self):
        check(self.lib.hydro_bind(self.handle, ctypes.c_void_p(self.U.data_ptr()), self.pitch,
                                  _DTYPE[self.dtype], ctypes.c_void_p(self.stream.cuda_stream)))

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            self.lib.hydro_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def state(self) -> torch.Tensor:
        return self.U[:, :, : self.nx]

    @property
    def h(self) -> float:
        return 1.0 / max(self.nx, self.ny)

    def set_state(self, U) -> None:
        """Copy a [4 + nscalars, ny, nx] array (numpy or torch) into the bound
        state."""
        t = torch.as_tensor(np.asarray(U) if not isinstance(U, torch.Tensor) else U)
        if tuple(t.shape) != (self.nv, self.ny, self.nx):
            raise ValueError(f"state shape {tuple(t.shape)} != ({self.nv}, {self.ny}, {self.nx})")
        self.stream.synchronize()
        torch.cuda.synchronize(self.device)
        self.state.copy_(t.to(device=self.device, dtype=self.dtype))
        torch.cuda.synchronize(self.device)
        check(self.lib.hydro_invalidate(self.handle))

    def get_state(self) -> np.ndarray:
        self.stream.synchronize()
        return self.state.detach().to("cpu").numpy().copy()

    def graph_steps(self, nsteps: int) -> None:
        """nsteps time steps as one replay of a captured HIP graph."""
        check(self.lib.hydro_graph_steps(self.handle, int(nsteps)))

    # ------------------------------------------------------------ ABI calls
    def set_options(self, **kw) -> None:
        o = _lib.hydro_options_t()
        check(self.lib.hydro_get_options(self.handle, ctypes.byref(o)))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        check(self.lib.hydro_set_options(self.handle, ctypes.byref(o)))

    def options(self) -> dict:
        o = _lib.hydro_options_t()
        check(self.lib.hydro_get_options(self.handle, ctypes.byref(o)))
        return {k: getattr(o, k) for k, _ in o._fields_}

    def compute_dt(self) -> float:
        dt = self.lib.hydro_compute_dt(self.handle)
        if dt < 0:
            raise HydroError(int(dt), _lib.last_error())
        return dt

    def sweep(self, direction: int) -> None:
        check(self.lib.hydro_sweep(self.handle, int(direction)))

    def step(self, n: int = 1) -> None:
        for _ in range(n):
            check(self.lib.hydro_step(self.handle))

    def totals(self) -> np.ndarray:
        out = (ctypes.c_double * self.nv)()
        check(self.lib.hydro_conserved_totals(self.handle, out))
        return np.array(list(out))

    def clock(self):
        t, dt = ctypes.c_double(), ctypes.c_double()
        step = ctypes.c_long()
        check(self.lib.hydro_get_clock(self.handle, ctypes.byref(t), ctypes.byref(step),
                                       ctypes.byref(dt)))
        return t.value, step.value, dt.value

    def set_clock(self, t: float, step: int) -> None:
        check(self.lib.hydro_set_clock(self.handle, float(t), int(step)))

    def invalidate(self) -> None:
        check(self.lib.hydro_invalidate(self.handle))

    def set_profiling(self, enable: bool = True) -> None:
        check(self.lib.hydro_set_profiling(self.handle, int(enable)))

    def profile(self, reset: bool = True) -> dict:
        """Summed kernel time (ms) and launch count per step phase."""
        ms = (ctypes.c_double * _lib.HYDRO_NPHASES)()
        n = (ctypes.c_longlong * _lib.HYDRO_NPHASES)()
        check(self.lib.hydro_get_profile(self.handle, ms, n, int(reset)))
        return _profile_dict(ms, n)

    def stats(self, reset: bool = False) -> dict:
        s = _lib.hydro_stats_t()
        check(self.lib.hydro_riemann_stats(self.handle, ctypes.byref(s), int(reset)))
        return _stats_dict(s)

    def autotune(self, use_cache: bool = True) -> dict:
        """Pick the fastest launch shape of both sweeps on the bound state."""
        t = _lib.hydro_tune_t()
        check(self.lib.hydro_autotune(self.handle, ctypes.byref(t), int(use_cache)))
        return _tune_dict(t)

    def set_mlp(self, net) -> None:
        """Attach a packed network (``mlp.GuessNetwork``) or detach it (None)."""
        self._net = net
        if net is not None:
            self.stream.wait_stream(net.stream)  # the packed weights are ready
        ptr = ctypes.c_void_p(net.dev.data_ptr()) if net is not None else None
        check(self.lib.hydro_set_mlp(self.handle, ptr))

    def set_logger(self, records: torch.Tensor | None, seed: int = 0, rate_smooth: float = 0.01,
                   rate_strong: float = 1.0) -> None:
        """Log sampled interface states into records (float32 [capacity, 8])."""
        self._log = records
        ptr = ctypes.c_void_p(records.data_ptr()) if records is not None else None
        cap = records.shape[0] if records is not None else 0
        check(self.lib.hydro_set_logger(self.handle, ptr, cap, seed, rate_smooth, rate_strong))

    def logger_count(self) -> int:
        c = self.lib.hydro_logger_count(self.handle)
        if c < 0:
            raise HydroError(int(c), _lib.last_error())
        return c


def _stats_dict(s) -> dict:
    return {"interfaces": s.interfaces, "hist": list(s.hist), "fallbacks": s.fallbacks,
            "wave_hist": list(s.wave_hist)}


def _tune_dict(t) -> dict:
    return {k: getattr(t, k) for k, _ in t._fields_}


def _profile_dict(ms, n) -> dict:
    return {name: {"ms": ms[k], "launches": n[k]} for k, name in enumerate(_lib.PHASE_NAMES)}


class HydroBatch:
    """Independent grids of uneven sizes advanced together: one kernel launch
    per sweep over all of them, each grid with its own dt and clock.

    ``shapes`` is a list of (nx, ny); ``bc`` one boundary type or one per grid.
    The packed state lives in ``self.buf`` (1D torch tensor, layout of
    hydro_batch_layout); ``self.view(g)`` is grid g's [4 + nscalars, ny, nx]
    view.
    """

    def __init__(self, shapes, gamma: float = 1.4, cfl: float = 0.8, bc="reflect",
                 dtype: torch.dtype = torch.float32, device="cuda",
                 stream: torch.cuda.Stream | None = None, nscalars: int = 0):
        self.lib = _lib.load()
        if dtype not in _DTYPE:
            raise ValueError(f"dtype {dtype}: float64 or float32")
        self.shapes = [(int(a), int(b)) for a, b in shapes]
        self.n = len(self.shapes)
        bcs = [_bc_code(bc)] * self.n if not isinstance(bc, (list, tuple)) else [
            _bc_code(b) for b in bc]
        nx = (ctypes.c_int * self.n)(*[s[0] for s in self.shapes])
        ny = (ctypes.c_int * self.n)(*[s[1] for s in self.shapes])
        bcc = (ctypes.c_int * self.n)(*bcs)
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.handle = self.lib.hydro_batch_create(self.n, nx, ny, float(gamma), float(cfl), bcc)
            if not self.handle:
                raise HydroError(_lib.HYDRO_EINVAL, _lib.last_error())
            check(self.lib.hydro_batch_set_scalars(self.handle, int(nscalars)))
            self.nv = 4 + int(nscalars)
            offs = (ctypes.c_longlong * self.n)()
            pitches = (ctypes.c_long * self.n)()
            total = self.lib.hydro_batch_layout(self.handle, _DTYPE[dtype], offs, pitches)
            if total < 0:
                raise HydroError(int(total), _lib.last_error())
            self.offsets = list(offs)
            self.pitches = list(pitches)
            self.buf = torch.zeros(int(total), dtype=dtype, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            check(self.lib.hydro_batch_bind(self.handle, ctypes.c_void_p(self.buf.data_ptr()),
                                            _DTYPE[dtype], ctypes.c_void_p(self.stream.cuda_stream)))

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            self.lib.hydro_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view(self, g: int) -> torch.Tensor:
        nx, ny = self.shapes[g]
        p = self.pitches[g]
        o = self.offsets[g]
        return self.buf[o: o + self.nv * ny * p].view(self.nv, ny, p)[:, :, :nx]

    def set_states(self, states) -> None:
        self.stream.synchronize()
        torch.cuda.synchronize(self.device)
        for g, U in enumerate(states):
            t = torch.as_tensor(np.asarray(U) if not isinstance(U, torch.Tensor) else U)
            nx, ny = self.shapes[g]
            if tuple(t.shape) != (self.nv, ny, nx):
                raise ValueError(f"grid {g}: shape {tuple(t.shape)} != ({self.nv}, {ny}, {nx})")
            self.view(g).copy_(t.to(device=self.device, dtype=self.dtype))
        torch.cuda.synchronize(self.device)
        check(self.lib.hydro_batch_invalidate(self.handle))

    def get_states(self) -> list:
        self.stream.synchronize()
        return [self.view(g).detach().to("cpu").numpy().copy() for g in range(self.n)]

    def set_options(self, **kw) -> None:
        o = _lib.hydro_options_t(niter=10, tol=1e-8, guess=0, stats=0, seg_x=0, seg_y=0,
                                learned_gate=_lib.HYDRO_LEARNED_GATE_DEFAULT)
        for k, v in getattr(self, "_opts", {}).items():
            setattr(o, k, v)
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        check(self.lib.hydro_batch_set_options(self.handle, ctypes.byref(o)))
        self._opts = {k: getattr(o, k) for k, _ in o._fields_}

    def compute_dt(self) -> np.ndarray:
        out = (ctypes.c_double * self.n)()
        check(self.lib.hydro_batch_compute_dt(self.handle, out))
        return np.array(list(out))

    def step(self, n: int = 1) -> None:
        for _ in range(n):
            check(self.lib.hydro_batch_step(self.handle))

    def graph_steps(self, nsteps: int) -> None:
        check(self.lib.hydro_batch_graph_steps(self.handle, int(nsteps)))

    def totals(self) -> np.ndarray:
        out = (ctypes.c_double * (self.nv * self.n))()
        check(self.lib.hydro_batch_totals(self.handle, out))
        return np.array(list(out)).reshape(self.n, self.nv)

    def clock(self):
        t = (ctypes.c_double * self.n)()
        st = (ctypes.c_long * self.n)()
        dt = (ctypes.c_double * self.n)()
        check(self.lib.hydro_batch_get_clock(self.handle, t, st, dt))
        return np.array(list(t)), np.array(list(st)), np.array(list(dt))

    def stats(self, reset: bool = False) -> dict:
        s = _lib.hydro_stats_t()
        check(self.lib.hydro_batch_riemann_stats(self.handle, ctypes.byref(s), int(reset)))
        return _stats_dict(s)

    def autotune(self, use_cache: bool = True) -> dict:
        t = _lib.hydro_tune_t()
        check(self.lib.hydro_batch_autotune(self.handle, ctypes.byref(t), int(use_cache)))
        return _tune_dict(t)

    def set_profiling(self, enable: bool = True) -> None:
        check(self.lib.hydro_batch_set_profiling(self.handle, int(enable)))

    def set_mlp(self, net) -> None:
        self._net = net
        if net is not None:
            self.stream.wait_stream(net.stream)
        ptr = ctypes.c_void_p(net.dev.data_ptr()) if net is not None else None
        check(self.lib.hydro_batch_set_mlp(self.handle, ptr))

    def set_logger(self, records: torch.Tensor | None, seed: int = 0, rate_smooth: float = 0.01,
                   rate_strong: float = 1.0) -> None:
        self._log = records
        ptr = ctypes.c_void_p(records.data_ptr()) if records is not None else None
        cap = records.shape[0] if records is not None else 0
        check(self.lib.hydro_batch_set_logger(self.handle, ptr, cap, seed, rate_smooth,
                                              rate_strong))

    def logger_count(self) -> int:
        c = self.lib.hydro_batch_logger_count(self.handle)
        if c < 0:
            raise HydroError(int(c), _lib.last_error())
        return c

    def profile(self, reset: bool = True) -> dict:
        ms = (ctypes.c_double * _lib.HYDRO_NPHASES)()
        n = (ctypes.c_longlong * _lib.HYDRO_NPHASES)()
        check(self.lib.hydro_batch_get_profile(self.handle, ms, n, int(reset)))
        return _profile_dict(ms, n)


def step_noalloc(U: torch.Tensor, U_half: torch.Tensor, U_out: torch.Tensor, shapes, offsets,
                 pitches, bc, gamma: float = 1.4, cfl: float = 0.8,
                 dt_out: torch.Tensor | None = None,
                 stream: torch.cuda.Stream | None = None) -> None:
    """One time step of up to HYDRO_NOALLOC_MAX_GRIDS grids through
    hydro_step_noalloc (no handle, no device allocation).  U, U_half, U_out are
    flat device tensors of one dtype holding the grids at ``offsets`` with row
    ``pitches``; U_out may be U.  ``dt_out`` (float64, one per grid) receives
    each grid's dt.  Enqueued on ``stream`` (default: the current stream)."""
    lib = _lib.load()
    if U.dtype not in _DTYPE or U_half.dtype != U.dtype or U_out.dtype != U.dtype:
        raise ValueError("U, U_half, U_out: one dtype, float64 or float32")
    n = len(shapes)
    bcs = [_bc_code(bc)] * n if not isinstance(bc, (list, tuple)) else [_bc_code(b) for b in bc]
    nx = (ctypes.c_int * n)(*[int(s[0]) for s in shapes])
    ny = (ctypes.c_int * n)(*[int(s[1]) for s in shapes])
    bcc = (ctypes.c_int * n)(*bcs)
    offs = (ctypes.c_longlong * n)(*[int(o) for o in offsets])
    pit = (ctypes.c_long * n)(*[int(p) for p in pitches])
    if dt_out is not None and (dt_out.dtype != torch.float64 or dt_out.numel() < n):
        raise ValueError("dt_out: float64 tensor of at least one value per grid")
    s = stream if stream is not None else torch.cuda.current_stream(U.device)
    dtp = ctypes.c_void_p(dt_out.data_ptr()) if dt_out is not None else None
    check(lib.hydro_step_noalloc(n, nx, ny, bcc, offs, pit, _DTYPE[U.dtype], float(gamma),
                                 float(cfl), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(U_half.data_ptr()),
                                 ctypes.c_void_p(U_out.data_ptr()), dtp,
                                 ctypes.c_void_p(s.cuda_stream)))
