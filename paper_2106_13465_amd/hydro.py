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

__all__ = ["Hydro", "HydroError", "BC", "DIR_X", "DIR_Y"]

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

    The state lives in ``self.U`` (a torch tensor [4, ny, pitch] on the current
    HIP device; planes rho, rho u, rho v, E); ``self.state`` is its [4, ny, nx]
    view.  Work runs on a stream of the handle's own (a new torch stream at the
    default priority unless one is given), so the step can be graph-captured.
    """

    def __init__(self, nx: int, ny: int, gamma: float = 1.4, cfl: float = 0.8,
                 bc="periodic", dtype: torch.dtype = torch.float64, device="cuda",
                 pitch: int | None = None, stream: torch.cuda.Stream | None = None):
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
            self.pitch = int(pitch) if pitch is not None else _padded_pitch(self.nx, dtype)
            self.U = torch.zeros((4, self.ny, self.pitch), dtype=dtype, device=self.device)
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
        """Copy a [4, ny, nx] array (numpy or torch) into the bound state."""
        t = torch.as_tensor(np.asarray(U) if not isinstance(U, torch.Tensor) else U)
        if tuple(t.shape) != (4, self.ny, self.nx):
            raise ValueError(f"state shape {tuple(t.shape)} != (4, {self.ny}, {self.nx})")
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
        out = (ctypes.c_double * 4)()
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
        return {name: {"ms": ms[k], "launches": n[k]} for k, name in enumerate(_lib.PHASE_NAMES)}

    def stats(self, reset: bool = False) -> dict:
        s = _lib.hydro_stats_t()
        check(self.lib.hydro_riemann_stats(self.handle, ctypes.byref(s), int(reset)))
        return {"interfaces": s.interfaces, "hist": list(s.hist), "fallbacks": s.fallbacks}
