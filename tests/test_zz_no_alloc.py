"""hydro_step_noalloc (the entry point for callers that cannot allocate device
memory) against hydro_step and hydro_batch_step on the same inputs: two calls
in a row on one GPU, the second with a smaller input, so the second call runs
on scratch the first one left behind."""
import ctypes

import numpy as np
import pytest

from paper_2106_13465_amd import _lib, inputs
from test_gpu_parity import TOL64, rel_err


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def pack(torch, states, dtype):
    """Grids packed one after another, rows padded to 256 bytes."""
    per = 256 // torch.tensor([], dtype=dtype).element_size()
    offsets, pitches, total = [], [], 0
    for U in states:
        ny, nx = U.shape[1:]
        p = (nx + per - 1) // per * per
        offsets.append(total)
        pitches.append(p)
        total += 4 * ny * p
    buf = torch.zeros(total, dtype=dtype, device="cuda")
    for U, o, p in zip(states, offsets, pitches):
        ny, nx = U.shape[1:]
        buf[o: o + 4 * ny * p].view(4, ny, p)[:, :, :nx].copy_(torch.as_tensor(U))
    return buf, offsets, pitches


def unpack(buf, states, offsets, pitches):
    out = []
    for U, o, p in zip(states, offsets, pitches):
        ny, nx = U.shape[1:]
        out.append(buf[o: o + 4 * ny * p].view(4, ny, p)[:, :, :nx].cpu().numpy().copy())
    return out


def run_noalloc(torch, states, bcs, dtype, in_place):
    from paper_2106_13465_amd.hydro import step_noalloc

    U, offsets, pitches = pack(torch, states, dtype)
    half = torch.full_like(U, float("nan"))
    out = U if in_place else torch.full_like(U, float("nan"))
    dt = torch.full((len(states),), -1.0, dtype=torch.float64, device="cuda")
    shapes = [(s.shape[2], s.shape[1]) for s in states]
    torch.cuda.synchronize()
    step_noalloc(U, half, out, shapes, offsets, pitches, bcs, 1.4, 0.8, dt_out=dt)
    torch.cuda.synchronize()
    return unpack(out, states, offsets, pitches), dt.cpu().numpy()


@pytest.mark.gpu
def test_two_calls_match_hydro_step_and_batch_step(torch_cuda):
    from paper_2106_13465_amd.hydro import Hydro, HydroBatch

    torch = torch_cuda
    # first call: three grids of a batch (the larger input)
    grids = [(300, 200, 1, 11), (130, 70, 3, 12), (61, 190, 2, 13)]
    states = [inputs.random_states(nx, ny, seed=s, rough=0.6) for nx, ny, _, s in grids]
    got, dts = run_noalloc(torch, states, [g[2] for g in grids], torch.float64, in_place=False)
    b = HydroBatch([(nx, ny) for nx, ny, _, _ in grids], 1.4, 0.8, [g[2] for g in grids],
                   dtype=torch.float64)
    b.set_states(states)
    b.step(1)
    ref = b.get_states()
    _, _, ref_dt = b.clock()
    for g in range(len(grids)):
        assert dts[g] == ref_dt[g], (g, dts[g], ref_dt[g])
        err = rel_err(got[g], ref[g])
        print(f"call 1 grid {g}: rel err {err:.2e}, bitwise {np.array_equal(got[g], ref[g])}")
        assert err <= TOL64, g

    # second call: one smaller grid, in place
    nx, ny = 70, 33
    U0 = inputs.random_states(nx, ny, seed=21, rough=0.6)
    got2, dt2 = run_noalloc(torch, [U0], [3], torch.float64, in_place=True)
    h = Hydro(nx, ny, 1.4, 0.8, "periodic", dtype=torch.float64)
    h.set_state(U0)
    h.step(1)
    ref2 = h.get_state()
    assert dt2[0] == h.clock()[2]
    err = rel_err(got2[0], ref2)
    print(f"call 2: rel err {err:.2e}, bitwise {np.array_equal(got2[0], ref2)}")
    assert err <= TOL64


@pytest.mark.gpu
def test_float32_matches_hydro_step(torch_cuda):
    from paper_2106_13465_amd.hydro import Hydro

    torch = torch_cuda
    nx, ny = 200, 96
    U0 = inputs.random_states(nx, ny, seed=31, rough=0.6)
    got, dt = run_noalloc(torch, [U0], [1], torch.float32, in_place=False)
    h = Hydro(nx, ny, 1.4, 0.8, "reflect", dtype=torch.float32)
    h.set_state(U0)
    h.step(1)
    ref = h.get_state()
    assert dt[0] == h.clock()[2]
    # same kernels, same inputs: agreement far inside the FP32 L1 bound
    l1 = max(np.abs(got[0][k] - ref[k]).sum() / np.abs(ref[k]).sum() for k in range(4))
    print(f"float32: rel L1 {l1:.2e}, bitwise {np.array_equal(got[0], ref)}")
    assert l1 <= 1e-6


def test_rejects_too_many_grids_before_device_work():
    """More grids than the static scratch holds: HYDRO_EINVAL from the
    argument check, before any HIP call (runs without a GPU)."""
    lib = _lib.load()
    n = _lib.HYDRO_NOALLOC_MAX_GRIDS + 1
    ints = (ctypes.c_int * n)(*([8] * n))
    bcs = (ctypes.c_int * n)(*([3] * n))
    offs = (ctypes.c_longlong * n)(*range(n))
    pit = (ctypes.c_long * n)(*([8] * n))
    dummy = ctypes.c_void_p(64)
    rc = lib.hydro_step_noalloc(n, ints, ints, bcs, offs, pit, _lib.HYDRO_F64, 1.4, 0.8, dummy,
                                ctypes.c_void_p(128), ctypes.c_void_p(256), None, None)
    assert rc == _lib.HYDRO_EINVAL
    assert "static device scratch" in _lib.last_error()


def test_rejects_overlapping_buffers_before_device_work():
    lib = _lib.load()
    ints = (ctypes.c_int * 1)(64)
    bcs = (ctypes.c_int * 1)(3)
    offs = (ctypes.c_longlong * 1)(0)
    pit = (ctypes.c_long * 1)(64)
    base = 1 << 20
    nbytes = 4 * 64 * 64 * 8
    U = ctypes.c_void_p(base)
    # U_half overlapping U
    rc = lib.hydro_step_noalloc(1, ints, ints, bcs, offs, pit, _lib.HYDRO_F64, 1.4, 0.8, U,
                                ctypes.c_void_p(base + nbytes // 2), ctypes.c_void_p(base),
                                None, None)
    assert rc == _lib.HYDRO_EINVAL and "U_half" in _lib.last_error()
    # U_out partly overlapping U
    rc = lib.hydro_step_noalloc(1, ints, ints, bcs, offs, pit, _lib.HYDRO_F64, 1.4, 0.8, U,
                                ctypes.c_void_p(base + 4 * nbytes),
                                ctypes.c_void_p(base + 8), None, None)
    assert rc == _lib.HYDRO_EINVAL and "U_out" in _lib.last_error()
