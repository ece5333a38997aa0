"""C ABI argument validation that returns before any device work, checked on
the CPU: every bad call returns its error code (or NULL) and leaves a
message; nothing aborts.  Also: without a GPU, a valid create fails cleanly."""
import ctypes
import threading

import pytest

from paper_2106_13465_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def err():
    return _lib.last_error()


def test_create_validation(lib):
    assert not lib.hydro_create(1, 5, 1.4, 0.8, 3) and ">= 2" in err()
    assert not lib.hydro_create(5, 1, 1.4, 0.8, 3)
    assert not lib.hydro_create(8, 8, 1.0, 0.8, 3) and "gamma" in err()
    assert not lib.hydro_create(8, 8, float("nan"), 0.8, 3)
    assert not lib.hydro_create(8, 8, 1.4, 0.0, 3) and "cfl" in err()
    assert not lib.hydro_create(8, 8, 1.4, 1.01, 3)
    assert not lib.hydro_create(8, 8, 1.4, 0.8, 0) and "bc" in err()
    assert not lib.hydro_create(8, 8, 1.4, 0.8, 4)


def test_batch_create_validation(lib):
    nx = (ctypes.c_int * 2)(8, 8)
    ny = (ctypes.c_int * 2)(8, 1)
    bc = (ctypes.c_int * 2)(1, 2)
    assert not lib.hydro_batch_create(0, nx, nx, 1.4, 0.8, bc)
    assert not lib.hydro_batch_create(2, None, nx, 1.4, 0.8, bc)
    assert not lib.hydro_batch_create(2, nx, ny, 1.4, 0.8, bc) and ">= 2" in err()


def test_null_handles(lib):
    o = _lib.hydro_options_t()
    assert lib.hydro_set_options(None, ctypes.byref(o)) == _lib.HYDRO_EINVAL
    assert lib.hydro_step(None) == _lib.HYDRO_EINVAL
    assert lib.hydro_sweep(None, 0) == _lib.HYDRO_EINVAL
    assert lib.hydro_compute_dt(None) < 0
    out = (ctypes.c_double * 4)()
    assert lib.hydro_conserved_totals(None, out) == _lib.HYDRO_EINVAL
    assert lib.hydro_bind(None, None, 8, 0, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_batch_layout(None, 0, None, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_set_scalars(None, 0) == _lib.HYDRO_EINVAL
    assert lib.hydro_batch_set_scalars(None, 1) == _lib.HYDRO_EINVAL
    st = _lib.hydro_stats_t()
    assert lib.hydro_riemann_stats(None, ctypes.byref(st), 0) == _lib.HYDRO_EINVAL
    lib.hydro_destroy(None)  # no-op
    lib.hydro_batch_destroy(None)


def test_mlp_argument_validation(lib):
    assert lib.hydro_mlp_dev_bytes() > 4 * 1313 // 2
    assert lib.hydro_mlp_grad_scratch_bytes(0) == lib.hydro_mlp_grad_scratch_bytes(1) > 0
    assert lib.hydro_mlp_pack(None, None, None) == _lib.HYDRO_EINVAL
    buf = (ctypes.c_float * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert lib.hydro_mlp_features(None, 4, 1.4, p, p, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_mlp_features(p, 4, 1.0, p, p, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_mlp_features(p, 0, 1.4, p, p, None) == _lib.HYDRO_OK  # nothing to do
    assert lib.hydro_mlp_forward(p, p, p, -1, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_mlp_forward(p, p, p, 0, None) == _lib.HYDRO_OK
    assert lib.hydro_mlp_grad(p, p, p, 0, p, p, p, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_mlp_adam(p, p, p, p, 0, 1e-3, 0.9, 0.999, 1e-8, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_mlp_adam(p, p, p, p, 1, 0.0, 0.9, 0.999, 1e-8, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_mlp_adam(p, p, p, p, 1, 1e-3, 1.0, 0.999, 1e-8, None) == _lib.HYDRO_EINVAL
    assert "Adam" in err()


def test_last_error_is_per_thread(lib):
    assert not lib.hydro_create(1, 5, 1.4, 0.8, 3)
    main_msg = err()
    seen = {}

    def other():
        seen["before"] = err()
        lib.hydro_create(8, 8, 1.4, 0.8, 9)
        seen["after"] = err()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["before"] == ""
    assert "bc" in seen["after"]
    assert err() == main_msg


def test_create_without_gpu_fails_cleanly(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = lib.hydro_create(8, 8, 1.4, 0.8, 3)
    assert not h
    assert err()  # a device error with the runtime's message


def test_stream_copy_validation(lib):
    """hydro_stream_copy rejects NULL, misaligned or overlapping arguments and
    sizes that are not whole 16-byte words before touching any memory (the
    addresses below are never dereferenced); 0 bytes is a no-op."""
    vp = ctypes.c_void_p
    assert lib.hydro_stream_copy(None, vp(4096), 16, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_stream_copy(vp(4096), None, 16, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_stream_copy(vp(4096), vp(8192), 24, None) == _lib.HYDRO_EINVAL
    assert "nbytes" in err()
    assert lib.hydro_stream_copy(vp(4096), vp(8192), -16, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_stream_copy(vp(4104), vp(8192), 16, None) == _lib.HYDRO_EINVAL
    assert "aligned" in err()
    assert lib.hydro_stream_copy(vp(4096), vp(8200), 16, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_stream_copy(vp(4096), vp(4096 + 32), 64, None) == _lib.HYDRO_EINVAL
    assert "overlap" in err()
    assert lib.hydro_stream_copy(vp(4096 + 32), vp(4096), 64, None) == _lib.HYDRO_EINVAL
    assert lib.hydro_stream_copy(vp(4096), vp(8192), 0, None) == _lib.HYDRO_OK
