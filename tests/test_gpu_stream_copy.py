"""hydro_stream_copy, the streaming kernel bench.py measures the achievable
bandwidth with: a bitwise copy for sizes that exercise the four-word main loop
and the tail, on the caller's stream."""
import ctypes

import pytest

from paper_2106_13465_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("nbytes", [16, 1024 + 16, 256 * 1024 * 4 * 3 + 48, (64 << 20) + 16 * 5])
def test_stream_copy_is_bitwise(torch_cuda, nbytes):
    torch = torch_cuda
    print(f"stream copy {nbytes} B", flush=True)
    lib = _lib.load()
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 2**31 - 1, (nbytes // 4,), dtype=torch.int32, device="cuda",
                        generator=g)
    # 64 words of slack after the destination must stay untouched
    dst_full = torch.full((nbytes // 4 + 64,), -7, dtype=torch.int32, device="cuda")
    dst = dst_full[: nbytes // 4]
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    _lib.check(lib.hydro_stream_copy(ctypes.c_void_p(dst.data_ptr()),
                                     ctypes.c_void_p(src.data_ptr()), nbytes,
                                     ctypes.c_void_p(stream.cuda_stream)))
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert torch.all(dst_full[nbytes // 4:] == -7)
