"""Parity of the batched path at its full benchmark sizes: the 256-grid
multi-blast batch (sides 64..1024, reflective) and the 64-grid quadrant batch
(sides 512..2048, outflow), one step in the launch configuration bench.py
times (autotuned, one persistent launch per sweep over all grids), every cell
of every grid against the oracle's step of that grid: FP64 to the parity bar,
FP32 by relative L1."""
import numpy as np
import pytest

from paper_2106_13465_amd import inputs
from test_gpu_parity import TOL64, rel_err

pytestmark = pytest.mark.gpu

BATCHES = {"multiblast": (inputs.multiblast_batch, 1), "quadrant": (inputs.quadrant_batch, 2)}


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module", params=sorted(BATCHES))
def batch_case(request, orc):
    gen, bc = BATCHES[request.param]
    print(f"full-size batch {request.param}: generating inputs", flush=True)
    grids = gen()
    c = orc.cfg(bc=bc)
    refs, dts = [], []
    for U in grids:
        V = U.copy()
        dts.append(orc.step(V, c))
        refs.append(V)
    return request.param, bc, grids, refs, np.array(dts)


def run_batch(torch, grids, bc, dtype):
    from paper_2106_13465_amd.hydro import HydroBatch

    b = HydroBatch([(U.shape[2], U.shape[1]) for U in grids], 1.4, 0.8, bc, dtype=dtype)
    b.set_states(grids)
    b.autotune(use_cache=True)
    b.set_states(grids)
    b.step(1)
    out = b.get_states()
    _, n, dt = b.clock()
    b.close()
    return out, n, dt


def test_fullsize_batch_fp64(torch_cuda, batch_case):
    name, bc, grids, refs, dts = batch_case
    print(f"full-size batch {name}: FP64 step of {len(grids)} grids", flush=True)
    got, n, dt = run_batch(torch_cuda, grids, bc, torch_cuda.float64)
    assert np.all(n == 1)
    assert np.all(np.abs(dt - dts) <= 1e-13 * dts)
    worst = 0.0
    for g, (a, r) in enumerate(zip(got, refs)):
        e = rel_err(a, r)
        worst = max(worst, e)
        assert e <= TOL64, (name, g, grids[g].shape, e)
    print(f"{name}: {len(grids)} grids, worst relative error {worst:.2e}")


def test_fullsize_batch_fp32_l1(torch_cuda, batch_case):
    name, bc, grids, refs, _ = batch_case
    print(f"full-size batch {name}: FP32 step of {len(grids)} grids", flush=True)
    got, _, _ = run_batch(torch_cuda, grids, bc, torch_cuda.float32)
    num = np.zeros(4)
    den = np.zeros(4)
    for a, r in zip(got, refs):
        a = a.astype(np.float64)
        for k in range(4):
            num[k] += np.abs(a[k] - r[k]).sum()
            den[k] += np.abs(r[k]).sum()
            if k in (0, 3):  # density and energy of each grid on its own as well
                assert np.abs(a[k] - r[k]).sum() <= 1e-5 * np.abs(r[k]).sum(), (name, k)
    l1 = num / den
    print(f"{name}: FP32 relative L1 over all grids {l1}")
    assert np.all(l1 < 1e-5)
