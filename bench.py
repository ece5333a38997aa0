#!/usr/bin/env python3
"""Throughput of the split second-order Godunov step on one MI355X.

A step is one pass of the whole hot path over the grid: the CFL time step
(max wave speed fused into the previous y-sweep), the x-sweep and the y-sweep
(paper, Figure 5).  The default workload is the 8192 x 8192 periodic flow of 16
seeded Fourier modes plus 8 point blasts, 200 steps; the state is resident in
HBM before timing starts.

Prints one JSON line: whole-step cell-updates/s (two cell-updates per cell per
step), per-sweep times from HIP events recorded on the library's stream, the
roofline of the dominant sweep kernel, the FP32 variant, and the FP64 CPU
oracle timed on this host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per split step & HBM GB/s vs peak; learned+FP32 vs plain FP64"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# rocprofv3 counter summaries (HBM bytes per launch), one per workload
PMC_SUMMARY = {"fourier_blasts": "sweep_fourier_blasts_8192_pmc.json",
               "multiblast_batch": "sweep_multiblast_batch_256_pmc.json",
               "quadrant_batch": "sweep_quadrant_batch_64_pmc.json"}
KERNEL_SOURCES = ["paper_2106_13465_amd/csrc/kernels.hip", "paper_2106_13465_amd/csrc/sweeps.hpp",
                  "paper_2106_13465_amd/csrc/godunov.hpp",
                  "paper_2106_13465_amd/csrc/fastmath.hpp", "paper_2106_13465_amd/csrc/device_state.hpp",
                  "paper_2106_13465_amd/csrc/mlp.hpp"]


def code_of(text: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed: the
    part of a kernel source that the compiler turns into code (string and
    character literals are kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the kernel sources' code (comments and layout excluded), which
    the committed counter summaries record: bench.py takes traffic and issue
    figures from a summary only while it matches."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_of(f.read()).encode())
    return h.hexdigest()[:16]


def workload(name: str, n: int):
    from paper_2106_13465_amd import inputs

    if name == "fourier_blasts":
        return inputs.fourier_blasts(n), "periodic", (
            f"fourier_blasts {n}x{n}: rho = 1 + 0.3 S, u, v in [-0.5, 0.5] from 16 seeded "
            "Fourier modes (k <= 8), p = 1, 8 seeded point blasts E = 1/h^2; periodic")
    if name == "fourier_smooth":
        return inputs.fourier_blasts(n, nblasts=0), "periodic", (
            f"fourier_smooth {n}x{n}: the fourier_blasts field without the blasts (the "
            "flow moves: dt ~ 1e-4 instead of 2e-8); periodic")
    if name == "shear_layer":
        return inputs.shear_layer(n), "periodic", (
            f"shear_layer {n}x{n}: Kelvin-Helmholtz layer rho 2/1, u +-0.5, p 2.5, "
            "seeded v noise 0.01; periodic")
    if name == "blast_corner":
        return inputs.blast_corner(n), "reflect", (
            f"blast_corner {n}x{n}: rho 1, p 1e-5, corner cell E = 1/h^2; reflective")
    raise SystemExit(f"unknown workload {name}")


LIMITERS = {"minmod": 0, "mc": 1, "vanleer": 2}
ORDERS = {"xy": 0, "alternate": 1}
SOLVERS = {"two_shock": 0, "exact": 1, "hllc": 2}
YSWEEPS = {"march": 0, "tile": 1}


def run_gpu(U, bc, dtype_name, steps, warmup, seg_x=0, seg_y=0, autotune=True, limiter=0,
            order=0, riemann=0, ysweep=0):
    """U has 4 + n planes for n passive scalars."""
    import torch

    from paper_2106_13465_amd.hydro import Hydro

    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    _, ny, nx = U.shape
    h = Hydro(nx, ny, 1.4, 0.8, bc, dtype=dtype, device="cuda:0", nscalars=U.shape[0] - 4)
    h.set_options(limiter=limiter, order=order, riemann=riemann, ysweep=ysweep)
    if seg_x or seg_y:
        h.set_options(seg_x=seg_x, seg_y=seg_y)
    h.set_state(U)
    tune = h.autotune(use_cache=True) if autotune else None
    h.step(warmup)
    torch.cuda.synchronize()
    h.profile(reset=True)
    h.set_profiling(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(h.stream)
    t0 = time.perf_counter()
    h.step(steps)
    stop.record(h.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    prof = h.profile(reset=True)
    h.set_profiling(False)
    t, nsteps, dt = h.clock()
    return h, {"ms_total": ms_total, "wall_s": wall, "profile": prof, "t": t, "steps_done": nsteps,
               "dt": dt, "tune": tune}


def newton_report(h):
    """Newton iterations per interface over one extra (untimed) step."""
    h.set_options(stats=1)
    h.stats(reset=True)
    h.step(1)
    s = h.stats(reset=True)
    h.set_options(stats=0)
    hist = s["hist"]
    conv = sum(hist[1:])
    mean = sum(k * n for k, n in enumerate(hist) if k > 0) / max(conv, 1)
    wh = s["wave_hist"]
    waves = sum(wh)
    return {"interfaces": s["interfaces"], "mean_iterations": mean, "unconverged": hist[0],
            "hist": {str(k): n for k, n in enumerate(hist) if n},
            "wave_mean_max_iterations": sum(k * n for k, n in enumerate(wh)) / max(waves, 1),
            "wave_hist": {str(k): n for k, n in enumerate(wh) if n}}


def sweep_record(cells, elem, phase, nv=4):
    ms = phase["ms"] / max(phase["launches"], 1)
    alg_bytes = cells * 2 * nv * elem  # read nv words + write nv words per cell
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    return {"avg_ms": ms, "launches": phase["launches"], "cell_updates_per_s": cells / (ms * 1e-3),
            "algorithmic_bytes": alg_bytes, "hbm_gbps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def copy_bandwidth(nbytes: int, reps: int = 10) -> dict:
    """GB/s of a plain device-to-device copy of nbytes (nbytes read and nbytes
    written, timed with HIP events on one stream): the library's streaming
    copy kernel (hydro_stream_copy: 8 KiB per block, nontemporal loads and stores) and
    torch's copy, the bandwidth a streaming kernel reaches on this GPU for a
    transfer as large as one sweep's."""
    import ctypes

    import torch
    from paper_2106_13465_amd import _lib

    lib = _lib.load()
    n = max(nbytes // 16, 1) * 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    out = {}
    for name, fn in (("hip_stream_copy", lambda: _lib.check(lib.hydro_stream_copy(
            ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), 4 * n, sp))),
                     ("torch_copy", lambda: dst.copy_(src))):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = 2.0 * 4 * n / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    assert torch.equal(dst, src)
    del src, dst
    torch.cuda.empty_cache()
    return out


def with_copy(roofline: dict) -> dict:
    """Adds the achievable streaming bandwidth (a device copy of the dominant
    sweep's algorithmic bytes, half read and half written: the faster of the
    library's streaming kernel and torch's copy) and the sweep's fraction of
    it; frac stays against the published peak."""
    cb = copy_bandwidth(int(roofline["algorithmic_bytes_per_launch"]) // 2)
    roofline["copy"] = cb
    roofline["copy_gbps"] = max(cb.values())
    roofline["frac_of_copy"] = roofline["achieved"] / roofline["copy_gbps"]
    return roofline


def pmc_traffic(workload_name: str, kernel: str, dtype_name: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of the workload, or None if missing or taken from different kernel
    sources."""
    if workload_name not in PMC_SUMMARY:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", PMC_SUMMARY[workload_name])) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(f"{kernel}_{dtype_name}")
    return None if ent is None else ent.get("bytes_per_launch")


VALU_SUMMARY = {"fourier_blasts": "sweep_fourier_blasts_8192_valu.json"}


def valu_issue(workload_name: str, kernel: str, dtype_name: str, measured_ms: float):
    """The competing bound beside HBM: the committed instruction-count summary
    gives the sweep's VALU instructions per launch; at 4 cycles per wave64
    instruction on 1024 SIMDs they need `issue_floor_ms` at the shader clock
    the same counter run measured (GRBM_GUI_ACTIVE cycles of the 8 XCDs over
    the kernel's duration), and `issue_floor_ms_2p4ghz` at the 2.4 GHz peak
    clock.  frac = floor at the measured clock / the launch time measured now.
    None if missing or taken from different kernel sources."""
    if workload_name not in VALU_SUMMARY:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", VALU_SUMMARY[workload_name])) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(f"{kernel}_{dtype_name}")
    if ent is None:
        return None
    c = ent["counters"]
    clock_ghz = c["GRBM_GUI_ACTIVE"] / 8.0 / (c["_t"] * 1e-3) / 1e9
    floor_ms = c["SQ_INSTS_VALU"] * 4.0 / (1024 * clock_ghz * 1e9) * 1e3
    return {"valu_per_lane_cell": ent["valu_per_lane_cell"], "clock_ghz": clock_ghz,
            "issue_floor_ms": floor_ms, "issue_floor_ms_2p4ghz": ent["issue_floor_ms"],
            "measured_ms": measured_ms, "frac": floor_ms / measured_ms,
            "frac_2p4ghz": ent["issue_floor_ms"] / measured_ms}


def cpu_model() -> str:
    """Model name of this host's CPU (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def compare_to_oracle(got, ref):
    """FP64 parity figure and FP32 accuracy figure of a GPU state against the
    oracle's: per variable the largest difference over the variable's scale
    (max |.| for rho and E; for the momenta max(max |m|, sqrt(2 rho E)) cell by
    cell, the scale of a momentum that is a difference of large impulses), and
    the relative L1 error sum |got - ref| / sum |ref|."""
    import numpy as np

    got = got.astype(np.float64, copy=False)
    out = {"max_rel_err": [], "rel_l1": []}
    for k in range(ref.shape[0]):
        d = np.abs(got[k] - ref[k])
        if k in (1, 2):
            mmax = max(float(np.abs(ref[1]).max()), float(np.abs(ref[2]).max()))
            scale = np.maximum(mmax, np.sqrt(2.0 * np.abs(ref[0] * ref[3])))
            out["max_rel_err"].append(float((d / scale).max()))
        else:
            out["max_rel_err"].append(float(d.max() / max(float(np.abs(ref[k]).max()), 1e-300)))
        out["rel_l1"].append(float(d.sum() / max(float(np.abs(ref[k]).sum()), 1e-300)))
        del d
    return out


def gpu_steps_from(U, bc, dtype_name, nsteps, limiter=0, order=0, riemann=0):
    """State after nsteps eager steps from U on the GPU (default launch shape;
    results do not depend on it)."""
    import torch

    from paper_2106_13465_amd.hydro import Hydro

    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    _, ny, nx = U.shape
    h = Hydro(nx, ny, 1.4, 0.8, bc, dtype=dtype, device="cuda:0", nscalars=U.shape[0] - 4)
    h.set_options(limiter=limiter, order=order, riemann=riemann)
    h.set_state(U)
    h.step(nsteps)
    out = h.get_state()
    h.close()
    del h
    torch.cuda.empty_cache()
    return out


def cpu_baseline(U, bc_name, limiter=0, order=0, riemann=0, state_out=None):
    """The oracle timed on this host: one full step of the whole input on all
    OpenMP threads (the reported value), and one step of its top-left 2048^2
    corner (same boundary rule) on one thread.  The state after the full step
    is appended to state_out when given."""
    import numpy as np

    import oracle

    bc = {"periodic": oracle.BC_PERIODIC, "reflect": oracle.BC_REFLECT,
          "outflow": oracle.BC_OUTFLOW}[bc_name]
    c = oracle.cfg(bc=bc, limiter=limiter, order=order, riemann=riemann,
                   nscalars=U.shape[0] - 4)
    V = U.copy()
    _, ny, nx = V.shape
    threads = oracle.threads()
    t0 = time.perf_counter()
    oracle.step(V, c)
    sec = time.perf_counter() - t0
    if state_out is not None:
        state_out.append(V)
    del V
    m = min(2048, nx, ny)
    W = np.ascontiguousarray(U[:, :m, :m])
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.step(W, c)
        sec1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    # the paper's three OpenMP schemes on the same corner (speedup tables in
    # the form of its Figures 11-13); each step equals the serial one bitwise
    names = {oracle.SCHEME_FINE: "fine_grain", oracle.SCHEME_COARSE: "coarse_grain",
             oracle.SCHEME_TASKS: "tasks"}
    counts = [t for t in (1, 2, 4, 8, 16) if t <= max(threads, 1)]
    schemes = {}
    for sc, name in names.items():
        rows = []
        for t in counts:
            X = W.copy()
            t2 = time.perf_counter()
            oracle.step_scheme(X, c, sc, t)
            rows.append({"threads": t, "seconds": time.perf_counter() - t2})
        for r in rows:
            r["speedup"] = rows[0]["seconds"] / r["seconds"]
            r["efficiency"] = r["speedup"] / r["threads"]
        schemes[name] = rows
    oracle.set_threads(threads)
    return {"value": 2.0 * nx * ny / sec, "unit": "cell-updates/s", "cores": threads,
            "cpu_model": cpu_model(), "kind": "oracle", "seconds": sec,
            "sample": f"1 full step (dt, x-sweep, y-sweep) of the same {nx}x{ny} input, FP64, "
                      f"{threads} OpenMP threads over pencils",
            "single_core": {"value": 2.0 * m * m / sec1, "seconds": sec1,
                            "sample": f"1 step of the top-left {m}x{m} corner, 1 thread"},
            "openmp_schemes": {"sample": f"1 step of the top-left {m}x{m} corner per entry",
                               **schemes}}


def oracle_cfg(bc_name, limiter=0, order=0, riemann=0, nscalars=0):
    import oracle

    bc = {"periodic": oracle.BC_PERIODIC, "reflect": oracle.BC_REFLECT,
          "outflow": oracle.BC_OUTFLOW}[bc_name]
    return oracle.cfg(bc=bc, limiter=limiter, order=order, riemann=riemann, nscalars=nscalars)


def c1_cpu(U, bc_name, steps, state_out):
    """The point-explosion configuration's own metric: seconds of the whole
    run (steps time steps) of the FP64 oracle on one core and on every core of
    this host; both runs give the same state (pencils are independent)."""
    import numpy as np

    import oracle

    c = oracle_cfg(bc_name)
    threads = oracle.threads()
    res = {}
    finals = []
    for name, t in (("one_core", 1), ("all_cores", threads)):
        oracle.set_threads(t)
        V = U.copy()
        t0 = time.perf_counter()
        for _ in range(steps):
            oracle.step(V, c)
        res[name] = {"threads": t, "seconds": time.perf_counter() - t0}
        finals.append(V)
    oracle.set_threads(threads)
    _, ny, nx = U.shape
    state_out.append(finals[0])
    return {"value": res["all_cores"]["seconds"], "unit": "s (whole run)", "cores": threads,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"the whole run: {steps} steps of the {nx}x{ny} input, FP64",
            "one_core_seconds": res["one_core"]["seconds"],
            "all_cores_seconds": res["all_cores"]["seconds"],
            "cell_updates_per_s_all_cores": 2.0 * nx * ny * steps / res["all_cores"]["seconds"],
            "cell_updates_per_s_one_core": 2.0 * nx * ny * steps / res["one_core"]["seconds"],
            "one_core_equals_all_cores_bitwise": bool(np.array_equal(finals[0], finals[1]))}


STRONG_FAMILY = {"p_decades": 4.0, "rho_decades": 2.0, "speed": 3.0}


def bench_strong(args) -> dict:
    """Strong jumps, the regime where the Riemann solve iterates: 4096^2 cells
    of independent random states (p over 4 decades, rho over 2, |u|, |v| up to
    3), periodic.  One step from the same input, repeated: the per-sweep times
    and the iteration histogram of that step, FP64 and FP32, against the
    oracle's step of the whole grid."""
    import numpy as np
    import torch

    from paper_2106_13465_amd import inputs
    from paper_2106_13465_amd.hydro import Hydro

    n = args.size or 4096
    reps = args.steps if args.steps_given else 20
    print(f"# generating strong_jumps {n}^2", file=sys.stderr, flush=True)
    U = inputs.strong_jumps(n, n, 32, **STRONG_FAMILY)
    cells = n * n
    desc = (f"strong_jumps {n}x{n}: independent random states per cell, rho log-uniform over 2 "
            "decades, p over 4, u, v uniform in [-3, 3] (seed 32); periodic; one step from "
            "this input, repeated")
    results = {}
    for dn in ("f64", "f32"):
        print(f"# gpu {dn}: {reps} x (reset, 1 step)", file=sys.stderr, flush=True)
        dtype = torch.float64 if dn == "f64" else torch.float32
        elem = 8 if dn == "f64" else 4
        h = Hydro(n, n, 1.4, 0.8, "periodic", dtype=dtype, device="cuda:0")
        h.set_state(U)
        tune = None if args.no_autotune else h.autotune(use_cache=True)
        h.set_state(U)
        h.set_options(stats=1)
        h.stats(reset=True)
        h.step(1)
        it = h.stats(reset=True)
        h.set_options(stats=0)
        got = h.get_state()
        h.set_profiling(True)
        steps_ms = []
        h.profile(reset=True)
        for _ in range(reps):
            h.set_state(U)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(h.stream)
            h.step(1)
            b.record(h.stream)
            torch.cuda.synchronize()
            steps_ms.append(a.elapsed_time(b))
        prof = h.profile(reset=True)
        h.set_profiling(False)
        h.close()
        del h
        torch.cuda.empty_cache()
        hist = it["hist"]
        conv = sum(hist[1:])
        wh = it["wave_hist"]
        ms = float(np.median(steps_ms))
        results[dn] = {
            "value": 2.0 * cells / (ms * 1e-3), "ms_per_step": ms,
            "sweeps": {"x": sweep_record(cells, elem, prof["sweep_x"]),
                       "y": sweep_record(cells, elem, prof["sweep_y"])},
            "launch_shape": tune,
            "newton": {"interfaces": it["interfaces"], "unconverged": hist[0],
                       "mean_iterations": sum(k * m for k, m in enumerate(hist) if k > 0)
                       / max(conv, 1),
                       "hist": {str(k): m for k, m in enumerate(hist) if m},
                       "wave_mean_max_iterations": sum(k * m for k, m in enumerate(wh))
                       / max(sum(wh), 1),
                       "wave_hist": {str(k): m for k, m in enumerate(wh) if m}},
            "state": got}
    res = results["f64"]
    sx, sy = res["sweeps"]["x"], res["sweeps"]["y"]
    dom_name, dom = ("sweep_x", sx) if sx["avg_ms"] >= sy["avg_ms"] else ("sweep_y", sy)
    line = {
        "metric": METRIC, "value": res["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": reps, "warmup": 0, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "nx": n, "ny": n, "bc": "periodic", "gamma": 1.4,
                   "cfl": 0.8, "limiter": "minmod", "riemann": "two_shock", "newton_cap": 10,
                   "newton_tol": 1e-8, "parallelism": "single GPU"},
        "sweeps": res["sweeps"], "launch_shape": res["launch_shape"], "newton": res["newton"],
        "roofline": with_copy({"bound": "hbm", "kernel": dom_name, "achieved": dom["hbm_gbps"],
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": dom["hbm_gbps"] / HBM_PEAK_GBS, "traffic": None,
                               "algorithmic_bytes_per_launch": dom["algorithmic_bytes"],
                               "avg_launch_ms": dom["avg_ms"]}),
        "f32": {k: v for k, v in results["f32"].items() if k != "state"},
    }
    line["f32"]["speedup_vs_f64"] = results["f32"]["value"] / res["value"]
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle, whole grid, one step)", file=sys.stderr, flush=True)
        ref = []
        line["cpu_baseline"] = cpu_baseline(U, "periodic", state_out=ref)
        line["vs_oracle_after_1_step"] = {
            "f64": compare_to_oracle(results["f64"]["state"], ref[0]),
            "f32": compare_to_oracle(results["f32"]["state"], ref[0])}
    return line


BATCH_WORKLOADS = {
    "multiblast_batch": ("reflect", 100, (
        "multiblast_batch: 256 square grids, side log-uniform 64..1024 (sum of cells "
        "{cells}), rho 1, u = v = 0, p log-uniform 1e-5..1, 1-8 blasts per grid with energy "
        "log-uniform 1e-2..1e2; reflective")),
    "quadrant_batch": ("outflow", 200, (
        "quadrant_batch: 64 square grids, side log-uniform 512..2048 (sum of cells {cells}), "
        "four constant states with rho, p log-uniform 0.1..2 (2e-5..2 for p in 10% of grids), "
        "u, v uniform -1..1; outflow")),
}


def bench_batch(args) -> dict:
    """Batched workloads: one persistent launch per sweep over all grids, the
    step captured in a HIP graph; compared with a loop of per-grid handles."""
    import numpy as np
    import torch

    from paper_2106_13465_amd import inputs
    from paper_2106_13465_amd.hydro import Hydro, HydroBatch

    bc, default_steps, desc = BATCH_WORKLOADS[args.workload]
    steps = args.steps if args.steps_given else default_steps
    print(f"# generating {args.workload}", file=sys.stderr, flush=True)
    grids = (inputs.multiblast_batch() if args.workload == "multiblast_batch"
             else inputs.quadrant_batch())
    shapes = [(U.shape[2], U.shape[1]) for U in grids]
    cells = sum(nx * ny for nx, ny in shapes)
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    elem = 8 if args.dtype == "f64" else 4
    b = HydroBatch(shapes, 1.4, 0.8, bc, dtype=dtype, device="cuda:0")
    b.set_states(grids)
    tune = None if args.no_autotune else b.autotune(use_cache=True)
    graph_n = min(steps, 50)
    # warmup (also captures the graph)
    b.step(args.warmup)
    b.graph_steps(graph_n)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    done = 0
    start.record(b.stream)
    while done + graph_n <= steps:
        b.graph_steps(graph_n)
        done += graph_n
    b.step(steps - done)
    stop.record(b.stream)
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    # per-kernel times from an eager, profiled pass of a few steps
    b.set_profiling(True)
    b.profile(reset=True)
    b.step(10)
    prof = b.profile(reset=True)
    b.set_profiling(False)
    sx = sweep_record(cells, elem, prof["sweep_x"])
    sy = sweep_record(cells, elem, prof["sweep_y"])
    b.set_options(stats=1)
    b.stats(reset=True)
    b.step(1)
    st = b.stats(reset=True)
    b.set_options(stats=0)
    hist = st["hist"]
    conv = sum(hist[1:])
    newton = {"interfaces": st["interfaces"], "unconverged": hist[0],
              "mean_iterations": sum(k * n for k, n in enumerate(hist) if k > 0) / max(conv, 1),
              "wave_mean_max_iterations": sum(k * n for k, n in enumerate(st["wave_hist"]))
              / max(sum(st["wave_hist"]), 1)}
    t, n, _ = b.clock()
    b.close()
    del b
    torch.cuda.empty_cache()

    # baseline: one handle per grid, eager steps in a loop (3 launches per grid per step)
    print("# per-grid launch loop", file=sys.stderr, flush=True)
    hs = []
    for U in grids:
        h = Hydro(U.shape[2], U.shape[1], 1.4, 0.8, bc, dtype=dtype, device="cuda:0")
        h.set_state(U)
        hs.append(h)
    loop_steps = max(1, min(steps, 20))
    for h in hs:
        h.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(loop_steps):
        for h in hs:
            h.step(1)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3 / loop_steps
    for h in hs:
        h.close()
    del hs
    torch.cuda.empty_cache()

    ms_step = ms_total / steps
    dom_name, dom = ("sweep_x", sx) if sx["avg_ms"] >= sy["avg_ms"] else ("sweep_y", sy)
    line = {
        "metric": METRIC, "value": 2.0 * cells * steps / (ms_total * 1e-3),
        "unit": "cell-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": desc.format(cells=cells), "grids": len(grids), "cells": cells,
                   "bc": bc, "gamma": 1.4, "cfl": 0.8, "graph_steps_per_replay": graph_n,
                   "parallelism": "single GPU, one persistent launch per sweep"},
        "sweeps": {"x": sx, "y": sy},
        "launch_shape": tune,
        "newton": newton,
        "roofline": with_copy({"bound": "hbm", "kernel": dom_name, "achieved": dom["hbm_gbps"],
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": dom["hbm_gbps"] / HBM_PEAK_GBS,
                               "traffic": pmc_traffic(args.workload, dom_name, args.dtype),
                               "algorithmic_bytes_per_launch": dom["algorithmic_bytes"],
                               "avg_launch_ms": dom["avg_ms"]}),
        "per_grid_loop": {"ms_per_step": loop_ms, "speedup_of_batched_graph": loop_ms / ms_step},
        "sim_time": {"min": float(np.min(t)), "max": float(np.max(t))},
    }
    if not args.no_cpu_baseline:
        import oracle

        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        sample = grids[:16]
        t0 = time.perf_counter()
        cu = 0
        for U, (nx, ny) in zip(sample, shapes[:16]):
            V = U.copy()
            oracle.step(V, oracle.cfg(bc={"reflect": 1, "outflow": 2, "periodic": 3}[bc]))
            cu += 2 * nx * ny
        sec = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": cu / sec, "unit": "cell-updates/s",
                                "cores": oracle.threads(), "kind": "oracle", "seconds": sec,
                                "sample": f"1 step of the first 16 grids ({cu // 2} cells), FP64, "
                                          f"{oracle.threads()} OpenMP threads"}
    return line


def _iter_stats(obj):
    s = obj.stats(reset=True)
    hist = s["hist"]
    conv = sum(hist[1:])
    wh = s["wave_hist"]
    return {"interfaces": s["interfaces"], "unconverged": hist[0], "fallbacks": s["fallbacks"],
            "mean_iterations": sum(k * n for k, n in enumerate(hist) if k > 0) / max(conv, 1),
            "wave_mean_max_iterations": sum(k * n for k, n in enumerate(wh)) / max(sum(wh), 1),
            "fallback_rate": s["fallbacks"] / max(s["interfaces"], 1)}


def _timed_steps(obj, steps, graph=False):
    import torch

    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(obj.stream)
    if graph:
        obj.graph_steps(steps)
    else:
        obj.step(steps)
    b.record(obj.stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


STRONG_FAMILIES = {"strong_jumps_p2": dict(p_decades=2.0, rho_decades=1.0, speed=2.0),
                   "strong_jumps_p4": dict(p_decades=4.0, rho_decades=2.0, speed=3.0)}


def strong_jump_study(fam, n=4096, reps=3) -> dict:
    """The learned guess where the two-rarefaction guess is poor: a network
    trained (20 epochs) on the interface states the solver logs in one step of
    a 1024^2 grid of strong jumps of the family, then the first step of a fresh
    n^2 grid of the family with the two-rarefaction guess, the gated learned
    guess and the learned guess everywhere, FP64 and FP32: iterations, sweep
    times (best of reps), and the time ratio to the two-rarefaction start."""
    import torch

    from paper_2106_13465_amd import inputs
    from paper_2106_13465_amd.hydro import Hydro
    from paper_2106_13465_amd._lib import HYDRO_LEARNED_GATE_DEFAULT as GATE_DEFAULT
    from paper_2106_13465_amd.mlp import GuessNetwork

    rec = torch.zeros((2_200_000, 8), dtype=torch.float32, device="cuda:0")
    h = Hydro(1024, 1024, 1.4, 0.8, "periodic", dtype=torch.float64, device="cuda:0")
    h.set_state(inputs.strong_jumps(1024, 1024, 31, **fam))
    h.set_logger(rec, seed=7, rate_smooth=1.0, rate_strong=1.0)
    h.step(1)
    nrec = min(h.logger_count(), rec.shape[0])
    h.set_logger(None)
    h.close()
    net_s = GuessNetwork(seed=0, device="cuda:0")
    X, Y = net_s.features(rec[:nrec])
    del rec
    hist = net_s.train(X, Y, epochs=20, batch=2048, lr=2e-3, seed=1)
    err = (net_s.forward(X) - Y).abs()[Y.abs() < 8].float()
    sres = {"family": fam, "grid": f"{n}^2, periodic, first step of a fresh seed",
            "training": {"records": nrec, "epochs": 20, "batch": 2048, "lr": 2e-3,
                         "loss_first_last": [hist[0], hist[-1]],
                         "median_abs_ln_error": float(err.median().item()),
                         "p90_abs_ln_error": float(torch.quantile(err[:1_000_000], 0.9).item())}}
    del X, Y, err
    U4 = inputs.strong_jumps(n, n, 32, **fam)
    for dn, dt in (("f64", torch.float64), ("f32", torch.float32)):
        for name, guess, gate in (("two_rarefaction", 0, 0.0), ("learned", 1, GATE_DEFAULT),
                                  ("learned_everywhere", 1, 0.0)):
            h = Hydro(n, n, 1.4, 0.8, "periodic", dtype=dt, device="cuda:0")
            if guess:
                h.set_mlp(net_s)
            h.set_options(guess=guess, learned_gate=gate, stats=1)
            h.set_state(U4)
            h.step(1)
            it = _iter_stats(h)
            h.set_options(stats=0)
            h.set_profiling(True)
            xs, ys = [], []
            for _ in range(reps):
                h.set_state(U4)
                h.profile(reset=True)
                h.step(1)
                pr = h.profile(reset=True)
                xs.append(pr["sweep_x"]["ms"])
                ys.append(pr["sweep_y"]["ms"])
            h.close()
            del h
            sres[f"{dn}_{name}"] = {"newton": it, "sweep_x_ms": min(xs), "sweep_y_ms": min(ys)}
        base = sres[f"{dn}_two_rarefaction"]
        for name in ("learned", "learned_everywhere"):
            r = sres[f"{dn}_{name}"]
            r["iteration_ratio_vs_two_rarefaction"] = (
                r["newton"]["mean_iterations"] / base["newton"]["mean_iterations"])
            r["wave_max_iteration_ratio_vs_two_rarefaction"] = (
                r["newton"]["wave_mean_max_iterations"]
                / base["newton"]["wave_mean_max_iterations"])
            r["sweep_time_ratio_vs_two_rarefaction"] = (
                (r["sweep_x_ms"] + r["sweep_y_ms"]) / (base["sweep_x_ms"] + base["sweep_y_ms"]))
    del U4
    torch.cuda.empty_cache()
    return sres


def bench_learned(args) -> dict:
    """Learned Riemann guess: log interface states from the corner-blast and
    Fourier+blasts runs, train the network on the GPU, then compare it with the
    two-rarefaction guess (iterations, time, results) on the 4096^2 shear
    layer and on the 64-grid quadrant batch; the batch is also run in plain
    FP64 for the speedup of learned + batched FP32 over the plain FP64 path."""
    import numpy as np
    import torch

    from paper_2106_13465_amd import inputs
    from paper_2106_13465_amd.hydro import Hydro, HydroBatch
    from paper_2106_13465_amd._lib import HYDRO_LEARNED_GATE_DEFAULT as GATE_DEFAULT
    from paper_2106_13465_amd.mlp import GuessNetwork

    out = {}
    cap = args.train_records
    records = torch.zeros((cap, 8), dtype=torch.float32, device="cuda:0")
    # --- logging: corner blast 128^2 FP64 (100 steps), Fourier+blasts 8192^2 FP32
    print("# logging interface states", file=sys.stderr, flush=True)
    h = Hydro(128, 128, 1.4, 0.8, "reflect", dtype=torch.float64, device="cuda:0")
    h.set_state(inputs.blast_corner(128))
    h.set_logger(records, seed=11, rate_smooth=0.05, rate_strong=1.0)
    h.step(100)
    n1 = min(h.logger_count(), cap)
    h.set_logger(None)
    h.close()
    U2 = inputs.fourier_blasts(8192)
    h = Hydro(8192, 8192, 1.4, 0.8, "periodic", dtype=torch.float32, device="cuda:0")
    h.set_state(U2)
    del U2
    h.set_logger(records[n1:], seed=12, rate_smooth=0.0065, rate_strong=1.0)
    h.step(12)
    n2 = min(h.logger_count(), cap - n1)
    h.set_logger(None)
    h.close()
    del h
    torch.cuda.empty_cache()
    n = n1 + n2
    out["training_data"] = {"records": n, "from_blast_corner_128": n1,
                            "from_fourier_blasts_8192": n2}
    # --- training
    print(f"# training on {n} records", file=sys.stderr, flush=True)
    net = GuessNetwork(seed=0, device="cuda:0")
    X, Y = net.features(records[:n])
    del records
    t0 = time.perf_counter()
    hist = net.train(X, Y, epochs=args.train_epochs, batch=8192, lr=1e-3, seed=1)
    train_s = time.perf_counter() - t0
    keep = Y.abs() < 8
    err = (net.forward(X) - Y).abs()[keep].float()
    out["training"] = {"epochs": args.train_epochs, "batch": 8192, "lr": 1e-3,
                       "loss_per_epoch": hist, "seconds": train_s,
                       "median_abs_ln_error": float(err.median().item()),
                       "p90_abs_ln_error": float(torch.quantile(err[:1_000_000], 0.9).item())}
    del X, Y, err, keep
    torch.cuda.empty_cache()

    # --- shear layer 4096^2 FP32: two-rarefaction vs learned guess
    print("# shear layer 4096^2 FP32", file=sys.stderr, flush=True)
    U3 = inputs.shear_layer(4096)
    steps = 200 if not args.steps_given else args.steps
    res = {}
    finals = {}
    for guess, gate in (("two_rarefaction", 0.0), ("learned", GATE_DEFAULT),
                        ("learned_everywhere", 0.0)):
        h = Hydro(4096, 4096, 1.4, 0.8, "periodic", dtype=torch.float32, device="cuda:0")
        h.set_state(U3)
        if guess != "two_rarefaction":
            h.set_mlp(net)
            h.set_options(guess=1, learned_gate=gate)
        h.autotune(use_cache=True)
        h.step(args.warmup)
        h.set_profiling(True)
        h.profile(reset=True)
        ms = _timed_steps(h, steps)
        prof = h.profile(reset=True)
        h.set_profiling(False)
        h.set_options(stats=1)
        h.stats(reset=True)
        h.step(1)
        it = _iter_stats(h)
        res[guess] = {"ms_per_step": ms, "cell_updates_per_s": 2 * 4096 * 4096 / (ms * 1e-3),
                      "sweep_x_ms": prof["sweep_x"]["ms"] / max(prof["sweep_x"]["launches"], 1),
                      "sweep_y_ms": prof["sweep_y"]["ms"] / max(prof["sweep_y"]["launches"], 1),
                      "newton": it}
        finals[guess] = h.get_state()
        h.close()
        del h
        torch.cuda.empty_cache()
    b = finals["two_rarefaction"].astype(np.float64)
    for name in ("learned", "learned_everywhere"):
        a = finals[name].astype(np.float64)
        res[name]["rel_l1_vs_two_rarefaction"] = [
            float(np.abs(a[k] - b[k]).sum() / max(np.abs(b[k]).sum(), 1e-300)) for k in range(4)]
        res[name]["speedup_vs_two_rarefaction"] = (res["two_rarefaction"]["ms_per_step"] /
                                                   res[name]["ms_per_step"])
    res["learned_gate"] = GATE_DEFAULT
    out["shear_layer_4096_f32"] = res
    del U3, finals
    # --- quadrant batch: plain FP64 vs FP32 two-rarefaction vs FP32 learned (graph steps)
    print("# quadrant batch", file=sys.stderr, flush=True)
    grids = inputs.quadrant_batch()
    shapes = [(U.shape[2], U.shape[1]) for U in grids]
    cells = sum(a_ * b_ for a_, b_ in shapes)
    qsteps = 50 if not args.steps_given else args.steps
    qres = {}
    qfinal = {}
    for name, dtype, guess, gate in (
            ("plain_f64", torch.float64, 0, 0.0), ("f32_two_rarefaction", torch.float32, 0, 0.0),
            ("f32_learned", torch.float32, 1, GATE_DEFAULT),
            ("f32_learned_everywhere", torch.float32, 1, 0.0)):
        bt = HydroBatch(shapes, 1.4, 0.8, "outflow", dtype=dtype, device="cuda:0")
        bt.set_states(grids)
        if guess:
            bt.set_mlp(net)
            bt.set_options(guess=1, learned_gate=gate)
        bt.autotune(use_cache=True)
        bt.graph_steps(qsteps)  # warm-up, captures the graph
        bt.set_states(grids)
        ms = _timed_steps(bt, qsteps, graph=True)
        qfinal[name] = bt.get_states()
        bt.set_options(stats=1)
        bt.stats(reset=True)
        bt.step(1)
        qres[name] = {"ms_per_step": ms, "cell_updates_per_s": 2 * cells / (ms * 1e-3),
                      "newton": _iter_stats(bt)}
        bt.close()
        del bt
        torch.cuda.empty_cache()
    for name in ("f32_two_rarefaction", "f32_learned", "f32_learned_everywhere"):
        num = sum(np.abs(x.astype(np.float64)[0] - y[0]).sum()
                  for x, y in zip(qfinal[name], qfinal["plain_f64"]))
        den = sum(np.abs(y[0]).sum() for y in qfinal["plain_f64"])
        qres[name]["rel_l1_density_vs_plain_f64"] = float(num / den)
        qres[name]["speedup_vs_plain_f64"] = (qres["plain_f64"]["ms_per_step"] /
                                              qres[name]["ms_per_step"])
    qres["cells"] = cells
    qres["steps"] = qsteps
    out["quadrant_batch_64"] = qres

    # --- strong jumps: a network trained on logs of such grids, first step of a fresh grid
    for fname, fam in STRONG_FAMILIES.items():
        print(f"# {fname}", file=sys.stderr, flush=True)
        out[fname] = strong_jump_study(fam)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=0,
                    help="grid side (default: 8192 fourier_blasts and fourier_smooth, 4096 shear_layer, "
                         "128 blast_corner)")
    ap.add_argument("--workload", default="fourier_blasts",
                    choices=["fourier_blasts", "fourier_smooth", "shear_layer", "blast_corner",
                             "strong_jumps", "multiblast_batch", "quadrant_batch", "learned",
                             "learned_strong"])
    ap.add_argument("--train-records", type=int, default=10_000_000)
    ap.add_argument("--train-epochs", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32 variant")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--limiter", choices=sorted(LIMITERS), default="minmod",
                    help="slope limiter of the reconstruction")
    ap.add_argument("--order", choices=sorted(ORDERS), default="xy",
                    help="sweep order: x then y every step, or alternating xy / yx")
    ap.add_argument("--riemann", choices=sorted(SOLVERS), default="two_shock",
                    help="interface solver")
    ap.add_argument("--scalars", type=int, choices=[0, 1], default=0,
                    help="passive scalars carried (a smooth seeded field)")
    ap.add_argument("--ysweep", choices=sorted(YSWEEPS), default="march",
                    help="form of the y-sweep kernel: column march (default) or LDS tiles")
    ap.add_argument("--seg-x", type=int, default=0)
    ap.add_argument("--seg-y", type=int, default=0)
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="also run a plain device copy of the state (counter calibration)")
    args = ap.parse_args()
    args.steps_given = "--steps" in sys.argv
    args.dtype_given = "--dtype" in sys.argv

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the sweep runs on a single MI355X "
              "(multi-GPU slab decomposition is not implemented); run with --gpus 1",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.workload == "learned":
        print(json.dumps(bench_learned(args)), flush=True)
        return 0
    if args.workload == "learned_strong":
        # the strong-jump part of the learned-guess study alone (p over 4 decades)
        print(json.dumps({"strong_jumps_p4": strong_jump_study(
            STRONG_FAMILIES["strong_jumps_p4"], n=args.size or 4096)}), flush=True)
        return 0

    if args.workload == "strong_jumps":
        print(json.dumps(bench_strong(args)), flush=True)
        return 0

    if args.workload in BATCH_WORKLOADS:
        if args.dtype == "f64" and not args.dtype_given:
            args.dtype = "f32"
        print(json.dumps(bench_batch(args)), flush=True)
        return 0

    if not args.size:
        args.size = {"fourier_blasts": 8192, "fourier_smooth": 8192, "shear_layer": 4096,
                     "blast_corner": 128}.get(
            args.workload, 8192)
    if args.workload == "blast_corner" and not args.steps_given:
        args.steps = 100  # the point-explosion configuration's run length
    print(f"# generating {args.workload} {args.size}^2", file=sys.stderr, flush=True)
    U, bc, desc = workload(args.workload, args.size)
    _, ny, nx = U.shape
    cells = nx * ny
    if args.scalars:
        from paper_2106_13465_amd import inputs

        U = inputs.with_scalars(U, inputs.random_scalars(nx, ny, seed=7, k=args.scalars))
        desc += f"; {args.scalars} passive scalar (seeded smooth field plus noise)"
    nv = U.shape[0]

    variants = [args.dtype] + ([] if args.no_f32 or args.dtype == "f32" else ["f32"])
    results = {}
    states = {}
    for dn in variants:
        print(f"# gpu {dn}: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
              flush=True)
        h, r = run_gpu(U, bc, dn, args.steps, args.warmup, args.seg_x, args.seg_y,
                       not args.no_autotune, LIMITERS[args.limiter], ORDERS[args.order],
                       SOLVERS[args.riemann], YSWEEPS[args.ysweep])
        elem = 8 if dn == "f64" else 4
        ms_step = r["ms_total"] / args.steps
        sx = sweep_record(cells, elem, r["profile"]["sweep_x"], nv)
        sy = sweep_record(cells, elem, r["profile"]["sweep_y"], nv)
        results[dn] = {
            "value": 2.0 * cells * args.steps / (r["ms_total"] * 1e-3),
            "ms_per_step": ms_step,
            "sweeps": {"x": sx, "y": sy},
            "dt_phase_avg_ms": r["profile"]["dt"]["ms"] / max(r["profile"]["dt"]["launches"], 1),
            "sim_time": r["t"],
            "launch_shape": r["tune"],
        }
        states[dn] = h.get_state()
        results[dn]["newton"] = newton_report(h)
        if args.copy_calibrate:
            src = h.U.clone()
            torch.cuda.synchronize()
            for _ in range(3):
                h.U.copy_(src)
            torch.cuda.synchronize()
            del src
        h.close()
        del h
        torch.cuda.empty_cache()

    main_dn = variants[0]
    res = results[main_dn]
    sx, sy = res["sweeps"]["x"], res["sweeps"]["y"]
    dom_name, dom = ("sweep_x", sx) if sx["avg_ms"] >= sy["avg_ms"] else ("sweep_y", sy)
    # the counter summaries are taken with the default limiter, order and solver
    default_opts = (args.limiter == "minmod" and args.order == "xy" and args.riemann == "two_shock"
                    and args.scalars == 0 and args.ysweep == "march")
    traffic = pmc_traffic(args.workload, dom_name, main_dn) if default_opts else None
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": dom["hbm_gbps"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["hbm_gbps"] / HBM_PEAK_GBS,
                "traffic": traffic, "algorithmic_bytes_per_launch": dom["algorithmic_bytes"],
                "avg_launch_ms": dom["avg_ms"],
                "valu_issue": valu_issue(args.workload, dom_name, main_dn, dom["avg_ms"])
                if default_opts else None}
    with_copy(roofline)

    line = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_dn,
        "data": "synthetic",
        "config": {"workload": desc, "nx": nx, "ny": ny, "bc": bc, "gamma": 1.4, "cfl": 0.8,
                   "limiter": args.limiter, "sweep_order": args.order,
                   "riemann": args.riemann, "passive_scalars": args.scalars,
                   "ysweep": args.ysweep,
                   "newton_cap": 10, "newton_tol": 1e-8,
                   "parallelism": "single GPU"},
        "sweeps": res["sweeps"],
        "launch_shape": res["launch_shape"],
        "newton": res["newton"],
        "roofline": roofline,
    }
    if "f32" in results and main_dn != "f32":
        r32 = results["f32"]
        a, b = states["f32"].astype(np.float64), states[main_dn]
        l1 = [float(np.abs(a[k] - b[k]).sum() / max(np.abs(b[k]).sum(), 1e-300)) for k in range(nv)]
        line["f32"] = {"value": r32["value"], "ms_per_step": r32["ms_per_step"],
                       "sweeps": r32["sweeps"], "newton": r32["newton"],
                       "speedup_vs_f64": r32["value"] / res["value"],
                       "rel_l1_vs_f64_after_steps": l1}
    del states
    if not args.no_cpu_baseline:
        opts = (LIMITERS[args.limiter], ORDERS[args.order], SOLVERS[args.riemann])
        ref = []
        if args.workload == "blast_corner":
            # the configuration's own metric: the whole run on the CPU
            print(f"# cpu baseline (oracle, {args.steps} steps)", file=sys.stderr, flush=True)
            line["cpu_baseline"] = c1_cpu(U, bc, args.steps, ref)
            line["cpu_baseline"]["gpu_seconds_whole_run"] = res["ms_per_step"] * args.steps * 1e-3
            nref = args.steps
        else:
            print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline(U, bc, *opts, state_out=ref)
            import oracle

            oracle.step(ref[0], oracle_cfg(bc, *opts, nscalars=nv - 4))
            nref = 2
        # the GPU results against the oracle's from the same input: FP64 parity
        # (max relative error) and the FP32 relative L1 error, whole grid
        print(f"# gpu vs oracle after {nref} steps", file=sys.stderr, flush=True)
        cmp = {}
        for dn in variants:
            got = gpu_steps_from(U, bc, dn, nref, *opts)
            cmp[dn] = compare_to_oracle(got, ref[0])
            del got
        line["vs_oracle"] = {"steps": nref, "cells": "every cell of the grid", **cmp}
        if "f32" in line:
            line["f32"]["rel_l1_vs_oracle"] = cmp["f32"]["rel_l1"]
        del ref
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
