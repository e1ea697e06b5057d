"""Benchmark of the dose product d = A x on one MI355X.

Default workload (the headline): the largest single-GPU dose matrix,
256 x 256 x 128 = 8,388,608 voxels x 60,000 spots, ~200 stored entries per
row over all rows (60% of rows empty, 1.68e9 entries), stored in the paper's
format (FP16 values, int32 column indices) and multiplied in the paper's
half/double arithmetic (FP64 spot weights, FP64 products, sums and dose).
One step is one product over the whole matrix with the inputs resident in
HBM.  Prints ONE JSON line.

The same line carries, as variants: on the same matrix the FP32-vector
product in FP16, BF16 and E4M3 values (32- and 16-bit indices), the
SELL-C-sigma products, and the adjoints over spot rows and over voxel slabs;
on one clinical-scale beam (2,097,152 x 25,000) the FP32, 16-bit index,
half/double and Single (FP32 values) products, the adjoint (both layouts), one
plan-optimisation iteration (with either adjoint) and the bias controls (beam
along x, irregular row lengths); the batched robust-scenario product at full size (36 matrices,
4 spot-weight vectors each, one autotuned graph launch); the robust-plan step
(9 scenarios x 4 beams on one dose grid, then the scenario epilogue); and a
small cache-resident matrix.  Besides them: the roofline of the dominant
kernel (with the HBM traffic the committed rocprofv3 record gives while the
kernel code is unchanged), the median and standard deviation of single
launches, a read-only HBM ceiling probe, and the CPU oracle timed on the
host, one thread and all threads.  --robust-step and --scenario-epilogue time
only the robust-plan step or its epilogue; --part times one part alone (for
profiling runs); --quick skips the variants.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "dose SpMV GNNZ/s and % HBM roofline, plain vs batched/adjoint at rel err ≤1e-5"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_spmv_f64_sweep_large_fp16.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2103_09683_amd", "csrc", f)
                  for f in ("spmv_kernels.hip", "dose_internal.h")]


def _code_only(text: str) -> str:
    """C++ source without comments and blank space: what the compiler sees."""
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif text[i] == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(text[i])
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the product kernel's code (comments and spacing excluded): the
    HBM traffic record is valid while it matches."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_launches(fn, steps: int, warmup: int):
    """Mean ms per call of fn over `steps` back-to-back calls on the current
    stream, bracketed by HIP events on that stream (the library launches its
    kernels on torch's current stream)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def launch_stats(fn, steps: int, warmup: int):
    """Median and standard deviation of single calls (an event pair around
    each call on the current stream), beside time_launches' mean."""
    import statistics
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = [a.elapsed_time(b) for a, b in ev]
    return statistics.median(t), statistics.pstdev(t)


def measured_traffic(bytes_per_launch_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def hbm_read_ceiling(torch, dm, gib: float = 4.0) -> float:
    buf = torch.empty(int(gib * 2 ** 30) // 4, dtype=torch.float32, device="cuda")
    buf.fill_(1.0)
    sink = torch.zeros(65536, dtype=torch.float32, device="cuda")
    ms = time_launches(lambda: dm.probe_stream_read(buf, sink), 20, 3)
    gbps = buf.numel() * 4 / (ms * 1e-3) / 1e9
    del buf
    return gbps


def cpu_baseline(spec, rp, cols, vals, x, y_gpu, budget_s: float):
    """The CPU oracle (plain FP64 CSR product over the decoded FP16 values) on
    the same matrix and spot weights, timed on all host threads (rows shared
    among them) and on one thread, each repeated to fill about budget_s / 2
    seconds; also the GPU dose against the oracle's, on every row."""
    import numpy as np

    import oracle
    dec, _ = oracle.decode_matrix("fp16", rp, vals)
    nnz = int(rp[-1])

    def timed(fn):
        t0 = time.perf_counter()
        y = fn(rp, cols, dec, x)
        t1 = time.perf_counter()
        reps = 1
        while (t1 - t0) < budget_s / 2 and reps < 50:
            fn(rp, cols, dec, x)
            reps += 1
            t1 = time.perf_counter()
        return y, (t1 - t0) / reps, reps

    y_ref, sec_all, reps_all = timed(oracle.spmv_parallel)
    _, sec_one, reps_one = timed(oracle.spmv)
    threads = oracle.num_threads()
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    err = oracle.max_rel_err(y_gpu, y_ref)
    return {"value": round(nnz / sec_all / 1e9, 4), "unit": "GNNZ/s", "cores": threads, "kind": "oracle",
            "sample": f"full {spec.name} matrix ({nnz} nnz, FP16 values decoded), FP64 sums: {reps_all} passes "
                      f"with the rows shared among {threads} OpenMP threads, {sec_all:.3f} s per pass; "
                      f"{reps_one} single-thread passes, {sec_one:.3f} s per pass",
            "single_thread_GNNZ_per_s": round(nnz / sec_one / 1e9, 4),
            "host_cpus": os.cpu_count(), "host_cpus_usable": affinity,
            "max_rel_err_gpu_vs_oracle": err}


def bench_headline(torch, dm, dosegen, args):
    """The largest workload in the paper's format and arithmetic: FP16 values,
    int32 indices, FP64 spot weights and dose (dose_spmv_f64).  Returns the
    matrix and its host arrays for the variants on the same matrix."""
    import numpy as np
    spec = dosegen.sweep_large()
    t0 = time.time()
    rp, cols, vals = dosegen.csr(spec)
    log(f"generated {spec.name}: {int(rp[-1])} nnz in {time.time() - t0:.1f}s")
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    t0 = time.time()
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose=not args.quick)
    log(f"created matrix (fp16) in {time.time() - t0:.1f}s: {A.info()}")
    info = A.info()
    nnz = info["nnz"]
    x64 = torch.from_numpy(x_h.astype(np.float64)).cuda()
    y64 = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    ms = time_launches(lambda: A.spmv(x64, y64), args.steps, args.warmup)
    nbytes = dm.byte_model(nnz, spec.n_rows, spec.n_cols, value_bytes=2, index_bytes=4, row_ptr_bytes=4,
                           x_bytes=8, y_bytes=8) + 4
    gnnz = nnz / (ms * 1e-3) / 1e9
    achieved = nbytes / (ms * 1e-3) / 1e9
    log(f"headline half/double: {ms:.4f} ms/step, {gnnz:.1f} GNNZ/s, {achieved:.0f} GB/s algorithmic")
    med, sd = launch_stats(lambda: A.spmv(x64, y64), args.steps, 2)
    out = {
        "metric": METRIC, "value": round(gnnz, 3), "unit": "GNNZ/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded ray-run dose-deposition matrix; the paper's patient matrices are not public)",
        "config": {"workload": spec.name, "n_rows": spec.n_rows, "n_cols": spec.n_cols, "nnz": nnz,
                   "empty_row_frac": float(np.mean(np.diff(rp) == 0)),
                   "value_format": "fp16", "index_format": "i32", "x_y": "f64", "accumulate": "f64",
                   "arithmetic": "half/double (Sec. II-D)",
                   "group_nnz": info["group_nnz"], "n_groups": info["n_groups"],
                   "n_groups_x_in_lds": info["n_groups_windowed"], "n_groups_split": info["n_groups_split"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": measured_traffic(nbytes), "algorithmic_bytes_per_launch": nbytes,
                     "byte_model": "6 nnz + 4 (n_rows + 1) + 8 n_rows + 8 n_cols (the paper's 6 nnz + 12 nr + 8 nc)",
                     "kernel": "k_spmv_f64<fp16, int32> (row groups, x window in LDS)"},
        "ms_per_launch_median": round(med, 5), "ms_per_launch_std": round(sd, 5),
    }
    return out, spec, A, rp, cols, vals, x_h, y64


def bench_same_matrix(torch, dm, spec, A, rp, cols, vals, x_h, args):
    """On the headline matrix: FP32 vectors in FP16 (the stored A), the
    adjoint in FP32 and FP64; then BF16 and E4M3 values (forward and adjoint),
    the adjoint over A^T in voxel slabs (FP16 and E4M3, FP32 and FP64),
    16-bit indices in the three formats (forward), and the FP16 matrix in
    SELL-C-sigma form (sigma 65,536) with run-length and 16-bit indices, one
    and four FP32 vectors and one FP64 vector (half/double)."""
    import numpy as np
    reps = max(20, args.steps)
    x = torch.from_numpy(x_h).cuda()
    v_h = dosegen_signed(spec)
    v = torch.from_numpy(v_h).cuda()
    y = torch.empty(spec.n_rows, dtype=torch.float32, device="cuda")
    g = torch.empty(spec.n_cols, dtype=torch.float32, device="cuda")
    res = {"workload": spec.name}

    def entry(M):
        info = M.info()
        ms = time_launches(lambda: M.spmv(x, y), reps, 3)
        e = {"forward_ms": round(ms, 4), "forward_GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 1),
             "forward_GBps": round(info["spmv_bytes"] / (ms * 1e-3) / 1e9, 1),
             "forward_frac": round(info["spmv_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
             "spmv_bytes": info["spmv_bytes"]}
        if info["has_transpose"]:
            ms_a = time_launches(lambda: M.adjoint(v, g), reps, 3)
            e.update({"adjoint_ms": round(ms_a, 4),
                      "adjoint_GNNZ_per_s": round(info["nnz"] / (ms_a * 1e-3) / 1e9, 1),
                      "adjoint_GBps": round(info["adjoint_bytes"] / (ms_a * 1e-3) / 1e9, 1),
                      "adjoint_frac": round(info["adjoint_bytes"] / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                      "adjoint_bytes": info["adjoint_bytes"],
                      "n_groups_t_x_in_lds": info["n_groups_windowed_t"], "n_groups_t": info["n_groups_t"]})
            if info["slab_voxels"]:
                e["slab_voxels"] = info["slab_voxels"]
        return e

    def slab_entry(fmt, rows_model_bytes):
        # the adjoint over A^T in voxel slabs; frac on its own byte model and
        # on the spot-row model (the paper format's minimum)
        t0 = time.time()
        M = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose="slabs")
        log(f"{spec.name} {fmt} slabs: created in {time.time() - t0:.1f}s")
        e = entry(M)
        e["adjoint_frac_spot_row_model"] = round(rows_model_bytes / (e["adjoint_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
        ms64 = time_launches(lambda: M.adjoint(v64, g64), reps, 3)
        e["adjoint_f64_ms"] = round(ms64, 4)
        e["adjoint_f64_frac"] = round((M.info()["adjoint_bytes"] + 4 * (spec.n_rows + spec.n_cols)) / (ms64 * 1e-3)
                                      / 1e9 / HBM_PEAK_GBPS, 4)
        M.close()
        torch.cuda.empty_cache()
        return e

    res["fp16"] = entry(A)
    v64 = v.double()
    g64 = torch.empty(spec.n_cols, dtype=torch.float64, device="cuda")
    ms = time_launches(lambda: A.adjoint(v64, g64), reps, 3)
    ab = A.info()["adjoint_bytes"] + 4 * (spec.n_rows + spec.n_cols)
    res["fp16"]["adjoint_f64_ms"] = round(ms, 4)
    res["fp16"]["adjoint_f64_frac"] = round(ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    A.close()
    torch.cuda.empty_cache()
    for fmt in ("bf16", "fp8e4m3_rowscale"):
        t0 = time.time()
        M = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, transpose=True)
        log(f"{spec.name} {fmt}: created in {time.time() - t0:.1f}s")
        res[fmt] = entry(M)
        M.close()
        torch.cuda.empty_cache()
    for fmt in ("fp16", "fp8e4m3_rowscale"):
        res[fmt + "_slabs"] = slab_entry(fmt, res[fmt]["adjoint_bytes"])
    for fmt in ("fp16", "bf16", "fp8e4m3_rowscale"):
        M = dm.DoseMatrix(rp, cols, vals, spec.n_cols, fmt, index_format="u16")
        res[fmt + "_u16"] = entry(M)
        M.close()
        torch.cuda.empty_cache()
    X = torch.from_numpy(np.stack([x_h] + [dosegen_weights(spec, r) for r in range(1, 4)], 1)).cuda().contiguous()
    Y = torch.empty(spec.n_rows, 4, dtype=torch.float32, device="cuda")
    x64 = x.double()
    y64 = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    for idx in ("runs", "u16"):
        t0 = time.time()
        S = dm.SellMatrix(rp, cols, vals, spec.n_cols, "fp16", sigma=65536, index_format=idx)
        log(f"{spec.name} SELL {idx}: created in {time.time() - t0:.1f}s")
        info = S.info()
        ms = time_launches(lambda: S.spmv(x, y), reps, 3)
        ms4 = time_launches(lambda: S.spmv(X, Y), max(10, reps // 4), 3)
        ms64 = time_launches(lambda: S.spmv(x64, y64), max(10, reps // 4), 3)
        b4 = info["spmv_bytes"] + 3 * 4 * (spec.n_cols + spec.n_rows)
        b64 = info["spmv_bytes"] + 4 * (spec.n_cols + spec.n_rows)  # 8-byte x and y
        res["fp16_sell_" + idx] = {
            "sigma": 65536, "forward_ms": round(ms, 4), "forward_GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 1),
            "forward_GBps": round(info["spmv_bytes"] / (ms * 1e-3) / 1e9, 1),
            "forward_frac": round(info["spmv_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "spmv_bytes": info["spmv_bytes"], "padding_frac": round(info["stored_slots"] / max(info["nnz"], 1) - 1, 4),
            "four_vectors_ms": round(ms4, 4), "four_vectors_GNNZ_per_s": round(info["nnz"] / (ms4 * 1e-3) / 1e9, 1),
            "four_vectors_frac": round(b4 / (ms4 * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "half_double_ms": round(ms64, 4), "half_double_GNNZ_per_s": round(info["nnz"] / (ms64 * 1e-3) / 1e9, 1),
            "half_double_frac": round(b64 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
        S.close()
        torch.cuda.empty_cache()
    log(f"{spec.name} variants: " + json.dumps(res))
    return res


def dosegen_signed(spec):
    import dosegen
    return dosegen.signed_values(spec.seed, 3, spec.n_rows)


def dosegen_weights(spec, r):
    import dosegen
    return dosegen.spot_weights(spec.seed, r, spec.n_cols)


def bench_clinical(torch, dm, dosegen, args):
    """One clinical-scale beam (2,097,152 x 25,000, 4.2e8 entries): the FP32
    product in the paper's format, its adjoint, one plan-optimisation
    iteration, 16-bit indices, half/double, Single, and the bias controls."""
    import numpy as np
    spec = dosegen.clinical_beam()
    rp, cols, vals = dosegen.csr(spec)
    x_h = dosegen.spot_weights(spec.seed, 0, spec.n_cols)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose=True)
    info = A.info()
    nnz = info["nnz"]
    x = torch.from_numpy(x_h).cuda()
    y = torch.empty(spec.n_rows, dtype=torch.float32, device="cuda")
    ms = time_launches(lambda: A.spmv(x, y), args.steps, args.warmup)
    res = {"workload": spec.name, "nnz": nnz, "ms": round(ms, 5),
           "GNNZ_per_s": round(nnz / (ms * 1e-3) / 1e9, 3),
           "GBps_algorithmic": round(info["spmv_bytes"] / (ms * 1e-3) / 1e9, 1),
           "frac": round(info["spmv_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "x_y_accumulate": "f32", "group_nnz": info["group_nnz"], "n_groups": info["n_groups"],
           "n_groups_x_in_lds": info["n_groups_windowed"]}
    log(f"clinical beam FP32: {ms:.4f} ms/step")
    v = torch.from_numpy(dosegen.signed_values(spec.seed, 1, spec.n_rows)).cuda()
    g = torch.empty(spec.n_cols, dtype=torch.float32, device="cuda")
    ms_a = time_launches(lambda: A.adjoint(v, g), args.steps, args.warmup)
    res["adjoint"] = {"ms": round(ms_a, 5), "GNNZ_per_s": round(nnz / (ms_a * 1e-3) / 1e9, 3),
                      "GBps_algorithmic": round(info["adjoint_bytes"] / (ms_a * 1e-3) / 1e9, 1),
                      "frac": round(info["adjoint_bytes"] / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                      "group_nnz_t": info["group_nnz_t"], "n_groups_t": info["n_groups_t"],
                      "n_groups_t_x_in_lds": info["n_groups_windowed_t"],
                      "n_groups_t_split": info["n_groups_split_t"]}
    p_h, w_h = dosegen.objective_masks(spec.nx, spec.ny, spec.nz)
    p, w = torch.from_numpy(p_h).cuda(), torch.from_numpy(w_h).cuda()
    seed = torch.empty_like(y)
    fbuf = torch.empty(1, dtype=torch.float64, device="cuda")
    nbuf = torch.empty(1, dtype=torch.float64, device="cuda")

    def iteration():
        A.spmv(x, y)
        dm.objective(y, p, w, seed=seed, out=fbuf)
        A.adjoint(seed, g)
        dm.norm2(g, out=nbuf)

    ms_i = time_launches(iteration, max(20, args.steps // 4), args.warmup)
    res["optimisation_iteration"] = {
        "ms": round(ms_i, 5), "what": "dose A x, FP64 objective + FP32 seed, adjoint A^T seed, FP64 norm",
        "GNNZ_per_s_two_products": round(2 * nnz / (ms_i * 1e-3) / 1e9, 3)}
    A.spmv(x, y)
    rows_model = info["adjoint_bytes"]
    A.close()
    torch.cuda.empty_cache()
    # the same with A^T in voxel slabs
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose="slabs")
    info_s = A.info()
    ms_s = time_launches(lambda: A.adjoint(v, g), args.steps, args.warmup)
    v64, g64 = v.double(), torch.empty(spec.n_cols, dtype=torch.float64, device="cuda")
    ms_s64 = time_launches(lambda: A.adjoint(v64, g64), max(20, args.steps // 4), args.warmup)
    ms_si = time_launches(iteration, max(20, args.steps // 4), args.warmup)
    res["adjoint_slabs"] = {
        "ms": round(ms_s, 5), "GNNZ_per_s": round(nnz / (ms_s * 1e-3) / 1e9, 3),
        "GBps_algorithmic": round(info_s["adjoint_bytes"] / (ms_s * 1e-3) / 1e9, 1),
        "frac": round(info_s["adjoint_bytes"] / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "frac_spot_row_model": round(rows_model / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "adjoint_bytes": info_s["adjoint_bytes"], "slab_voxels": info_s["slab_voxels"],
        "group_nnz_t": info_s["group_nnz_t"], "n_groups_t": info_s["n_groups_t"],
        "n_groups_t_x_in_lds": info_s["n_groups_windowed_t"], "f64_ms": round(ms_s64, 5),
        "optimisation_iteration_ms": round(ms_si, 5)}
    log(f"clinical beam adjoint over voxel slabs: {ms_s:.4f} ms, iteration {ms_si:.4f} ms")
    del v, g, seed, v64, g64
    A.close()
    res["u16_indices"] = bench_u16(torch, dm, spec, rp, cols, vals, x, y, args)
    res["half_double"] = bench_f64(torch, dm, spec, rp, cols, vals, x_h, args)
    res["single_fp32_values"] = bench_single(torch, dm, spec, rp, cols, vals, x, y, args)
    res["sell_c_sigma"] = bench_sell(torch, dm, spec, rp, cols, vals, x, y, args)
    res["bias_controls"] = bench_bias_controls(torch, dm, dosegen, spec, x, args)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle CPU work")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--quick", action="store_true", help="time the headline product only")
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="grid-depth scale of the 36-matrix robust batch (1.0 = full size)")
    ap.add_argument("--scenario-scale", type=float, default=0.1,
                    help="grid-depth scale of the robust-plan step (1.0 = 128 x 128 x 64 voxels)")
    ap.add_argument("--probe-copy-gib", type=float, default=0.0,
                    help="only run the copy probe over this many GiB (counter calibration)")
    ap.add_argument("--scenario-epilogue", action="store_true",
                    help="only time the robust-plan epilogue on the full 1,048,576-voxel grid")
    ap.add_argument("--robust-step", action="store_true",
                    help="only time the robust-plan step (9 scenarios x 4 beams, then the epilogue)")
    ap.add_argument("--sell-sigmas", default="16384,65536", help="sigmas of the SELL-C-sigma variants")
    ap.add_argument("--sell-index", default="i32,u16,runs", help="index formats of the SELL-C-sigma variants")
    ap.add_argument("--adjoint-layout", choices=["rows", "slabs"], default="rows",
                    help="A^T of --part adjoint: one row per spot, or voxel slabs")
    ap.add_argument("--adjoint-workload", choices=["clinical", "largest"], default="clinical",
                    help="matrix of --part adjoint: the clinical beam or the largest workload")
    ap.add_argument("--part", choices=["clinical", "adjoint", "batched", "sell"],
                    help="only one part: the clinical-beam variants, the clinical-beam adjoint, the full-size "
                         "batched robust scenarios, or the SELL-C-sigma variants on the clinical beam")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; multi-GPU sharding is a design "
                                   "note (row ranges per GPU, replicated x), not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import dosegen
    import paper_2103_09683_amd as dm

    torch.cuda.set_device(0)
    if args.probe_copy_gib > 0:
        n = int(args.probe_copy_gib * 2 ** 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ms = time_launches(lambda: dm.probe_copy(src, dst), 10, 2)
        print(json.dumps({"probe": "copy", "bytes_each_way": n * 4, "ms": ms,
                          "GBps_read_plus_write": 2 * n * 4 / (ms * 1e-3) / 1e9}))
        return

    if args.scenario_epilogue:
        print(json.dumps({"scenario_epilogue": bench_epilogue_full(torch, dm, args.steps)}))
        return
    if args.robust_step:
        print(json.dumps({"robust_scenarios": bench_scenarios(torch, dm, dosegen, args)}))
        return
    if args.part:
        print(json.dumps({args.part: bench_part(torch, dm, dosegen, args)}))
        return

    out, spec, A, rp, cols, vals, x_h, y64 = bench_headline(torch, dm, dosegen, args)
    y_h = y64.cpu().numpy()
    out["hbm_read_ceiling_GBps"] = round(hbm_read_ceiling(torch, dm), 1)
    out["roofline"]["frac_of_read_ceiling"] = round(out["roofline"]["achieved"] / out["hbm_read_ceiling_GBps"], 4)
    if not args.quick:
        variants = {}
        variants["same_matrix"] = bench_same_matrix(torch, dm, spec, A, rp, cols, vals, x_h, args)
        variants["clinical_beam"] = bench_clinical(torch, dm, dosegen, args)
        variants["batched"] = bench_batched(torch, dm, dosegen, args)
        variants["robust_scenarios"] = bench_scenarios(torch, dm, dosegen, args)
        variants["small_plain"] = bench_small(torch, dm, dosegen)
        out["variants"] = variants
    else:
        A.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, rp, cols, vals, x_h, y_h, args.cpu_budget)
        out["cpu_baseline"]["gpu_over_cpu"] = round(out["value"] / out["cpu_baseline"]["value"], 1)
    print(json.dumps(out))


def bench_part(torch, dm, dosegen, args):
    """One part of the bench alone (for profiling runs)."""
    if args.part == "clinical":
        return bench_clinical(torch, dm, dosegen, args)
    if args.part == "batched":
        return bench_batched(torch, dm, dosegen, args)
    spec = dosegen.sweep_large() if args.part == "adjoint" and args.adjoint_workload == "largest" \
        else dosegen.clinical_beam()
    rp, cols, vals = dosegen.csr(spec)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    if args.part == "sell":
        A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16")
        y = A.spmv(x)
        A.close()
        return bench_sell(torch, dm, spec, rp, cols, vals, x, y, args)
    # the adjoint of the clinical beam (or --adjoint-workload largest), FP16,
    # FP32 vectors, over spot rows or (--adjoint-layout slabs) voxel slabs
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16",
                      transpose="slabs" if args.adjoint_layout == "slabs" else True)
    info = A.info()
    v = torch.from_numpy(dosegen.signed_values(spec.seed, 1, spec.n_rows)).cuda()
    g = torch.empty(spec.n_cols, dtype=torch.float32, device="cuda")
    ms = time_launches(lambda: A.adjoint(v, g), args.steps, args.warmup)
    A.close()
    gbps = info["adjoint_bytes"] / (ms * 1e-3) / 1e9
    return {"workload": spec.name, "ms": round(ms, 5), "GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 3),
            "GBps_algorithmic": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
            "algorithmic_bytes_per_launch": info["adjoint_bytes"], "n_groups_t": info["n_groups_t"],
            "n_groups_t_split": info["n_groups_split_t"], "layout": args.adjoint_layout,
            "slab_voxels": info["slab_voxels"]}


def bench_u16(torch, dm, spec, rp, cols, vals, x, y, args):
    """The same product with 16-bit column indices (4 bytes per entry in
    FP16 instead of 6); its result must equal the 32-bit one bit for bit."""
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", index_format="u16")
    info = A.info()
    y16 = torch.empty_like(y)
    ms = time_launches(lambda: A.spmv(x, y16), args.steps, args.warmup)
    same = bool(torch.equal(y16.view(torch.int32), y.view(torch.int32)))
    A.close()
    gbps = info["spmv_bytes"] / (ms * 1e-3) / 1e9
    log(f"u16 indices: {ms:.4f} ms/step, {gbps:.0f} GB/s algorithmic, bitwise equal: {same}")
    return {"ms": round(ms, 5), "GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 3),
            "GBps_algorithmic": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
            "algorithmic_bytes_per_launch": info["spmv_bytes"], "bitwise_equal_to_i32": same}


def bench_f64(torch, dm, spec, rp, cols, vals, x_h, args):
    """The paper's half/double configuration (Sec. II-D): the same FP16 matrix
    with FP64 spot weights and dose, FP64 products and sums.  Algorithmic bytes
    per product: 6 nnz + 4 (n_rows + 1) + 8 n_rows + 8 n_cols (the paper's
    6 nnz + 12 nr + 8 nc)."""
    import numpy as np
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16")
    info = A.info()
    x64 = torch.from_numpy(x_h.astype(np.float64)).cuda()
    y64 = torch.empty(spec.n_rows, dtype=torch.float64, device="cuda")
    ms = time_launches(lambda: A.spmv(x64, y64), args.steps, args.warmup)
    A.close()
    nbytes = info["nnz"] * 6 + 4 * (spec.n_rows + 1) + 8 * spec.n_cols + 8 * spec.n_rows
    gbps = nbytes / (ms * 1e-3) / 1e9
    log(f"half/double: {ms:.4f} ms/step, {gbps:.0f} GB/s algorithmic")
    return {"ms": round(ms, 5), "GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 3),
            "GBps_algorithmic": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
            "algorithmic_bytes_per_launch": nbytes, "x_y_accumulate": "f64"}


def bench_single(torch, dm, spec, rp, cols, vals, x, y, args):
    """The paper's Single control (Sec. V): FP32 matrix values (8 bytes per
    entry with int32 indices), FP32 spot weights and dose."""
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp32")
    info = A.info()
    y32 = torch.empty_like(y)
    ms = time_launches(lambda: A.spmv(x, y32), args.steps, args.warmup)
    A.close()
    gbps = info["spmv_bytes"] / (ms * 1e-3) / 1e9
    log(f"single (FP32 values): {ms:.4f} ms/step, {gbps:.0f} GB/s algorithmic")
    return {"ms": round(ms, 5), "GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 3),
            "GBps_algorithmic": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
            "algorithmic_bytes_per_launch": info["spmv_bytes"]}


def bench_sell(torch, dm, spec, rp, cols, vals, x, y_csr, args):
    """SELL-C-sigma storage (C = 64; the format the paper names as the next
    to try, Sec. II-C, VII) of the same matrix, FP16 values, int32, 16-bit and
    run-length column indices: GNNZ/s, the fraction of 8 TB/s of the
    algorithmic bytes (every code, index or run and row offset once, x and y
    once) and of the bytes the SELL product streams (padding, per-row position
    records), and the largest relative difference from the CSR dose (both are
    within 1e-5 of the oracle)."""
    res = {}
    for sigma in [int(v) for v in args.sell_sigmas.split(",")]:
        for idx in args.sell_index.split(","):
            S = dm.SellMatrix(rp, cols, vals, spec.n_cols, "fp16", sigma=sigma, index_format=idx)
            info = S.info()
            ys = torch.empty_like(y_csr)
            ms = time_launches(lambda: S.spmv(x, ys), args.steps, args.warmup)
            d = (ys.double() - y_csr.double()).abs()
            rel = float((d / y_csr.double().abs().clamp_min(1e-300)).max())
            S.close()
            gb = info["spmv_bytes"] / (ms * 1e-3) / 1e9
            sb = info["stream_bytes"] / (ms * 1e-3) / 1e9
            log(f"sell sigma {sigma} {idx}: {ms:.4f} ms/step, {gb:.0f} GB/s (CSR model), {sb:.0f} GB/s streamed")
            res[f"sigma{sigma}_{idx}"] = {
                "ms": round(ms, 5), "GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 3),
                "GBps_algorithmic": round(gb, 1), "frac": round(gb / HBM_PEAK_GBPS, 4),
                "GBps_streamed": round(sb, 1), "frac_streamed": round(sb / HBM_PEAK_GBPS, 4),
                "padding_frac": round(info["stored_slots"] / max(info["nnz"], 1) - 1, 4),
                "algorithmic_bytes_per_launch": info["spmv_bytes"], "n_runs": info["n_runs"],
                "n_groups": info["n_groups"], "n_groups_windowed": info["n_groups_windowed"],
                "max_rel_diff_vs_csr": rel}
    return res


def bench_bias_controls(torch, dm, dosegen, spec, x, args):
    """The clinical beam's shape with the beam along x (neighbouring rows no
    longer share spots, so row groups gather x over wider windows) and with the
    paper's irregular row lengths (sigma 1.0, rows up to 16,000 entries)."""
    res = {}
    for var in (dosegen.beam_along_x(spec), dosegen.paper_irregular(spec)):
        rp, cols, vals = dosegen.csr(var)
        A = dm.DoseMatrix(rp, cols, vals, var.n_cols, "fp16")
        info = A.info()
        y = torch.empty(var.n_rows, dtype=torch.float32, device="cuda")
        ms = time_launches(lambda: A.spmv(x, y), args.steps, args.warmup)
        A.close()
        gbps = info["spmv_bytes"] / (ms * 1e-3) / 1e9
        log(f"{var.name}: {ms:.4f} ms/step, {gbps:.0f} GB/s algorithmic")
        res[var.name] = {"ms": round(ms, 5), "nnz": info["nnz"], "GNNZ_per_s": round(info["nnz"] / (ms * 1e-3) / 1e9, 3),
                         "GBps_algorithmic": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
                         "n_groups": info["n_groups"], "n_groups_x_in_lds": info["n_groups_windowed"],
                         "n_groups_split": info["n_groups_split"], "max_row_nnz": int((rp[1:] - rp[:-1]).max())}
        del rp, cols, vals
    return res


BATCH_SELL_SIGMA = 8192


def bench_batched(torch, dm, dosegen, args):
    """The 36 beam x scenario matrices of a robust plan, four spot-weight
    vectors each, in one autotuned CSR plan launch (FP16 and BF16), and the
    FP16 matrices in SELL-C-sigma form (sigma 8,192, run-length indices;
    16-bit ones where a chunk holds too many runs) in one SELL plan launch.
    Sigma 8,192 keeps a chunk's rows near one another, so nearly every
    chunk's four-vector x window fits in LDS (at a quarter of the batch:
    1.38 ms, against 1.54 ms at 16,384, 2.80 ms at 65,536 and 1.67 ms with
    16-bit indices at 16,384).
    Algorithmic bytes: the paper format's 6 bytes per entry and 4 per row
    offset, x and y read / written once (four vectors); the SELL line also
    gives its own format's algorithmic bytes."""
    import numpy as np
    specs = dosegen.robust_batch(args.batch_scale)
    res = {}
    for fmt in ("fp16", "bf16"):
        mats, sells, entries, sentries = [], [], [], []
        nnz_tot = bytes_tot = sell_bytes = 0
        sell_idx = set()
        t0 = time.time()
        for s in specs:
            rp, cols, vals = dosegen.csr(s)
            A = dm.DoseMatrix(rp, cols, vals, s.n_cols, fmt)
            X = torch.from_numpy(np.stack([dosegen.spot_weights(s.seed, 4 * s.matrix_id + r, s.n_cols)
                                           for r in range(4)], 1)).cuda().contiguous()
            Y = torch.empty(s.n_rows, 4, dtype=torch.float32, device="cuda")
            mats.append(A)
            entries.append((A, X, Y))
            inf = A.info()
            nnz_tot += inf["nnz"]
            extra = 4 * (4 * inf["n_cols"] + 4 * inf["n_rows"])
            bytes_tot += inf["nnz"] * 6 + (inf["n_rows"] + 1) * 4 + extra
            if fmt == "fp16":
                try:
                    S = dm.SellMatrix(rp, cols, vals, s.n_cols, fmt, sigma=BATCH_SELL_SIGMA, index_format="runs")
                except dm.DoseError:
                    S = dm.SellMatrix(rp, cols, vals, s.n_cols, fmt, sigma=BATCH_SELL_SIGMA,
                                      index_format="u16" if s.n_cols <= 65536 else "i32")
                sell_idx.add(S.index_format)
                sells.append(S)
                sentries.append((S, X, torch.empty_like(Y)))
                # the format's own bytes for one vector, plus three more of x and y
                sell_bytes += S.info()["spmv_bytes"] + 3 * 4 * (inf["n_cols"] + inf["n_rows"])
            del rp, cols, vals
        log(f"batched {fmt}: 36 matrices, {nnz_tot} nnz, built in {time.time() - t0:.1f}s")
        plan = dm.BatchPlan(entries, autotune=True)
        reps = max(10, args.steps // 10)
        ms = time_launches(plan.launch, reps, 3)
        res[fmt] = {"ms": round(ms, 4), "matrices": len(specs), "n_rhs": 4, "nnz": nnz_tot,
                    "GNNZ_rhs_per_s": round(4 * nnz_tot / (ms * 1e-3) / 1e9, 2),
                    "GNNZ_per_s": round(nnz_tot / (ms * 1e-3) / 1e9, 2),
                    "GBps_algorithmic": round(bytes_tot / (ms * 1e-3) / 1e9, 1),
                    "frac": round(bytes_tot / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                    "batch_scale": args.batch_scale}
        log(f"batched {fmt} CSR: {ms:.4f} ms, {res[fmt]['frac']:.3f} of 8 TB/s")
        plan.close()
        if sells:
            splan = dm.SellBatchPlan(sentries)
            ms_s = time_launches(splan.launch, reps, 3)
            splan.close()
            torch.cuda.synchronize()
            rel = 0.0
            for (_, _, Yc), (_, _, Ys) in zip(entries, sentries):
                d = (Ys.double() - Yc.double()).abs() / Yc.double().abs().clamp_min(1e-300)
                rel = max(rel, float(d.max()) if d.numel() else 0.0)
            res[fmt + "_sell"] = {
                "ms": round(ms_s, 4), "index": "/".join(sorted(sell_idx)), "sigma": BATCH_SELL_SIGMA, "n_rhs": 4,
                "GNNZ_rhs_per_s": round(4 * nnz_tot / (ms_s * 1e-3) / 1e9, 2),
                "GNNZ_per_s": round(nnz_tot / (ms_s * 1e-3) / 1e9, 2),
                "GBps_paper_format_bytes": round(bytes_tot / (ms_s * 1e-3) / 1e9, 1),
                "frac_paper_format_bytes": round(bytes_tot / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "GBps_algorithmic": round(sell_bytes / (ms_s * 1e-3) / 1e9, 1),
                "frac": round(sell_bytes / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                "speedup_vs_csr": round(ms / ms_s, 3), "max_rel_diff_vs_csr": rel}
            log(f"batched {fmt} SELL ({res[fmt + '_sell']['index']}): {ms_s:.4f} ms, "
                f"{ms / ms_s:.2f}x the CSR plan, max rel diff {rel:.2e}")
        for M in mats + sells:
            M.close()
        del entries, sentries
        torch.cuda.empty_cache()
    return res


def bench_scenarios(torch, dm, dosegen, args):
    """The robust-plan step: 9 setup-shift scenarios x 4 beams on one shared
    dose grid (128 x 128 x 64 * scenario_scale voxels), the 36 beam doses in one
    autotuned batched graph launch, then the epilogue (scenario doses, seeds,
    FP64 scenario objectives, worst case and expectation).  Reports the step,
    the epilogue alone and its share; epilogue algorithmic bytes are the beam
    doses read once, p and w read once, scenario doses and seeds written once.
    Also the step with the beam sum done by the products, the step with
    the beam products of one SELL-C-sigma plan launch (run-length indices;
    the largest relative difference of its scenario doses from the CSR
    step's), the gradient half of the iteration (robust seeds, then the 36
    adjoints in one adjoint plan over spot rows or voxel slabs, or issued one
    by one, or with each beam's gradient summed over the scenarios by the
    plan) and one whole iteration (the SELL step and that last plan)."""
    import numpy as np
    n_scen, n_beams = 9, 4
    specs = dosegen.robust_scenarios(args.scenario_scale, n_scen, n_beams)
    n = specs[0].n_rows
    xs = [torch.from_numpy(dosegen.spot_weights(dosegen.SEED0 + 6, b, specs[b].n_cols)).cuda()
          for b in range(n_beams)]
    part = torch.empty(n_scen, n_beams, n, dtype=torch.float32, device="cuda")
    part_s = torch.empty_like(part)
    mats, entries, sells, sentries, slabs, nnz_tot = [], [], [], [], [], 0
    for m, sp in enumerate(specs):
        rp, cols, vals = dosegen.csr(sp)
        A = dm.DoseMatrix(rp, cols, vals, sp.n_cols, "fp16", transpose=True)
        mats.append(A)
        # the gradient's adjoints over A^T in voxel slabs
        slabs.append(dm.DoseMatrix(rp, cols, vals, sp.n_cols, "fp16", transpose="slabs"))
        s, b = divmod(m, n_beams)
        entries.append((A, xs[b], part[s, b]))
        # the same beam products in SELL-C-sigma form (run-length indices)
        try:
            S = dm.SellMatrix(rp, cols, vals, sp.n_cols, "fp16", sigma=BATCH_SELL_SIGMA, index_format="runs")
        except dm.DoseError:
            S = dm.SellMatrix(rp, cols, vals, sp.n_cols, "fp16", sigma=BATCH_SELL_SIGMA, index_format="u16")
        sells.append(S)
        sentries.append((S, xs[b], part_s[s, b]))
        nnz_tot += int(rp[-1])
    g = np.random.default_rng(6)
    p = torch.from_numpy(g.choice([0.0, 20.0, 60.0], size=n).astype(np.float32)).cuda()
    w = torch.from_numpy(g.choice([1.0, 10.0], size=n).astype(np.float32)).cuda()
    prob = torch.full((n_scen,), 1.0 / n_scen, dtype=torch.float64, device="cuda")
    d_out = torch.empty(n_scen, n, dtype=torch.float32, device="cuda")
    seed = torch.empty(n_scen, n, dtype=torch.float32, device="cuda")
    out = torch.empty(n_scen + 3, dtype=torch.float64, device="cuda")
    plan = dm.BatchPlan(entries, autotune=True)

    def epilogue():
        dm.scenario_objective(part, p, w, prob=prob, d_out=d_out, seed=seed, out=out)

    def step():
        plan.launch()
        epilogue()

    reps = max(10, args.steps // 10)
    ms_step = time_launches(step, reps, 3)
    ms_epi = time_launches(epilogue, reps, 3)
    # the beam sum done by the products: one launch per beam (the first
    # storing, the others adding), then the epilogue on the scenario doses
    d_f = torch.empty(n_scen, n, dtype=torch.float32, device="cuda")
    fplan = dm.ScenarioPlan([[mats[s * n_beams + b] for b in range(n_beams)] for s in range(n_scen)],
                            [[xs[b] for b in range(n_beams)] for _ in range(n_scen)], d_f, autotune=True)
    out_f = torch.empty_like(out)

    def step_fused():
        fplan.launch()
        dm.scenario_objective(d_f.view(n_scen, 1, n), p, w, prob=prob, seed=seed, out=out_f)

    ms_fused = time_launches(step_fused, reps, 3)
    step()
    step_fused()
    torch.cuda.synchronize()
    fused_equal = bool(torch.equal(d_f.view(torch.int32), d_out.view(torch.int32))) and \
        bool(torch.equal(out_f.view(torch.int64), out.view(torch.int64)))
    fplan.close()
    # the step with the beam products of one SELL-C-sigma plan launch
    splan = dm.SellBatchPlan(sentries)
    d_s, seed_s, out_s = torch.empty_like(d_out), torch.empty_like(seed), torch.empty_like(out)

    def step_sell():
        splan.launch()
        dm.scenario_objective(part_s, p, w, prob=prob, d_out=d_s, seed=seed_s, out=out_s)

    ms_sell = time_launches(step_sell, reps, 3)
    # the gradient half of a robust iteration: the robust seeds (expected
    # objective), then the adjoint of every scenario's beam matrix with its
    # scenario's seed (A^T over spot rows, or in voxel slabs); with the SELL
    # step, one whole iteration
    wseed = torch.empty_like(seed_s)
    grads = [torch.empty(specs[m].n_cols, dtype=torch.float32, device="cuda") for m in range(len(specs))]
    grads_s = [torch.empty_like(gm) for gm in grads]

    def adjoints(ms_, gs_):
        dm.robust_seed(seed_s, "expected", out=out_s, prob=prob, wseed=wseed)
        for m, M in enumerate(ms_):
            M.adjoint(wseed[m // n_beams], gs_[m])

    # the 36 adjoints in one adjoint plan (one graph), or issued one by one
    aplan_rows = dm.AdjointPlan([(M, wseed[m // n_beams], grads[m]) for m, M in enumerate(mats)])
    aplan_slabs = dm.AdjointPlan([(M, wseed[m // n_beams], grads_s[m]) for m, M in enumerate(slabs)])
    aplan_tuned = dm.AdjointPlan([(M, wseed[m // n_beams], grads_s[m]) for m, M in enumerate(slabs)], autotune=True)
    # each beam's gradient summed over the scenarios by the plan itself
    beam_grads = [torch.empty(specs[b].n_cols, dtype=torch.float32, device="cuda") for b in range(n_beams)]
    aplan_acc = dm.AdjointPlan([(M, wseed[m // n_beams], beam_grads[m % n_beams]) for m, M in enumerate(slabs)],
                               accumulate=True)

    def gradient(ap):
        dm.robust_seed(seed_s, "expected", out=out_s, prob=prob, wseed=wseed)
        ap.launch()

    ms_grad_calls = time_launches(lambda: adjoints(slabs, grads_s), reps, 3)
    ms_grad_rows = time_launches(lambda: gradient(aplan_rows), reps, 3)
    ms_grad_slabs = time_launches(lambda: gradient(aplan_slabs), reps, 3)
    ms_grad_tuned = time_launches(lambda: gradient(aplan_tuned), reps, 3)
    ms_grad_acc = time_launches(lambda: gradient(aplan_acc), reps, 3)

    def iteration_sell_slabs():
        step_sell()
        gradient(aplan_acc)

    ms_iter = time_launches(iteration_sell_slabs, reps, 3)
    torch.cuda.synchronize()
    grad_rel = max(float(((a.double() - b.double()).abs().max() / b.double().abs().max().clamp_min(1e-300)))
                   for a, b in zip(grads_s, grads))
    aplan_rows.close()
    aplan_slabs.close()
    aplan_tuned.close()
    aplan_acc.close()
    step()
    step_sell()
    torch.cuda.synchronize()
    sell_rel = float(((d_s.double() - d_out.double()).abs() / d_out.double().abs().clamp_min(1e-300)).max())
    splan.close()
    for S in sells:
        S.close()
    epi_bytes = 4 * n * (n_scen * n_beams + 2 + 2 * n_scen)
    res = {"ms_step": round(ms_step, 4), "ms_epilogue": round(ms_epi, 4),
           "ms_step_beam_sum_in_products": round(ms_fused, 4), "beam_sum_in_products_bitwise_equal": fused_equal,
           "ms_step_sell_runs": round(ms_sell, 4), "sell_sigma": BATCH_SELL_SIGMA,
           "sell_max_rel_diff_of_scenario_doses": sell_rel,
           "ms_gradient_seeds_and_adjoint_plan_spot_rows": round(ms_grad_rows, 4),
           "ms_gradient_seeds_and_adjoint_plan_slabs": round(ms_grad_slabs, 4),
           "ms_gradient_seeds_and_adjoint_plan_slabs_autotuned": round(ms_grad_tuned, 4),
           "ms_gradient_seeds_and_adjoint_plan_slabs_beam_sums": round(ms_grad_acc, 4),
           "ms_gradient_seeds_and_36_adjoint_calls_slabs": round(ms_grad_calls, 4),
           "gradient_slabs_vs_spot_rows_max_rel_diff": grad_rel,
           "ms_iteration_sell_step_and_slab_gradient_plan_beam_sums": round(ms_iter, 4),
           "epilogue_share": round(ms_epi / ms_step, 4), "scenarios": n_scen, "beams": n_beams,
           "voxels": n, "nnz": nnz_tot, "GNNZ_per_s": round(nnz_tot / (ms_step * 1e-3) / 1e9, 2),
           "epilogue_GBps_algorithmic": round(epi_bytes / (ms_epi * 1e-3) / 1e9, 1),
           "scenario_scale": args.scenario_scale}
    plan.close()
    for A in mats + slabs:
        A.close()
    del entries, sentries, part, part_s, d_out, seed, d_f, d_s, seed_s, wseed, grads, grads_s
    torch.cuda.empty_cache()
    res["epilogue_full_grid"] = bench_epilogue_full(torch, dm, reps)
    return res


def bench_epilogue_full(torch, dm, reps: int):
    """The scenario epilogue alone on the full 128 x 128 x 64 grid: 9 scenarios
    x 4 beams of beam doses uniform in [0, 1), scenario doses and seeds written."""
    import numpy as np
    n_scen, n_beams, n = 9, 4, 128 * 128 * 64
    g = np.random.default_rng(7)
    part = torch.rand(n_scen, n_beams, n, dtype=torch.float32, device="cuda")
    p = torch.from_numpy(g.choice([0.0, 2.0], size=n).astype(np.float32)).cuda()
    w = torch.from_numpy(g.choice([1.0, 10.0], size=n).astype(np.float32)).cuda()
    prob = torch.full((n_scen,), 1.0 / n_scen, dtype=torch.float64, device="cuda")
    d_out = torch.empty(n_scen, n, dtype=torch.float32, device="cuda")
    seed = torch.empty(n_scen, n, dtype=torch.float32, device="cuda")
    out = torch.empty(n_scen + 3, dtype=torch.float64, device="cuda")
    ms = time_launches(lambda: dm.scenario_objective(part, p, w, prob=prob, d_out=d_out, seed=seed, out=out),
                       reps, 3)
    nbytes = 4 * n * (n_scen * n_beams + 2 + 2 * n_scen)
    del part, d_out, seed
    torch.cuda.empty_cache()
    return {"voxels": n, "scenarios": n_scen, "beams": n_beams, "ms": round(ms, 4), "algorithmic_bytes": nbytes,
            "GBps_algorithmic": round(nbytes / (ms * 1e-3) / 1e9, 1),
            "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}


def bench_small(torch, dm, dosegen):
    """The small plain matrix (20,000 x 500, about 40 entries per row; it fits in
    the caches, so this is launch latency, not bandwidth): mean time of 10,000
    back-to-back products, and of the plan-optimisation iteration on it (dose,
    FP64 objective with the target/organ masks, adjoint of the seed, FP64
    gradient norm)."""
    spec = dosegen.small_plain()
    rp, cols, vals = dosegen.csr(spec)
    A = dm.DoseMatrix(rp, cols, vals, spec.n_cols, "fp16", transpose=True)
    x = torch.from_numpy(dosegen.spot_weights(spec.seed, 0, spec.n_cols)).cuda()
    y = torch.empty(spec.n_rows, dtype=torch.float32, device="cuda")
    ms = time_launches(lambda: A.spmv(x, y), 10000, 100)
    p_h, w_h = dosegen.objective_masks(spec.nx, spec.ny, spec.nz)
    p, w = torch.from_numpy(p_h).cuda(), torch.from_numpy(w_h).cuda()
    seed = torch.empty_like(y)
    g = torch.empty(spec.n_cols, dtype=torch.float32, device="cuda")
    fbuf = torch.empty(1, dtype=torch.float64, device="cuda")
    nbuf = torch.empty(1, dtype=torch.float64, device="cuda")

    def iteration():
        A.spmv(x, y)
        dm.objective(y, p, w, seed=seed, out=fbuf)
        A.adjoint(seed, g)
        dm.norm2(g, out=nbuf)

    ms_i = time_launches(iteration, 10000, 100)
    nnz = int(rp[-1])
    A.close()
    return {"workload": spec.name, "nnz": nnz, "launches": 10000, "us_per_product": round(ms * 1e3, 2),
            "GNNZ_per_s": round(nnz / (ms * 1e-3) / 1e9, 2), "us_per_iteration": round(ms_i * 1e3, 2),
            "note": "cache-resident (the matrix is about 5 MB): latency, not an HBM-roofline figure"}


if __name__ == "__main__":
    main()
