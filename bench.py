"""Benchmark: selected inversion on one MI355X (FP64 GFLOP/s and % of MFMA peak).

Workload (default, the largest 3-D case): a 27-point complex-symmetric
stencil on a 64^3 grid (N = 262,144), 8 shifted matrices A - z_l I in one
batched run, complex128, geometric nested dissection, supernode cap 256 with
chain relaxation 0.05.  --workload C2 / C3 selects the 40^3 FP64 Laplacian or
the 32-shift 30^3 batch instead.

A step is one pass of the hot path on inputs resident in HBM: the
normalization of the LDL^T panels (Alg. 1 steps 1-2) followed by the
root-to-leaves selected inversion (steps 3-4 with the diagonal
symmetrization).  The LDL^T factors are produced once, before timing.
GFLOP/s counts sum_K 2 c^2 s + 2 c s^2 (x4 for complex) over the maximal
(unrelaxed) supernodes, i.e. the algorithmic work of the method.

Output: one JSON line (plus human-readable lines on stderr).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 matrix peak

WORKLOADS = {
    "C2": "C2: 3-D 7-point weighted Laplacian 40^3 (N=64000), weights U[0.5,1.5], shift 0.05, seed 2, "
          "nested dissection, FP64",
    "C3": "C3: 32 shifts H - z_l S of a 3-D 7-point weighted Laplacian 30^3 (N=27000), complex128, seed 3, "
          "nested dissection, one batched launch",
    "C5": "C5: 3-D 27-point complex-symmetric stencil 64^3 (N=262144), 8 shifts, complex128, seed 5, "
          "nested dissection, supernode cap 256",
    "H3": "H3: 16 real shifts H + sigma_l I of a Hermitian 3-D 7-point magnetic Laplacian 30^3 (N=27000), "
          "complex128 Hermitian (conjugate transposes), seed 6, nested dissection, one batched launch",
    "U3": "U3: 4 shifts A + sigma_l I of an unsymmetric 3-D 7-point convection-diffusion operator 30^3 "
          "(N=27000, symmetric pattern), FP64, seed 7, nested dissection, LU form of Alg. 1, one batched launch",
}

TRAFFIC_RECORDS = {
    "C2": os.path.join(ROOT, "profiles", "selinv_C2_levels_hbm_traffic.json"),
    "C5": os.path.join(ROOT, "profiles", "selinv_C5_levels_hbm_traffic.json"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TUNE_TABLE = None  # set in main(): the autotuner's table for this GPU and ROCm version, if committed


def tune_table_path():
    """paper_1604_02528_amd/tune/<arch>_rocm<version>.json for this build's key, or None."""
    from paper_1604_02528_amd import capi

    key = dict(kv.split("=") for kv in capi.selinv_tune_key().split())
    p = os.path.join(ROOT, "paper_1604_02528_amd", "tune", f"{key['arch']}_rocm{key['rocm']}.json")
    return p if os.path.exists(p) else None


KERNEL_SOURCES = [
    "paper_1604_02528_amd/csrc/kernels.hip",
    "paper_1604_02528_amd/csrc/items.hpp",
    "paper_1604_02528_amd/csrc/tile.hpp",
    "paper_1604_02528_amd/csrc/plan.hpp",
    "paper_1604_02528_amd/csrc/scalar.hpp",
]


def source_sha256(files):
    import hashlib

    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def plan_sha256(S):
    """Fingerprint of a context's forward plan: its work items and its level
    launches (kind, size, item type, depth), as the library lists them."""
    import hashlib

    from paper_1604_02528_amd import capi

    h = hashlib.sha256()
    h.update(np.ascontiguousarray(capi.selinv_items(S.h, 0)).tobytes())
    h.update(np.ascontiguousarray(capi.selinv_items(S.h, 2)).tobytes())
    return h.hexdigest()


def measured_traffic(workload, sched, plan_sha):
    """HBM bytes per traversal from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record of this workload (scaled by a 1 GiB copy), or None when
    there is none, or when the kernel sources or the plan (work items and
    launches) differ from those the record was taken on."""
    rec_path = TRAFFIC_RECORDS.get(workload)
    if sched != "levels" or rec_path is None or not os.path.exists(rec_path):
        return None
    rec = json.load(open(rec_path))
    if source_sha256(rec["source_files"]) != rec["source_sha256"] or plan_sha != rec.get("plan_sha256"):
        return None
    return rec["traffic_bytes_per_step"]


def algorithmic_bytes(w, relax):
    """sum_K [c(c+1)/2 + cs + s(s+1)/2] reads + [cs + s^2] writes over the
    supernode partition in use, times the scalar size."""
    from paper_1604_02528_amd import SelInv

    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=w.dtype, batch=1, cap=w.cap,
               relax=relax, device="cpu")
    sym = S.symbolic()
    S.close()
    s = np.diff(sym["xsuper"]).astype(np.float64)
    c = np.diff(sym["rowptr"]).astype(np.float64)
    elems = np.sum(c * (c + 1) / 2 + c * s + s * (s + 1) / 2 + c * s + s * s)
    return float(elems * (16 if w.is_complex else 8) * w.batch)


def timed_steps(S, ldlt, steps, warmup):
    """warmup + steps passes of the step, selinv_normalize_run (normalization
    and traversal on one stream, the deeper nodes' normalization overlapped
    with the top depths' traversal), timed by the wall clock between two
    device synchronizations; then `steps` passes of selinv_normalize and
    selinv_run as separate calls with HIP events around each, for the
    breakdown.  Returns wall seconds of the timed steps and the per-pass
    normalization and traversal times."""
    import torch

    from paper_1604_02528_amd import capi

    stream = torch.cuda.current_stream()
    h = S.h
    P, X, W = S._bufs["panels"], S._bufs["x"], S._bufs["work"]

    def step():
        capi.selinv_normalize_run(h, ldlt, P, X, W, None, stream.cuda_stream)

    def split(ev):
        ev[0].record(stream)
        capi.selinv_normalize(h, ldlt, P, W, None, stream.cuda_stream)
        ev[1].record(stream)
        capi.selinv_run(h, P, X, W, stream.cuda_stream)
        ev[2].record(stream)

    for _ in range(warmup):
        step()
    S.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    S.sync()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        split(evs[k])
    torch.cuda.synchronize()
    S.sync()
    t_norm = np.array([a.elapsed_time(b) for a, b, _ in evs]) * 1e-3
    t_run = np.array([b.elapsed_time(c) for _, b, c in evs]) * 1e-3
    return wall, t_norm, t_run


def factor_on_device(w, relax, sched, batch):
    """LDL^T panels of `batch` matrices on the device, from the library's GPU
    factorization (selinv_factor_device), outside every timed region.  Returns
    the panels and the factorization's wall time (after a warm-up call)."""
    import torch

    from paper_1604_02528_amd import SelInv

    dt = w.dtype
    S1 = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=batch, cap=w.cap, relax=relax, sched=sched,
                adjoint=False)
    vals = torch.from_numpy(np.ascontiguousarray(w.values[:batch])).to("cuda")
    out = S1.factor_device(vals)
    S1.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S1.factor_device(vals, out=out)
    S1.sync()
    torch.cuda.synchronize()
    t_fac = time.perf_counter() - t0
    S1.close()
    del vals
    return out, t_fac


def gpu_leg(w, relax, steps, warmup, sched="levels", batch=None, want_x=False):
    from paper_1604_02528_amd import SelInv

    batch = w.batch if batch is None else batch
    dt = w.dtype
    t0 = time.perf_counter()
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=batch, cap=w.cap, relax=relax, sched=sched,
               tune_cache=TUNE_TABLE, adjoint=False)
    t_an = time.perf_counter() - t0
    ldlt, t_fac = factor_on_device(w, relax, sched, batch)
    S._alloc(False)
    wall, t_norm, t_run = timed_steps(S, ldlt, steps, warmup)
    X = S.to_host("x") if want_x else None
    sym = S.symbolic()
    del ldlt
    return {
        "S": S, "X": X, "sym": sym, "wall": wall, "t_norm": t_norm, "t_run": t_run,
        "t_analyze": t_an, "t_factor": t_fac, "plan_sha256": plan_sha256(S),
    }


def summary(w, g, steps, name):
    sym = g["sym"]
    flops = sym["flops_exact"] * w.batch
    ms_step = g["wall"] / steps * 1e3
    t_run = float(np.mean(g["t_run"]))
    return {
        "workload": WORKLOADS[name], "dtype": "c128" if w.is_complex else "f64", "batch": w.batch,
        "gflops": round(flops / (ms_step * 1e-3) / 1e9, 2),
        "pct_fp64_mfma_peak": round(100.0 * flops / (ms_step * 1e-3) / (PEAK_FP64_TFLOPS * 1e12), 3),
        "ms_per_step": round(ms_step, 4), "s_per_solve": ms_step * 1e-3 / w.batch,
        "selinv_run_ms": round(t_run * 1e3, 4), "normalize_ms": round(float(np.mean(g["t_norm"])) * 1e3, 4),
        "traversal_tflops": round(flops / t_run / 1e12, 4),
        "traversal_frac_of_peak": round(flops / t_run / 1e12 / PEAK_FP64_TFLOPS, 5),
        "flops_per_solve": sym["flops_exact"], "nsuper": sym["nsuper"], "depth": sym["depth"],
        "t_factor_device_s": round(g["t_factor"], 4),
    }


def hermitian_leg(relax, sched):
    """H3: the Hermitian variant (Section 2.3) on 16 shifts in one launch,
    with the same 30^3 grid as C3 (complex-symmetric) for comparison."""
    from workloads import config

    w = config("H3")
    g = gpu_leg(w, relax, 3, 1, sched)
    out = summary(w, g, 3, "H3")
    g["S"].close()
    log(f"H3: {out['gflops']} GFLOP/s, step {out['ms_per_step']} ms, traversal "
        f"{out['traversal_frac_of_peak']:.3f} of the FP64 MFMA peak")
    return out


def lu_leg(relax):
    """U3: the LU form of Alg. 1 (unsymmetric values on a symmetric pattern),
    4 shifts in one launch on the level schedule.  Its traversal does both
    GEMM-1 products (X_{C,K} and X_{K,C}^T) and GEMM-2 per supernode:
    4 c^2 s + 2 c s^2 flops.  The L D U panels come from the host
    factorization (the LU form has no device factorization), uploaded once
    outside the timed region."""
    import torch

    from paper_1604_02528_amd import SelInv
    from workloads import config

    w = config("U3")
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="lu64", batch=w.batch, cap=w.cap, relax=relax,
               sched="levels", adjoint=False)
    t0 = time.perf_counter()
    ldlt = torch.from_numpy(S.factor_host(w.values)).to("cuda")
    t_fac = time.perf_counter() - t0
    S._alloc(False)
    wall, t_norm, t_run = timed_steps(S, ldlt, 3, 1)
    sym = S.symbolic()
    S.close()
    del ldlt
    s = np.diff(sym["xsuper"]).astype(np.float64)
    c = np.diff(sym["rowptr"]).astype(np.float64)
    fl_solve = float(np.sum(4.0 * c * c * s + 2.0 * c * s * s))
    flops = fl_solve * w.batch
    ms_step = wall / 3 * 1e3
    tr = float(np.mean(t_run))
    out = {
        "workload": WORKLOADS["U3"], "dtype": "f64", "batch": w.batch,
        "gflops": round(flops / (ms_step * 1e-3) / 1e9, 2),
        "ms_per_step": round(ms_step, 4), "selinv_run_ms": round(tr * 1e3, 4),
        "normalize_ms": round(float(np.mean(t_norm)) * 1e3, 4),
        "traversal_tflops": round(flops / tr / 1e12, 4),
        "traversal_frac_of_peak": round(flops / tr / 1e12 / PEAK_FP64_TFLOPS, 5),
        "flops_per_solve": fl_solve, "nsuper": sym["nsuper"], "depth": sym["depth"],
        "t_factor_host_s": round(t_fac, 4),
    }
    log(f"U3 (LU form): {out['gflops']} GFLOP/s, step {out['ms_per_step']} ms, traversal "
        f"{out['traversal_frac_of_peak']:.3f} of the FP64 MFMA peak")
    return out


def batched_leg(relax, sched):
    """C3: 32 complex128 shifts in one launch vs 32 single-shift runs."""
    import torch

    from workloads import config

    w = config("C3")
    g = gpu_leg(w, relax, 3, 1, sched)
    out = summary(w, g, 3, "C3")
    g["S"].close()
    del g
    torch.cuda.empty_cache()
    # 32 sequential single-shift solves (normalize + run each), same pattern
    from paper_1604_02528_amd import SelInv

    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128", batch=1, cap=w.cap, relax=relax, sched=sched,
               tune_cache=TUNE_TABLE, adjoint=False)
    ldlt, _ = factor_on_device(w, relax, sched, 1)
    S._alloc(False)
    wall, _, _ = timed_steps(S, ldlt, 3 * w.batch, w.batch)
    S.close()
    seq_ms = wall / 3 * 1e3  # per 32 sequential solves
    out["sequential_ms_per_32_solves"] = round(seq_ms, 4)
    out["batched_vs_sequential_speedup"] = round(seq_ms / out["ms_per_step"], 3)
    log(f"C3: batched {out['ms_per_step']} ms vs 32 sequential {seq_ms:.3f} ms "
        f"(x{out['batched_vs_sequential_speedup']})")
    return out


def host_cpu():
    """CPU model and the number of host cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count()
    return {"model": model, "cores_available": avail, "logical_cpus": os.cpu_count()}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()]))
    except Exception:
        return int(os.cpu_count())


def cpu_leg(w, relax, reps=3):
    """The oracle's Alg. 1 (selected-inversion phase) on the whole matrix 0 of
    the workload, on the host cores (numpy BLAS), median of `reps`."""
    from oracle import factor, selinv, symbolic

    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=relax)
    P = factor.factor(sym, w.values[0])
    lh, dt = factor.normalize(sym, P)
    times = []
    X = None
    for _ in range(reps):
        t0 = time.perf_counter()
        X = selinv.alg1(sym, lh, dt)
        times.append(time.perf_counter() - t0)
    return {"t": float(np.median(times)), "X": selinv.flatten(sym, X), "threads": blas_threads(),
            "flops": sym.flops(w.is_complex)}


_SAMPLE_SYM = {}


def cpu_leg_sample(w, relax, target_flops, one_thread=False):
    """The oracle's Alg. 1 on a bounded sample of the workload: the first M
    supernodes of its loop (root first; they need no other supernode), M the
    smallest count whose work reaches target_flops.  Alg. 1's time depends on
    the shapes only, so the normalized factors of the sample are seeded random
    values of the right shapes (the oracle's factorization of the whole
    matrix would take far longer than the sample).  Returns the rate in
    GFLOP/s of the sample's algorithmic flops."""
    from oracle import selinv, symbolic

    key = (w.name, w.n, relax)
    if key not in _SAMPLE_SYM:
        _SAMPLE_SYM[key] = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=relax)
    sym = _SAMPLE_SYM[key]
    mul = 4.0 if w.is_complex else 1.0
    rng = np.random.default_rng(0)
    lh, dt = [None] * sym.nsuper, [None] * sym.nsuper
    tot, M = 0.0, 0
    for K in reversed(range(sym.nsuper)):
        s_, c_ = sym.width(K), len(sym.rows[K])
        shape_l, shape_d = (c_, s_), (s_, s_)
        if w.is_complex:
            lh[K] = rng.standard_normal(shape_l) + 1j * rng.standard_normal(shape_l)
            dt[K] = rng.standard_normal(shape_d) + 1j * rng.standard_normal(shape_d)
        else:
            lh[K] = rng.standard_normal(shape_l)
            dt[K] = rng.standard_normal(shape_d)
        tot += mul * (2.0 * c_ * c_ * s_ + 2.0 * c_ * s_ * s_)
        M += 1
        if tot >= target_flops:
            break
    if one_thread:
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=1):
            threads = blas_threads()
            t0 = time.perf_counter()
            selinv.alg1(sym, lh, dt, stop_after=M)
            t = time.perf_counter() - t0
    else:
        threads = blas_threads()
        t0 = time.perf_counter()
        selinv.alg1(sym, lh, dt, stop_after=M)
        t = time.perf_counter() - t0
    return {"t": t, "flops": tot, "nodes": M, "nsuper": sym.nsuper, "threads": threads,
            "frac_of_workload": tot / (mul * sym.flops())}


def adjoint_leg(relax):
    """C4: the adjoint (selinv_backward) against the forward pass (normalize +
    run) on the 200 x 200 GMRF, loss = sum_i c_i (Q^{-1})_ii."""
    import torch

    from paper_1604_02528_amd import SelInv, capi
    from workloads import config

    w = config("C4")
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=1, cap=w.cap, relax=relax, sched="levels")
    S.factor(w.values, want_dtilde=True)
    S.run()
    ldlt = torch.from_numpy(S.factor_host(w.values)).to("cuda")
    # dloss/dx on A's pattern: c_i on the diagonal entries, scattered to the panel layout
    gx = np.zeros((1, w.nnz))
    gx[0, np.asarray(w.colptr[:-1])] = np.asarray(w.meta["c"], dtype=np.float64)
    xbar0 = S.scatter(torch.from_numpy(gx).to("cuda"))
    xbar = torch.empty_like(xbar0)
    abar = torch.empty((1, w.nnz), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    fw, bw = [], []
    for it in range(6):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        capi.selinv_normalize(S.h, ldlt, S._bufs["panels"], S._bufs["work"], S.dtilde, stream.cuda_stream)
        capi.selinv_run(S.h, S._bufs["panels"], S._bufs["x"], S._bufs["work"], stream.cuda_stream)
        e[1].record(stream)
        xbar.copy_(xbar0)
        e[2].record(stream)
        capi.selinv_backward(S.h, S._bufs["panels"], S._bufs["x"], S.dtilde, xbar, None, S._bufs["work"], abar,
                             stream.cuda_stream)
        e[3].record(stream)
        torch.cuda.synchronize()
        if it >= 2:
            fw.append(e[0].elapsed_time(e[1]))
            bw.append(e[2].elapsed_time(e[3]))
    S.sync()
    S.close()
    out = {"workload": "C4: 200 x 200 GMRF precision kappa^2 I + weighted 5-point Laplacian (N=40000), FP64, "
                       "loss sum_i c_i (Q^{-1})_ii",
           "forward_ms": round(float(np.median(fw)), 4), "backward_ms": round(float(np.median(bw)), 4)}
    out["backward_vs_forward"] = round(out["backward_ms"] / out["forward_ms"], 3)
    log(f"C4 adjoint: forward {out['forward_ms']} ms, backward {out['backward_ms']} ms "
        f"(x{out['backward_vs_forward']})")
    return out


def c2_leg(relax, sched, steps):
    """C2 (40^3 FP64 Laplacian) as an extra line: timing, and the GPU result
    against the oracle's Alg. 1 on the whole matrix."""
    from workloads import config

    w = config("C2")
    g = gpu_leg(w, relax, steps, 2, sched, want_x=True)
    out = summary(w, g, steps, "C2")
    c = cpu_leg(w, relax)
    out["max_rel_err_vs_oracle"] = float(np.max(np.abs(g["X"][0] - c["X"])) / np.max(np.abs(c["X"])))
    out["cpu_oracle_gflops"] = round(c["flops"] / c["t"] / 1e9, 3)
    out["cpu_oracle_threads"] = c["threads"]
    out["traffic"] = measured_traffic("C2", sched, g["plan_sha256"])
    g["S"].close()
    log(f"C2: {out['gflops']} GFLOP/s, step {out['ms_per_step']} ms, vs oracle {out['max_rel_err_vs_oracle']:.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--relax", type=float, default=0.05)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline legs")
    ap.add_argument("--sched", default="levels", choices=["persistent", "levels", "push"])
    ap.add_argument("--workload", default="C5", choices=["C2", "C3", "C5"])
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with three 1 GiB device-to-device copies (reference for HBM byte counters)")
    ap.add_argument("--no-tune", action="store_true", help="ignore the committed autotuner table")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the C2 line, the C3 batched-vs-sequential and the C4 adjoint-vs-forward legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each GPU would run its own "
              "shifts, or its own etree subtrees below a shared top). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    from workloads import config

    global TUNE_TABLE
    TUNE_TABLE = None if args.no_tune else tune_table_path()
    log(f"tune table: {TUNE_TABLE}")

    w = config(args.workload)
    log(f"workload {args.workload}: N={w.n} nnz(A)={w.nnz} batch={w.batch} relax={args.relax}")
    g = gpu_leg(w, args.relax, args.steps, args.warmup, args.sched,
                want_x=args.workload == "C2" and not args.no_cpu)
    sm = summary(w, g, args.steps, args.workload)
    flops = g["sym"]["flops_exact"] * w.batch
    ms_step = g["wall"] / args.steps * 1e3
    value = flops / (ms_step * 1e-3) / 1e9
    t_run = float(np.mean(g["t_run"]))
    t_norm = float(np.mean(g["t_norm"]))
    achieved = flops / t_run / 1e12
    log(f"analyze {g['t_analyze']:.2f}s device factor {g['t_factor']*1e3:.1f} ms | step {ms_step:.3f} ms "
        f"(normalize {t_norm*1e3:.3f} ms, selinv {t_run*1e3:.3f} ms) | {value:.1f} GFLOP/s")
    X0 = g["X"][0] if g["X"] is not None else None
    plan_sha = g["plan_sha256"]
    g["S"].close()
    del g
    torch.cuda.empty_cache()
    cpu = None
    err = None
    if not args.no_cpu:
        hc = host_cpu()
        if args.workload == "C2":
            c = cpu_leg(w, args.relax)
            err = float(np.max(np.abs(X0 - c["X"])) / np.max(np.abs(c["X"])))
            rate, secs, thr = c["flops"] / c["t"] / 1e9, c["t"], c["threads"]
            sample = ("whole workload: the oracle's Alg. 1 (selected-inversion phase, numpy BLAS) on the C2 "
                      "matrix with the same supernode partition, median of 3, factorization excluded")
            one = cpu_leg_sample(w, args.relax, 5e9, one_thread=True)
        else:
            c = cpu_leg_sample(w, args.relax, 3e12 if args.workload == "C5" else 3e11)
            rate, secs, thr = c["flops"] / c["t"] / 1e9, c["t"], c["threads"]
            sample = (f"the oracle's Alg. 1 (numpy BLAS) on the first {c['nodes']} of {c['nsuper']} supernodes of "
                      f"its root-first loop for one matrix ({100 * c['frac_of_workload']:.1f}% of one matrix's "
                      f"flops, {c['flops']:.3e}), with seeded random normalized factors of the same shapes (the "
                      f"time depends on the shapes only); GFLOP/s of that sample")
            one = cpu_leg_sample(w, args.relax, 6e11 if args.workload == "C5" else 6e10, one_thread=True)
        cpu = {"value": round(rate, 3), "unit": "GFLOP/s", "cores": thr, "kind": "oracle", "sample": sample,
               "seconds": round(secs, 3), "host_cpu": hc["model"], "host_cores_available": hc["cores_available"],
               "one_thread": {"value": round(one["flops"] / one["t"] / 1e9, 3), "cores": one["threads"],
                              "seconds": round(one["t"], 3),
                              "sample": f"first {one['nodes']} supernodes of the root-first loop "
                                        f"({one['flops']:.3e} flops), threadpoolctl limit 1"}}
        log(f"oracle Alg. 1: {rate:.2f} GFLOP/s on {thr} threads ({secs:.2f} s); one thread "
            f"{cpu['one_thread']['value']} GFLOP/s; host {hc['model']} x{hc['cores_available']}")
        if err is not None:
            log(f"GPU vs oracle max-norm rel err {err:.2e}")
    extras = {}
    if not args.no_extras:
        if args.workload != "C2":
            extras["c2"] = c2_leg(args.relax, args.sched, 10)
            torch.cuda.empty_cache()
        extras["batched"] = batched_leg(args.relax, args.sched)
        torch.cuda.empty_cache()
        extras["hermitian"] = hermitian_leg(args.relax, args.sched)
        torch.cuda.empty_cache()
        extras["lu"] = lu_leg(args.relax)
        torch.cuda.empty_cache()
        extras["adjoint"] = adjoint_leg(args.relax)
    wl = WORKLOADS[args.workload]
    if w.batch > 1:
        wl += f"; {w.batch} distinct shifts, each factored on the GPU (selinv_factor_device) before timing"
    out = {
        "metric": "selinv FP64 GFLOP/s (% MFMA peak) + s/solve; batched 32-shift & adjoint vs plain",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if w.is_complex else "f64",
        "data": "synthetic",
        "config": {
            "workload": wl, "batch": w.batch,
            "supernode_cap": w.cap, "relax": args.relax, "schedule": args.sched,
            "tune_table": os.path.relpath(TUNE_TABLE, ROOT) if TUNE_TABLE else None,
            "nsuper": sm["nsuper"], "depth": sm["depth"],
            "flops_per_solve": sm["flops_per_solve"],
        },
        "pct_fp64_mfma_peak": round(100.0 * value / (PEAK_FP64_TFLOPS * 1e3), 3),
        "s_per_solve": ms_step * 1e-3 / w.batch,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 5),
                     "traffic": measured_traffic(args.workload, args.sched, plan_sha),
                     "traffic_unit": "HBM bytes per traversal (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, calibrated "
                                     "on a 1 GiB device copy)",
                     "algorithmic_bytes": algorithmic_bytes(w, args.relax),
                     "kernel": {"levels": "k_ydense (GEMM-1 tiles of nodes with a dense X_{C,C} buffer), "
                                          "k_gather_list (gathers into those buffers), k_gemm2_list (GEMM-2 "
                                          "shares), k_items_list (the other items) and k_tiny / k_tiny64 "
                                          "(single-wavefront small nodes), one launch per etree depth and phase",
                                "persistent": "k_persistent, one launch",
                                "push": "k_push (the O/I/ID tiles of the left-looking form) and k_items_list "
                                        "(the D step), one launch per etree depth and step"}[args.sched],
                     "selinv_run_ms": round(t_run * 1e3, 4),
                     "note": "achieved = algorithmic flops of one traversal (all matrices of the batch) / "
                             "HIP-event time of selinv_run (all of its launches) on the launch stream; a complex "
                             "multiply-add counts 8 real flops (the usual convention), while k_ydense forms "
                             "complex products from three real MFMA chains (3M), so the MFMA counter reads "
                             "fewer executed flops than this count"},
        "normalize_ms": round(t_norm * 1e3, 4),
        "max_rel_err_vs_oracle": err,
        "t_factor_device_s": sm["t_factor_device_s"],
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration: three copies of 1 GiB (read 1 GiB + write 1 GiB each)")


if __name__ == "__main__":
    main()
