"""Autotuner: per (dtype, supernode-width bucket, |C(K)| bucket), how the
GEMM-1 of a supernode runs on this GPU, written as a tune table that
selinv_opts.tune_cache (SelInv(tune_cache=...)) reads.

Choices per bucket (see csrc/tune.cpp for the file format):
  dense_ydense  X_{C,C} gathered once into a dense buffer; GEMM-1 tiles in the
                dense-loader kernel (two workgroups per CU), each with its
                GEMM-2 share
  dense_fused   dense buffer; GEMM-1 tiles with their GEMM-2 share fused, in
                the general item kernel
  gather        X_{C,C} gathered by the GEMM-1 tiles on the fly (no buffer)
  dense_ydense128  as dense_ydense on 128 x 128 tiles (FP64 only: the tile
                shape is the choice), GEMM-2 in separate items
and, per workload dtype, the shortest part of a split contraction.

Method: coordinate descent on measured time.  Starting from the library
defaults, each bucket that holds supernodes of the workload tries each
choice with the other buckets fixed, keeping the one with the shortest
traversal (median of `reps` timed selinv_run calls, HIP events on the launch
stream); then split_min_k is swept for all buckets at once.  The LDL^T panels
are produced once (device factorization) and normalized in every trial
context; only the plan differs between trials.

    python -m paper_1604_02528_amd.tune --workload C5 --workload C2 \
        --out paper_1604_02528_amd/tune/gfx950_rocm7.2.0.json

The workloads are the seeded synthetic matrices of workloads/ (run from the
repository root).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

S_BUCKETS = (16, 64, 128, 256)
C_BUCKETS = (64, 256, 1024, 4096, 1 << 30)
CHOICES = {
    "dense_ydense": {"dense": 1, "ydense": 1},
    "dense_fused": {"dense": 1, "ydense": 0},
    "gather": {"dense": 0, "ydense": 0},
    "dense_ydense128": {"dense": 1, "ydense": 1, "tile": 128},  # FP64 only
}
FP64_ONLY = {"dense_ydense128"}
SPLITS = (128, 320, 640)


def bucket_of(s, c):
    sb = next(b for b in S_BUCKETS if s <= b)
    cb = next(b for b in C_BUCKETS if c <= b)
    return sb, cb


def table_json(key_arch, key_rocm, dtype, choice_of, split_min_k, extra=None):
    entries = []
    for (sb, cb), ch in sorted(choice_of.items()):
        e = {"arch": key_arch, "rocm": key_rocm, "dtype": dtype, "s_max": sb, "c_max": cb,
             "split_min_k": int(split_min_k), "choice": ch}
        e.update(CHOICES[ch])
        entries.append(e)
    out = {"format": "selinv-tune-1", "entries": entries}
    if extra:
        out.update(extra)
    return out


class Trial:
    """Times selinv_run for one tune table on one workload."""

    def __init__(self, w, relax, reps):
        import torch

        from . import SelInv

        self.w, self.relax, self.reps = w, relax, reps
        self.dt = w.dtype
        S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=self.dt, batch=w.batch, cap=w.cap, relax=relax)
        vals = torch.from_numpy(np.ascontiguousarray(w.values)).to("cuda")
        self.ldlt = S.factor_device(vals)
        S.sync()
        sym = S.symbolic()
        self.s = np.diff(sym["xsuper"])
        self.c = np.diff(sym["rowptr"])
        S.close()
        del vals

    def buckets(self):
        out = {}
        for s, c in zip(self.s, self.c):
            b = bucket_of(int(s), int(c))
            out[b] = out.get(b, 0) + 1
        return out

    def time(self, table, tag):
        import torch

        from . import SelInv, capi

        with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
            json.dump(table, f)
            path = f.name
        try:
            w = self.w
            S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=self.dt, batch=w.batch, cap=w.cap, relax=self.relax,
                       tune_cache=path)
            S._alloc(False)
            st = torch.cuda.current_stream()
            P, X, W = S._bufs["panels"], S._bufs["x"], S._bufs["work"]
            capi.selinv_normalize(S.h, self.ldlt, P, W, None, st.cuda_stream)
            capi.selinv_run(S.h, P, X, W, st.cuda_stream)
            S.sync()
            ts = []
            for _ in range(self.reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                capi.selinv_run(S.h, P, X, W, st.cuda_stream)
                e1.record(st)
                S.sync()
                ts.append(e0.elapsed_time(e1))
            S.close()
            del S
            torch.cuda.empty_cache()
        finally:
            os.unlink(path)
        t = float(np.median(ts))
        print(f"  {tag}: {t:.3f} ms", flush=True)
        return t


def tune_workload(name, relax, reps, key_arch, key_rocm):
    from workloads import config

    w = config(name)
    dtype = "c128" if w.is_complex else "f64"  # table key: Hermitian plans run the complex kernels
    print(f"tuning on {name} ({dtype}, N={w.n}, batch {w.batch})", flush=True)
    tr = Trial(w, relax, reps)
    counts = tr.buckets()
    # the library defaults, written out per bucket: dense from c >= 256 (ydense kernel), else gathered
    choice = {b: ("dense_ydense" if b[1] > 256 else "gather") for b in counts}
    split = 320
    best = tr.time(table_json(key_arch, key_rocm, dtype, choice, split), "defaults")
    base = best
    for b in sorted(counts, key=lambda b: (-b[1], -b[0])):
        if b[1] <= 64:  # single-item / single-wavefront nodes: no GEMM-1 tile to choose
            continue
        for ch in CHOICES:
            if ch == choice[b] or (ch in FP64_ONLY and dtype != "f64"):
                continue
            trial = dict(choice)
            trial[b] = ch
            t = tr.time(table_json(key_arch, key_rocm, dtype, trial, split), f"s<={b[0]} c<={b[1]} ({counts[b]} nodes): {ch}")
            if t < best * 0.995:
                best, choice = t, trial
    for sp in SPLITS:
        if sp == split:
            continue
        t = tr.time(table_json(key_arch, key_rocm, dtype, choice, sp), f"split_min_k {sp}")
        if t < best * 0.995:
            best, split = t, sp
    print(f"{name}: {base:.3f} ms with the defaults -> {best:.3f} ms tuned", flush=True)
    return dtype, choice, split, {"workload": name, "default_ms": base, "tuned_ms": best}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", action="append", default=None, help="C2, C3 or C5 (repeatable)")
    ap.add_argument("--relax", type=float, default=0.05)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    root = os.getcwd()
    if root not in sys.path:
        sys.path.insert(0, root)
    from . import capi

    key = dict(kv.split("=") for kv in capi.selinv_tune_key().split())
    entries, runs = [], []
    seen = set()
    t0 = time.time()
    for name in args.workload or ["C5", "C2"]:
        dtype, choice, split, rec = tune_workload(name, args.relax, args.reps, key["arch"], key["rocm"])
        if dtype in seen:
            print(f"{name}: {dtype} already tuned by an earlier workload; measured only", flush=True)
            runs.append(rec)
            continue
        seen.add(dtype)
        entries += table_json(key["arch"], key["rocm"], dtype, choice, split)["entries"]
        runs.append(rec)
    out = {"format": "selinv-tune-1", "key": capi.selinv_tune_key(),
           "generated_by": "python -m paper_1604_02528_amd.tune " + " ".join(sys.argv[1:]),
           "tuning_runs": runs, "seconds": round(time.time() - t0, 1), "entries": entries}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {args.out} ({len(entries)} entries)", flush=True)


if __name__ == "__main__":
    main()
