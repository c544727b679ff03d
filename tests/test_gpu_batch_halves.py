"""The level schedule runs a batch as two halves, matrices [0, ceil(B/2)) on
the caller's stream and the rest on a second stream of the context, and a
single matrix as its top chain followed by two subtree groups on the two
streams.  Halves and groups touch disjoint data, so X is bit for bit that of
the same plan launched on one stream (a traced run keeps one stream), through
selinv_run and selinv_normalize_run, and matches the oracle."""

import numpy as np
import pytest
import torch

from tests._ref import maxrel, oracle_x, workload

TOL = 1e-10


def _fp64_batch(batch):
    """C2's 10^3 Laplacian with `batch` diagonal shifts (0.1 l added to every
    diagonal entry of matrix l): an FP64 LDL^T batch."""
    w = workload("C2", 10)
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    diag = (np.asarray(w.rowind) == cols).astype(np.float64)
    vals = np.stack([w.values[0] + 0.1 * l * diag for l in range(batch)])
    return w, vals


def _run_three_ways(S, ldlt):
    """X after (a) selinv_normalize + selinv_run (two streams), (b) the same
    run traced (one stream) and (c) selinv_normalize_run (two streams)."""
    from paper_1604_02528_amd import capi

    st = torch.cuda.current_stream().cuda_stream
    P, X, W = S._bufs["panels"], S._bufs["x"], S._bufs["work"]
    out = []
    capi.selinv_normalize(S.h, ldlt, P, W, None, st)
    S.panels_view("x").zero_()
    capi.selinv_run(S.h, P, X, W, st)
    S.sync()
    out.append(S.to_host("x"))
    S.panels_view("x").zero_()
    S.trace_run()
    out.append(S.to_host("x"))
    S.panels_view("x").zero_()
    capi.selinv_normalize_run(S.h, ldlt, P, X, W, None, st)
    S.sync()
    out.append(S.to_host("x"))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,batch", [("C3", 8, 3), ("C3", 8, 2), ("H3", 8, 5), ("U3", 8, 3)])
def test_halves_match_one_stream_and_oracle(name, scale, batch):
    from paper_1604_02528_amd import SelInv

    w = workload(name, scale, batch)
    print(f"batch halves case {name} scale={scale} batch={batch}", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=w.dtype, batch=w.batch, cap=w.cap, relax=0.05, adjoint=False)
    S._alloc(False)
    ldlt = torch.from_numpy(S.factor_host(w.values)).cuda()
    xa, xb, xc = _run_three_ways(S, ldlt)
    assert np.array_equal(xa, xb) and np.array_equal(xa, xc)
    err = maxrel(xa, oracle_x(name, scale, batch, 0.05))
    print(f"  two streams == one stream == normalize_run; vs oracle {err:.3e}", flush=True)
    assert err <= TOL
    S.close()


@pytest.mark.gpu
def test_halves_fp64_batch():
    from oracle import factor, selinv, symbolic
    from paper_1604_02528_amd import SelInv

    w, vals = _fp64_batch(3)
    print("batch halves case FP64 C2 10^3 with 3 diagonal shifts", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="f64", batch=3, cap=w.cap, relax=0.05, adjoint=False)
    S._alloc(False)
    ldlt = torch.from_numpy(S.factor_host(vals)).cuda()
    xa, xb, xc = _run_three_ways(S, ldlt)
    assert np.array_equal(xa, xb) and np.array_equal(xa, xc)
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=0.05)
    for l in range(3):
        lh, dt = factor.normalize(sym, factor.factor(sym, vals[l]))
        ref = selinv.flatten(sym, selinv.alg1(sym, lh, dt))
        err = maxrel(xa[l], ref)
        print(f"  matrix {l}: vs oracle {err:.3e}", flush=True)
        assert err <= TOL
    S.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale", [("C2", 12), ("C2", None), ("C1", None), ("C3", 10), ("H3", 8), ("U3", 10)])
def test_subtree_groups_match_one_stream_and_oracle(name, scale):
    """Single-matrix plans: the ranges of selinv_items(which = 4) tile every
    launch below the top chain, and the two-stream X equals the one-stream X
    bit for bit and the oracle to 1e-10."""
    from paper_1604_02528_amd import SelInv, capi

    b = None if name in ("C1", "C2") else 1  # the oracle cache key of the other single-matrix tests
    w = workload(name, scale, b)
    print(f"subtree groups case {name} scale={scale}", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=w.dtype, batch=1, cap=w.cap, relax=0.05, adjoint=False)
    R = capi.selinv_items(S.h, 4)
    L = capi.selinv_items(S.h, 2)
    assert len(R) > 0 and set(R[:, 0]) == {1, 2}
    assert R[-1, 1] == len(L) - 1  # every launch below the chain has its ranges
    S._alloc(False)
    ldlt = torch.from_numpy(S.factor_host(w.values)).cuda()
    xa, xb, xc = _run_three_ways(S, ldlt)
    assert np.array_equal(xa, xb) and np.array_equal(xa, xc)
    err = maxrel(xa, oracle_x(name, scale, b, 0.05))
    print(f"  {len(R)} group ranges from launch {R[0, 1]}; two streams == one stream; vs oracle {err:.3e}", flush=True)
    assert err <= TOL
    S.close()
