"""GPU selected inversion vs the CPU oracle (element by element on the panels)."""

import numpy as np
import pytest
import torch

from tests._ref import maxrel, oracle_sym, oracle_x, workload

CASES = [
    # (name, scale, batch, relax)
    ("C1", None, None, 0.0),
    ("C4s", None, None, 0.0),
    ("C2", 12, None, 0.0),
    ("C2", 12, None, 0.05),
    ("C2", 20, None, 0.05),
    ("C3", 8, 2, 0.05),
    ("C3", 14, 2, 0.05),
    ("C5", 6, 2, 0.05),
]


@pytest.mark.gpu
@pytest.mark.parametrize("split", [0, 64], ids=["split_default", "split_64"])
@pytest.mark.parametrize("dense", [0, 65, -1], ids=["dense_default", "dense_all", "gather_only"])
@pytest.mark.parametrize("sched", ["levels", "persistent"])
@pytest.mark.parametrize("name,scale,batch,relax", CASES)
def test_selinv_matches_oracle(name, scale, batch, relax, sched, dense, split):
    """dense: threshold on |C(K)| for the dense X_{C,C} buffer (0 = library
    default, 65 = every node with more than one row tile, -1 = never); split:
    shortest contraction part of a split GEMM-1 tile (0 = library default,
    64 = split every node that has too few tiles), so the gathered and dense
    operand paths and the split-contraction path are all compared."""
    from paper_1604_02528_amd import SelInv

    w = workload(name, scale, batch)
    print(f"case {name} scale={scale} batch={batch} relax={relax} sched={sched} dense={dense} split={split}",
          flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
               cap=w.cap, relax=relax, sched=sched, watchdog_ms=20000, dense_min_c=dense, split_min_k=split)
    S.factor(w.values)
    S.run()
    S.sync()
    X = S.to_host("x")
    ref = oracle_x(name, scale, batch, relax)
    tol = 1e-9 if w.is_complex else 1e-10
    for l in range(w.batch):
        err = maxrel(X[l], ref[l])
        print(f"  matrix {l}: max-norm rel err {err:.3e}", flush=True)
        assert err <= tol


def _perturbed_values(w, seed):
    """Same pattern, new SPD values: off-diagonal entries scaled by U[0.8, 1]
    keep the weighted Laplacian diagonally dominant."""
    rng = np.random.default_rng(seed)
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    off = w.rowind != cols
    v = w.values.copy()
    v[:, off] *= rng.uniform(0.8, 1.0, size=(w.batch, int(off.sum())))
    return v


@pytest.mark.gpu
@pytest.mark.parametrize("sched", ["levels", "persistent"])
def test_rerun_new_values_and_determinism(sched):
    """A second factor + run on the same context and buffers with new values
    must give the new inverse (no stale data survives a launch), and a repeat
    run must reproduce X bit for bit (the traversal has no data races)."""
    from oracle import factor, selinv, symbolic
    from paper_1604_02528_amd import SelInv

    w = workload("C2", 12, None)
    print(f"rerun case C2 scale=12 relax=0.05 sched={sched}", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=w.batch, cap=w.cap, relax=0.05, sched=sched,
               watchdog_ms=20000)
    S.factor(w.values)
    S.run()
    S.sync()
    assert maxrel(S.to_host("x")[0], oracle_x("C2", 12, None, 0.05)[0]) <= 1e-10
    v2 = _perturbed_values(w, 77)
    S.factor(v2)
    S.run()
    S.sync()
    X1 = S.to_host("x")
    sym = oracle_sym("C2", 12, None, 0.05)
    lh, dt = factor.normalize(sym, factor.factor(sym, v2[0]))
    ref = selinv.flatten(sym, selinv.alg1(sym, lh, dt))
    err = maxrel(X1[0], ref)
    print(f"  new values: max-norm rel err {err:.3e}", flush=True)
    assert err <= 1e-10
    S.run()
    S.sync()
    assert np.array_equal(S.to_host("x"), X1)


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,batch,relax", [("C2", 20, None, 0.05), ("C3", 14, 2, 0.05)])
def test_normalize_matches_oracle_in_and_out_of_place(name, scale, batch, relax):
    """Alg. 1 steps 1-2 on the GPU: the normalized panels [Dt^{-1}; Lhat]
    match the oracle's, and the in-place path (selinv_factor) gives the same
    bits as selinv_normalize from a separate LDL^T buffer."""
    from oracle import factor, selinv
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale, batch)
    print(f"normalize case {name} scale={scale} batch={batch}", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
               cap=w.cap, relax=relax)
    S.factor(w.values)  # allocates the buffers
    ldlt = torch.from_numpy(S.factor_host(w.values)).to("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    pv = S.panels_view("panels")
    pv.zero_()
    capi.selinv_normalize(S.h, ldlt, S._bufs["panels"], S._bufs["work"], None, stream)
    torch.cuda.synchronize()
    outplace = S.to_host("panels")
    pv.copy_(ldlt)  # the same LDL^T panels, normalized in place
    capi.selinv_normalize(S.h, S._bufs["panels"], S._bufs["panels"], S._bufs["work"], None, stream)
    torch.cuda.synchronize()
    assert np.array_equal(S.to_host("panels"), outplace)
    sym = oracle_sym(name, scale, batch, relax)
    for l in range(w.batch):
        lh, dt = factor.normalize(sym, factor.factor(sym, w.values[l]))
        ref = selinv.flatten(sym, [np.vstack([d, L]) for d, L in zip(dt, lh)])
        err = maxrel(outplace[l], ref)
        print(f"  matrix {l}: max-norm rel err {err:.3e}", flush=True)
        assert err <= (1e-9 if w.is_complex else 1e-10)


@pytest.mark.gpu
@pytest.mark.parametrize("sched", ["levels", "persistent"])
@pytest.mark.parametrize("choice", ["gather", "dense_fused", "dense_ydense", "dense_ydense128"])
@pytest.mark.parametrize("name,scale,batch,relax", [("C2", 20, None, 0.05), ("C3", 14, 2, 0.05), ("C5", 6, 2, 0.05),
                                                    ("C4s", None, None, 0.0), ("C2", 24, None, 0.0)])
def test_every_tuned_variant_matches_oracle(name, scale, batch, relax, choice, sched):
    """Every GEMM-1 variant the autotuner can choose, forced on all
    supernodes by a tune table, against the oracle (the 128 x 128 tile is an
    FP64 choice: complex plans ignore it and keep their 64 x 64 tiles)."""
    from paper_1604_02528_amd import SelInv
    from tests._tune import forced_table, remove

    w = workload(name, scale, batch)
    print(f"tuned variant {choice} case {name} scale={scale} batch={batch} sched={sched}", flush=True)
    path = forced_table(choice, "c128" if w.is_complex else "f64")
    try:
        S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
                   cap=w.cap, relax=relax, sched=sched, tune_cache=path)
        assert S.symbolic()["tuned_nodes"] == S.symbolic()["nsuper"]
        S.factor(w.values)
        S.run()
        S.sync()
        X = S.to_host("x")
        S.close()
    finally:
        remove(path)
    ref = oracle_x(name, scale, batch, relax)
    for l in range(w.batch):
        err = maxrel(X[l], ref[l])
        print(f"  matrix {l}: max-norm rel err {err:.3e}", flush=True)
        assert err <= (1e-9 if w.is_complex else 1e-10)


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,batch,relax", CASES + [("C2", 20, None, 0.0)])
def test_push_schedule_matches_oracle(name, scale, batch, relax):
    """The paper's left-looking form (Alg. 2: per depth the D step, then the
    O / I / ID pushes into the descendants) against the oracle's Alg. 1."""
    from paper_1604_02528_amd import SelInv

    w = workload(name, scale, batch)
    print(f"push case {name} scale={scale} batch={batch} relax={relax}", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
               cap=w.cap, relax=relax, sched="push")
    S.factor(w.values)
    S.run()
    S.sync()
    X = S.to_host("x")
    ref = oracle_x(name, scale, batch, relax)
    for l in range(w.batch):
        err = maxrel(X[l], ref[l])
        print(f"  matrix {l}: max-norm rel err {err:.3e}", flush=True)
        assert err <= (1e-9 if w.is_complex else 1e-10)
    S.run()  # a second traversal starts again from zero
    S.sync()
    assert np.array_equal(S.to_host("x"), X)
    S.close()
