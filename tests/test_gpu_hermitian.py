"""GPU Hermitian variant (dtype h128: conjugate transposes, Section 2.3) against
the oracle's Hermitian route, itself pinned against numpy's dense inverse
(tests/test_oracle_hermitian.py)."""

import numpy as np
import pytest
import torch

from oracle import factor, selinv, symbolic
from tests._ref import maxrel, oracle_sym, oracle_x, workload
from tests.test_oracle_hermitian import dense_original, hermitian_random, selected_from_dense

TOL = 1e-9  # complex128

CASES = [
    # (name, scale, batch, relax)
    ("H3", 6, 2, 0.0),
    ("H3", 10, 2, 0.05),
    ("H3", 14, 2, 0.05),
]


def _ctx(w, relax, **kw):
    from paper_1604_02528_amd import SelInv

    return SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="h128", batch=w.batch, cap=w.cap, relax=relax,
                  watchdog_ms=20000, **kw)


@pytest.mark.gpu
@pytest.mark.parametrize("split", [0, 64], ids=["split_default", "split_64"])
@pytest.mark.parametrize("dense", [0, 65, -1], ids=["dense_default", "dense_all", "gather_only"])
@pytest.mark.parametrize("sched", ["levels", "persistent", "push"])
@pytest.mark.parametrize("name,scale,batch,relax", CASES)
def test_hermitian_matches_oracle(name, scale, batch, relax, sched, dense, split):
    """Every operand path (gathered X_{C,C} with conjugated upper part, dense
    buffer with conjugated mirror, split contractions, GEMM-2 with Lhat^H,
    the Hermitian symmetrization, single-wavefront nodes) on every schedule."""
    if sched == "push" and (dense, split) != (0, 0):
        pytest.skip("the push form has no dense buffers or split contractions")
    w = workload(name, scale, batch)
    print(f"hermitian case {name} scale={scale} batch={batch} relax={relax} sched={sched} dense={dense} "
          f"split={split}", flush=True)
    S = _ctx(w, relax, sched=sched, dense_min_c=dense, split_min_k=split)
    S.factor(w.values)
    S.run()
    S.sync()
    X = S.to_host("x")
    ref = oracle_x(name, scale, batch, relax)
    for l in range(w.batch):
        err = maxrel(X[l], ref[l])
        print(f"  matrix {l}: max-norm rel err {err:.3e}", flush=True)
        assert err <= TOL
    S.close()


@pytest.mark.gpu
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("sched", ["levels", "persistent"])
def test_hermitian_random_patterns_vs_dense_inverse(seed, sched):
    """Random Hermitian patterns (half of them indefinite) under random
    permutations, against numpy's dense inverse, and X on A's own pattern
    (selinv_extract conjugates the entries the permutation moved)."""
    from paper_1604_02528_amd import SelInv

    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(30, 260))
    colptr, rowind, v = hermitian_random(n, float(rng.uniform(0.01, 0.08)), rng, indefinite=bool(seed % 2))
    perm = rng.permutation(n).astype(np.int64)
    cap = int(rng.integers(4, 80))
    print(f"hermitian random case seed={seed} n={n} cap={cap} sched={sched}", flush=True)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=cap)
    S = SelInv(n, colptr, rowind, perm, dtype="h128", batch=1, cap=cap, relax=0.0, sched=sched,
               watchdog_ms=20000)
    S.factor(v[None, :])
    S.run()
    xa = S.extract()
    S.sync()
    A = dense_original(n, colptr, rowind, v)
    Ainv = np.linalg.inv(A)
    ref = selinv.flatten(sym, selected_from_dense(sym, Ainv))
    err = maxrel(S.to_host("x")[0], ref)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    want = Ainv[rowind, cols]
    err_a = float(np.max(np.abs(xa.cpu().numpy()[0] - want)) / np.max(np.abs(want)))
    print(f"  panels {err:.3e}, on A's pattern {err_a:.3e}", flush=True)
    assert err <= TOL and err_a <= TOL
    S.close()


@pytest.mark.gpu
@pytest.mark.parametrize("scale,batch,relax", [(8, 2, 0.0), (14, 3, 0.05)])
def test_hermitian_device_factor_matches_oracle(scale, batch, relax):
    """selinv_factor_device for h128: LDL^H against the oracle's factor, the
    log det (real for these positive definite shifts), and the selected
    inverse from the device factor."""
    w = workload("H3", scale, batch)
    print(f"hermitian device factor case H3 scale={scale} batch={batch} relax={relax}", flush=True)
    sym = oracle_sym("H3", scale, batch, relax)
    S = _ctx(w, relax)
    ldlt = S.factor_device(w.values)
    S.sync()
    P = ldlt.cpu().numpy()[:, S.packed_index()]
    mask = np.concatenate([np.tril(np.ones((sym.width(K) + sym.rows[K].shape[0], sym.width(K)), bool)).reshape(-1, order="F")
                           for K in range(sym.nsuper)])
    ld = S.logdet()
    for l in range(w.batch):
        Pref = factor.factor(sym, w.values[l], herm=True)
        ref = selinv.flatten(sym, Pref)
        err = np.max(np.abs(P[l][mask] - ref[mask])) / np.max(np.abs(ref[mask]))
        print(f"  matrix {l}: LDL^H max-norm rel err {err:.3e}", flush=True)
        assert err <= 1e-13
        assert abs(ld[l].real - np.real(factor.logdet(sym, Pref))) <= 1e-10 * max(1.0, abs(ld[l]))
        assert abs(ld[l].imag) <= 1e-10
    S.factor(w.values, on_device=True)
    S.run()
    S.sync()
    X = S.to_host("x")
    ref = oracle_x("H3", scale, batch, relax)
    for l in range(w.batch):
        assert maxrel(X[l], ref[l]) <= TOL
    S.close()


@pytest.mark.gpu
def test_hermitian_backward_is_unsupported():
    from paper_1604_02528_amd import capi

    w = workload("H3", 6, 1)
    S = _ctx(w, 0.0)
    S.factor(w.values, want_dtilde=True)
    S.run()
    xbar = torch.zeros((1, S.panel_elems), dtype=torch.complex128, device="cuda")
    with pytest.raises(capi.SelinvError) as ei:
        S.backward(xbar)
    assert ei.value.status == 7
    S.close()


def _row_identity_hermitian(w, xa):
    """max_i |sum_k A_ik X_ki - 1| per matrix from the stored lower values of
    A and the selected entries on A's pattern: A_ck = conj(A_kc) and
    X_ck = conj(X_kc) for the mirrored terms.  xa: [batch, nnz] device tensor."""
    n = w.n
    cols = torch.from_numpy(np.repeat(np.arange(n), np.diff(w.colptr))).cuda()
    rows = torch.from_numpy(np.asarray(w.rowind)).cuda()
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    off = (rows != cols).to(vals.dtype)
    out = []
    for l in range(w.batch):
        acc = torch.zeros(n, dtype=vals.dtype, device="cuda")
        acc.index_add_(0, rows, vals[l] * torch.conj(xa[l]) * off + vals[l] * xa[l] * (1 - off))
        acc.index_add_(0, cols, torch.conj(vals[l]) * xa[l] * off)
        out.append(float(torch.max(torch.abs(acc - 1.0))))
    return out


@pytest.fixture(scope="module")
def h3_full():
    w = workload("H3")
    print("full-size case H3 30^3 Hermitian, 16 shifts, device factorization, one launch", flush=True)
    S = _ctx(w, 0.05)
    S.factor(w.values, on_device=True)
    S.run()
    S.sync()
    X = S.to_host("x")
    xa = S.extract()
    S.sync()
    S.close()
    return X, xa


@pytest.mark.gpu
def test_h3_full_size_row_identity_every_shift(h3_full):
    w = workload("H3")
    errs = _row_identity_hermitian(w, h3_full[1])
    print(f"  H3 row identity, worst over rows and shifts: {max(errs):.3e}", flush=True)
    assert max(errs) <= 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("l", [0, 15])
def test_h3_full_size_shifts_vs_oracle(h3_full, l):
    w = workload("H3")
    sym = oracle_sym("H3", None, None, 0.05)
    lh, dt = factor.normalize(sym, factor.factor(sym, w.values[l], herm=True), herm=True)
    ref = selinv.flatten(sym, selinv.alg1(sym, lh, dt, herm=True))
    err = maxrel(h3_full[0][l], ref)
    print(f"  H3 shift {l}: max-norm rel err {err:.3e}", flush=True)
    assert err <= TOL
