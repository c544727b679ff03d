"""GPU LU form (dtype lu64: Alg. 1 with its U parts, unsymmetric A on a
symmetric pattern) against the oracle's alg1_lu, itself pinned against
numpy's dense inverse (tests/test_oracle_lu.py)."""

import numpy as np
import pytest
import torch

from oracle import selinv, symbolic
from tests._ref import maxrel, oracle_x, workload
from tests.test_oracle_lu import dense_original_lu, selected_from_dense_lu, unsymmetric_random

TOL = 1e-10  # float64

CASES = [
    # (name, scale, batch, relax)
    ("U3", 6, 2, 0.0),
    ("U3", 10, 2, 0.05),
    ("U3", 14, 2, 0.05),
    ("U3", 20, 1, 0.0),
]


def _ctx(w, relax, **kw):
    from paper_1604_02528_amd import SelInv

    return SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="lu64", batch=w.batch, cap=w.cap, relax=relax, **kw)


@pytest.mark.gpu
@pytest.mark.parametrize("dense", [0, 65, -1], ids=["dense_default", "dense_all", "gather_only"])
@pytest.mark.parametrize("name,scale,batch,relax", CASES)
def test_lu_matches_oracle(name, scale, batch, relax, dense):
    """Both panel sets: X_{C,K} from X_{C,C} (upper part from the X^T set),
    gathered on the fly or from the dense buffer, X_{K,C}^T from (X_{C,C})^T
    (the buffer read transposed), X_KK = Dt^{-1} - Uhat X_{C,K} with no
    symmetrization, and its transpose."""
    w = workload(name, scale, batch)
    print(f"lu case {name} scale={scale} batch={batch} relax={relax} dense={dense}", flush=True)
    S = _ctx(w, relax, dense_min_c=dense)
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
def test_lu_random_patterns_vs_dense_inverse(seed):
    """Random unsymmetric values on random symmetric patterns under random
    permutations, against numpy's dense inverse: both panel sets, and both
    triangles of A^{-1} on A's pattern from selinv_extract."""
    from paper_1604_02528_amd import SelInv

    rng = np.random.default_rng(1900 + seed)
    n = int(rng.integers(30, 260))
    colptr, rowind, lo, up = unsymmetric_random(n, float(rng.uniform(0.01, 0.08)), rng)
    perm = rng.permutation(n).astype(np.int64)
    cap = int(rng.integers(4, 80))
    print(f"lu random case seed={seed} n={n} cap={cap}", flush=True)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=cap)
    S = SelInv(n, colptr, rowind, perm, dtype="lu64", batch=1, cap=cap, relax=0.0, dense_min_c=65 if seed % 2 else 0)
    S.factor(np.concatenate([lo, up])[None, :])
    S.run()
    xa = S.extract()
    S.sync()
    A = dense_original_lu(n, colptr, rowind, lo, up)
    Ainv = np.linalg.inv(A)
    RL, RU = selected_from_dense_lu(sym, Ainv)
    ref = np.concatenate([selinv.flatten(sym, RL), selinv.flatten(sym, RU)])
    err = maxrel(S.to_host("x")[0], ref)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    want = np.concatenate([Ainv[rowind, cols], Ainv[cols, rowind]])
    err_a = maxrel(xa.cpu().numpy()[0], want)
    print(f"  panels {err:.3e}, on A's pattern {err_a:.3e}", flush=True)
    assert err <= TOL and err_a <= TOL
    S.close()


@pytest.mark.gpu
def test_lu_normalize_run_matches_normalize_then_run():
    """selinv_normalize_run (the normalization of both panel sets overlapped
    with the traversal's top depths) gives bit for bit the X of
    selinv_normalize then selinv_run on the same L D U panels (the host
    factorization itself sums sibling updates in thread order, so both
    sides start from one copy of it)."""
    from paper_1604_02528_amd import capi

    w = workload("U3", 14, 2)
    S = _ctx(w, 0.05)
    S.factor(w.values)
    ldlt = torch.from_numpy(S.factor_host(w.values)).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    P, X, W = S._bufs["panels"], S._bufs["x"], S._bufs["work"]
    capi.selinv_normalize(S.h, ldlt, P, W, None, stream)
    capi.selinv_run(S.h, P, X, W, stream)
    S.sync()
    X1 = S.to_host("x")
    capi.selinv_normalize_run(S.h, ldlt, P, X, W, None, stream)
    S.sync()
    X2 = S.to_host("x")
    assert np.array_equal(X1, X2)
    assert maxrel(X2, oracle_x("U3", 14, 2, 0.05)) <= TOL
    S.close()


@pytest.mark.gpu
def test_lu_unsupported_paths():
    from paper_1604_02528_amd import capi

    w = workload("U3", 6, 1)
    S = _ctx(w, 0.0)
    with pytest.raises(capi.SelinvError) as ei:
        S.factor(w.values, want_dtilde=True)
    assert ei.value.status == 7
    with pytest.raises(capi.SelinvError) as ei:
        S.factor_device(w.values)
    assert ei.value.status == 7
    S.factor(w.values)
    S.run()
    with pytest.raises(capi.SelinvError) as ei:
        S.scatter(torch.zeros((1, S.nvals), dtype=torch.float64, device="cuda"))
    assert ei.value.status == 7
    S.close()


def _row_identity_lu(w, xa):
    """max_i |sum_k A_ik X_ki - 1| per matrix, from A's lower values and their
    mirrors and the extracted entries of A^{-1} on both triangles of A's
    pattern.  xa: [batch, 2 nnz] device tensor."""
    n, nnz = w.n, w.colptr[-1]
    cols = torch.from_numpy(np.repeat(np.arange(n), np.diff(w.colptr))).cuda()
    rows = torch.from_numpy(np.asarray(w.rowind)).cuda()
    lo = torch.from_numpy(np.ascontiguousarray(w.lower_values)).cuda()
    up = torch.from_numpy(np.ascontiguousarray(w.upper_values)).cuda()
    off = (rows != cols).to(torch.float64)
    out = []
    for l in range(w.batch):
        xl, xu = xa[l, :nnz], xa[l, nnz:]  # X(r, c) and X(c, r) for stored entry (r, c)
        acc = torch.zeros(n, dtype=torch.float64, device="cuda")
        # row r: A(r, c) X(c, r) over the stored (r, c), r >= c
        acc.index_add_(0, rows, lo[l] * xu)
        # row c: A(c, r) X(r, c) over the stored (r, c), r > c
        acc.index_add_(0, cols, up[l] * xl * off)
        out.append(float(torch.max(torch.abs(acc - 1.0))))
    return out


@pytest.fixture(scope="module")
def u3_full():
    w = workload("U3")
    print("full-size case U3 30^3 convection-diffusion, 4 shifts, host L D U, one launch", flush=True)
    S = _ctx(w, 0.05)
    S.factor(w.values)
    S.run()
    S.sync()
    X = S.to_host("x")
    xa = S.extract()
    S.sync()
    S.close()
    return X, xa


@pytest.mark.gpu
def test_u3_full_size_row_identity_every_shift(u3_full):
    w = workload("U3")
    errs = _row_identity_lu(w, u3_full[1])
    print(f"  U3 row identity, worst over rows and shifts: {max(errs):.3e}", flush=True)
    assert max(errs) <= 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("l", [0, 3])
def test_u3_full_size_shifts_vs_oracle(u3_full, l):
    from oracle import factor
    from tests._ref import oracle_sym

    w = workload("U3")
    sym = oracle_sym("U3", None, None, 0.05)
    PL, PU = factor.factor_lu(sym, w.lower_values[l], w.upper_values[l])
    XL, XU = selinv.alg1_lu(sym, *factor.normalize_lu(sym, PL, PU))
    ref = np.concatenate([selinv.flatten(sym, XL), selinv.flatten(sym, XU)])
    err = maxrel(u3_full[0][l], ref)
    print(f"  U3 shift {l}: max-norm rel err {err:.3e}", flush=True)
    assert err <= TOL


def _lu_edge(name, rng):
    """(n, colptr, rowind, lo, up) of a degenerate LU input: A(r, c) for the
    stored lower entries, then their mirrors A(c, r)."""
    from workloads.grids import _lower_csc

    if name == "n1":
        return 1, np.array([0, 1]), np.array([0]), np.array([3.0]), np.array([3.0])
    if name == "diagonal":
        n = 50
        d = rng.uniform(1, 2, n)
        colptr, rowind, _ = _lower_csc(n, np.arange(n), np.arange(n), d[None, :])
        return n, colptr, rowind, d, d.copy()
    if name in ("dense40", "dense300"):  # dense300 is above the supernode cap: two supernodes
        n = 40 if name == "dense40" else 300
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        r, c = np.tril_indices(n)
        colptr, rowind, both = _lower_csc(n, r, c, np.stack([A[r, c], A[c, r]]))
        return n, colptr, rowind, both[0], both[1]
    if name == "arrow":  # every leaf has C(K) = {last column}
        n = 100
        r = np.concatenate([np.arange(n), np.full(n - 1, n - 1)])
        c = np.concatenate([np.arange(n), np.arange(n - 1)])
        lo = np.concatenate([np.full(n, float(n)), rng.uniform(-1, 1, n - 1)])
        up = np.concatenate([np.full(n, float(n)), rng.uniform(-1, 1, n - 1)])
        colptr, rowind, both = _lower_csc(n, r, c, np.stack([lo, up]))
        return n, colptr, rowind, both[0], both[1]
    raise KeyError(name)


@pytest.mark.gpu
@pytest.mark.parametrize("dense", [0, 65], ids=["dense_default", "dense_all"])
@pytest.mark.parametrize("name", ["n1", "diagonal", "dense40", "dense300", "arrow"])
def test_lu_edge_cases_vs_dense_inverse(name, dense):
    """Degenerate LU inputs (one unknown, a diagonal matrix, dense unsymmetric
    matrices below and above the supernode cap, an arrow) against numpy's dense
    inverse, on both panel sets and through selinv_extract."""
    from paper_1604_02528_amd import SelInv

    rng = np.random.default_rng(47)
    n, colptr, rowind, lo, up = _lu_edge(name, rng)
    perm = np.arange(n, dtype=np.int64)
    print(f"lu edge case {name} n={n} dense={dense}", flush=True)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=256, relax=0.0)
    S = SelInv(n, colptr, rowind, perm, dtype="lu64", batch=1, cap=256, relax=0.0, dense_min_c=dense)
    S.factor(np.concatenate([lo, up])[None, :])
    S.run()
    xa = S.extract()
    S.sync()
    A = dense_original_lu(n, colptr, rowind, lo, up)
    Ainv = np.linalg.inv(A)
    RL, RU = selected_from_dense_lu(sym, Ainv)
    err = maxrel(S.to_host("x")[0], np.concatenate([selinv.flatten(sym, RL), selinv.flatten(sym, RU)]))
    cols = np.repeat(np.arange(n), np.diff(colptr))
    err_a = maxrel(xa.cpu().numpy()[0], np.concatenate([Ainv[rowind, cols], Ainv[cols, rowind]]))
    print(f"  panels {err:.3e}, on A's pattern {err_a:.3e}", flush=True)
    assert err <= TOL and err_a <= TOL
    S.close()
