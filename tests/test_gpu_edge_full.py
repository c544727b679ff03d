"""GPU selected inversion on degenerate inputs and at the full benchmark sizes.

Edge cases compare every selected entry with a dense inverse (numpy) laid out
in the panel layout through the oracle's symbolic analysis.  The full-size
cases run in the configuration bench.py times (level schedule, relax 0.05,
library defaults): C2 against the oracle's Alg. 1 on the whole matrix, C3 on
two of its 32 shifts, and C5, which the oracle cannot finish in a test, on
sampled columns of A^{-1} obtained by independent Krylov solves.
"""

import numpy as np
import pytest
import torch

from oracle import selinv, symbolic
from tests._ref import maxrel, oracle_sym, oracle_x, workload
from workloads.grids import Workload, _lower_csc, random_pattern


def _dense_panels(sym, Xd):
    """Selected entries of a dense inverse of B = P A P^T in the panel layout."""
    out = []
    for K in range(sym.nsuper):
        f, l = int(sym.xsuper[K]), int(sym.xsuper[K + 1])
        rows = np.concatenate([np.arange(f, l), sym.rows[K]])
        out.append(Xd[np.ix_(rows, np.arange(f, l))])
    return selinv.flatten(sym, out)


def _spd_dense(n, rng, complex_values=False):
    M = rng.standard_normal((n, n))
    if complex_values:
        M = M + 0.3j * rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    r, c = np.tril_indices(n)
    return _lower_csc(n, r, c, A[r, c][None, :])


def _edge(name):
    rng = np.random.default_rng(31)
    if name == "n1":
        colptr, rowind, vals = np.array([0, 1]), np.array([0]), np.array([[3.0]])
        return Workload(name, 1, colptr, rowind, vals, np.arange(1))
    if name == "diagonal":
        n = 50
        colptr, rowind, vals = _lower_csc(n, np.arange(n), np.arange(n), rng.uniform(1, 2, (1, n)))
        return Workload(name, n, colptr, rowind, vals, np.arange(n))
    if name == "dense40":
        colptr, rowind, vals = _spd_dense(40, rng)
        return Workload(name, 40, colptr, rowind, vals, np.arange(40))
    if name == "dense300":  # above the supernode cap: two supernodes
        colptr, rowind, vals = _spd_dense(300, rng)
        return Workload(name, 300, colptr, rowind, vals, np.arange(300))
    if name == "dense70_c128":
        colptr, rowind, vals = _spd_dense(70, rng, complex_values=True)
        return Workload(name, 70, colptr, rowind, vals, np.arange(70))
    if name == "arrow":  # every leaf has C(K) = {last column}
        n = 100
        r = np.concatenate([np.arange(n), np.full(n - 1, n - 1)])
        c = np.concatenate([np.arange(n), np.arange(n - 1)])
        v = np.concatenate([np.full(n, float(n)), rng.uniform(-1, 1, n - 1)])
        colptr, rowind, vals = _lower_csc(n, r, c, v[None, :])
        return Workload(name, n, colptr, rowind, vals, np.arange(n))
    if name == "random_c128":  # random pattern, random permutation
        n = 400
        colptr, rowind, vals = random_pattern(n, 0.02, rng, complex_values=True)
        return Workload(name, n, colptr, rowind, vals, rng.permutation(n))
    raise KeyError(name)


EDGE = ["n1", "diagonal", "dense40", "dense300", "dense70_c128", "arrow", "random_c128"]


@pytest.mark.gpu
@pytest.mark.parametrize("sched", ["levels", "persistent"])
@pytest.mark.parametrize("name", EDGE)
def test_edge_cases_match_dense_inverse(name, sched):
    from paper_1604_02528_amd import SelInv

    w = _edge(name)
    print(f"edge case {name} n={w.n} sched={sched}", flush=True)
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=0.0)
    ref = _dense_panels(sym, np.linalg.inv(selinv.permuted_dense(sym, w.values[0])))
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=1, cap=w.cap,
               relax=0.0, sched=sched, watchdog_ms=20000)
    S.factor(w.values)
    S.run()
    S.sync()
    err = maxrel(S.to_host("x")[0], ref)
    print(f"  max-norm rel err {err:.3e}", flush=True)
    assert err <= (1e-9 if w.is_complex else 1e-10)
    S.close()


@pytest.mark.gpu
def test_c2_full_size_matches_oracle():
    """C2 at 40^3 in the benchmark configuration, every selected entry."""
    from paper_1604_02528_amd import SelInv

    w = workload("C2")
    print("full-size case C2 40^3 levels relax=0.05", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=1, cap=w.cap, relax=0.05, sched="levels")
    S.factor(w.values)
    S.run()
    S.sync()
    err = maxrel(S.to_host("x")[0], oracle_x("C2", None, None, 0.05)[0])
    print(f"  max-norm rel err {err:.3e}", flush=True)
    assert err <= 1e-10
    S.close()


@pytest.fixture(scope="module")
def c3_full_x():
    from paper_1604_02528_amd import SelInv

    w = workload("C3")
    print("full-size case C3 30^3, 32 shifts, one launch", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128", batch=w.batch, cap=w.cap, relax=0.05,
               sched="levels")
    S.factor(w.values)
    S.run()
    S.sync()
    X = S.to_host("x")
    S.close()
    return X


@pytest.mark.gpu
@pytest.mark.parametrize("l", [0, 31])
def test_c3_full_size_sampled_shifts(c3_full_x, l):
    """Shifts 0 and 31 of the 32-shift launch against the oracle."""
    from oracle import factor

    w = workload("C3")
    sym = oracle_sym("C3", None, None, 0.05)
    lh, dt = factor.normalize(sym, factor.factor(sym, w.values[l]))
    ref = selinv.flatten(sym, selinv.alg1(sym, lh, dt))
    err = maxrel(c3_full_x[l], ref)
    print(f"  C3 shift {l}: max-norm rel err {err:.3e}", flush=True)
    assert err <= 1e-9


@pytest.mark.gpu
def test_c5_full_size_sampled_columns():
    """C5 at 64^3 with 8 batch slots, as bench.py runs it (the LDL^T panels of
    shift 0 copied to every slot).  Columns of A_0^{-1} from GMRES (Jacobi
    preconditioned, relative residual 1e-14) are compared with the selected
    entries of four panel columns (first, middle, the first column of the
    supernode with the largest C(K), root) in slots 0 and 7.
    Tolerance 1e-9: the Krylov solutions of this diagonally dominant system
    are accurate to about 1e-13."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    from paper_1604_02528_amd import SelInv, capi

    w = workload("C5")
    print("full-size case C5 64^3, 8 slots, sampled columns", flush=True)
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=0.05)
    S1 = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128", batch=1, cap=w.cap, relax=0.05)
    one = torch.from_numpy(S1.factor_host(w.values[:1])).to("cuda")
    S1.close()
    ldlt = one.expand(w.batch, -1).contiguous()
    del one
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128", batch=w.batch, cap=w.cap, relax=0.05,
               sched="levels")
    S._alloc(False)
    stream = torch.cuda.current_stream().cuda_stream
    capi.selinv_normalize(S.h, ldlt, S._bufs["panels"], S._bufs["work"], None, stream)
    S.factored = True
    capi.selinv_run(S.h, S._bufs["panels"], S._bufs["x"], S._bufs["work"], stream)
    S.sync()
    X = S.to_host("x")
    S.close()
    del ldlt
    torch.cuda.empty_cache()

    n = w.n
    Lc = sp.csc_matrix((w.values[0], w.rowind, w.colptr), shape=(n, n))
    A = (Lc + Lc.T - sp.diags(Lc.diagonal())).tocsr()
    d = A.diagonal()
    M = spla.LinearOperator((n, n), matvec=lambda v: v / d, dtype=np.complex128)
    starts = np.concatenate([[0], np.cumsum([(sym.width(K) + len(sym.rows[K])) * sym.width(K)
                                             for K in range(sym.nsuper)])])
    kbig = int(np.argmax([len(r) for r in sym.rows]))  # the largest C(K): dense GEMM-1 tiles
    for jb in [0, n // 2, int(sym.xsuper[kbig]), n - 1]:  # columns of B = P A P^T
        K = int(sym.col2super[jb])
        f, s = int(sym.xsuper[K]), sym.width(K)
        rows = np.concatenate([np.arange(f, f + s), sym.rows[K]])
        e = np.zeros(n, dtype=np.complex128)
        e[w.perm[jb]] = 1.0
        x, info = spla.gmres(A, e, M=M, rtol=1e-14, atol=0.0, restart=60, maxiter=50)
        assert info == 0
        ref = x[w.perm[rows]]  # (A^{-1})(perm[r], perm[jb]) = X_B(r, jb)
        lo = starts[K] + (jb - f) * len(rows)
        for l in (0, w.batch - 1):
            got = X[l][lo: lo + len(rows)]
            err = maxrel(got, ref)
            print(f"  column {jb} (supernode {K}, {len(rows)} rows) slot {l}: max-norm rel err {err:.3e}", flush=True)
            assert err <= 1e-9
