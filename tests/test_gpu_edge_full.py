"""GPU selected inversion on degenerate inputs and at the full benchmark sizes.

Edge cases compare every selected entry with a dense inverse (numpy) laid out
in the panel layout through the oracle's symbolic analysis.  The full-size
cases run in the configuration bench.py times (level schedule, relax 0.05,
library defaults): C2 against the oracle's Alg. 1 on the whole matrix; C3
(32 shifts in one launch) by the row identity on every shift and against the
oracle on four shifts; C5 (8 distinct shifts, factored on the GPU), which the
oracle cannot finish in a test, by the row identity on every row of every
shift, the symmetry of every diagonal block, 16 columns of A_l^{-1} per shift
from independent Krylov solves, and two shifts re-run alone.
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


def _row_identity(w, xa):
    """max_i |sum_k A_ik X_ki - 1| for each matrix: X on A's stored lower
    pattern (extract), every term a selected entry (the pattern of A lies in
    the pattern of L).  xa: [batch, nnz] device tensor."""
    n = w.n
    cols = torch.from_numpy(np.repeat(np.arange(n), np.diff(w.colptr))).cuda()
    rows = torch.from_numpy(np.asarray(w.rowind)).cuda()
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).cuda()
    prod = vals * xa
    off = (rows != cols).to(prod.dtype)
    out = []
    for l in range(w.batch):
        acc = torch.zeros(n, dtype=prod.dtype, device="cuda")
        acc.index_add_(0, rows, prod[l])
        acc.index_add_(0, cols, prod[l] * off)
        out.append(float(torch.max(torch.abs(acc - 1.0))))
    return out


@pytest.fixture(scope="module")
def c3_full():
    from paper_1604_02528_amd import SelInv

    w = workload("C3")
    print("full-size case C3 30^3, 32 shifts, one launch (host factorization)", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128", batch=w.batch, cap=w.cap, relax=0.05,
               sched="levels")
    S.factor(w.values)
    S.run()
    S.sync()
    X = S.to_host("x")
    xa = S.extract()
    S.sync()
    S.close()
    return X, xa


@pytest.mark.gpu
def test_c3_full_size_row_identity_every_shift(c3_full):
    """sum_k A_ik X_ki = 1 on every row of all 32 shifts of the batched launch."""
    w = workload("C3")
    errs = _row_identity(w, c3_full[1])
    print(f"  C3 row identity, worst over rows, per shift: max {max(errs):.3e}", flush=True)
    assert max(errs) <= 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("l", [0, 10, 21, 31])
def test_c3_full_size_shifts_vs_oracle(c3_full, l):
    """Four of the 32 shifts, every selected entry, against the oracle."""
    from oracle import factor

    w = workload("C3")
    sym = oracle_sym("C3", None, None, 0.05)
    lh, dt = factor.normalize(sym, factor.factor(sym, w.values[l]))
    ref = selinv.flatten(sym, selinv.alg1(sym, lh, dt))
    err = maxrel(c3_full[0][l], ref)
    print(f"  C3 shift {l}: max-norm rel err {err:.3e}", flush=True)
    assert err <= 1e-9


def _c5_matvec_factory(w, l):
    """y = A_l x for a block of columns x [n, m] (complex), on the GPU: the
    stored lower entries act on both triangles."""
    n = w.n
    cols = torch.from_numpy(np.repeat(np.arange(n), np.diff(w.colptr))).cuda()
    rows = torch.from_numpy(np.asarray(w.rowind)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(w.values[l])).cuda()
    offm = rows != cols
    r_o, c_o, v_o = rows[offm], cols[offm], v[offm]
    diag = torch.zeros(n, dtype=v.dtype, device="cuda")
    diag.index_add_(0, rows[~offm], v[~offm])

    def mv(x):
        y = diag[:, None] * x
        y.index_add_(0, r_o, v_o[:, None] * x[c_o])
        y.index_add_(0, c_o, v_o[:, None] * x[r_o])
        return y

    return mv, diag


def _cocg(mv, diag, b, tol=1e-14, maxit=400):
    """Jacobi-preconditioned conjugate orthogonal CG (COCG) for a complex
    symmetric A (bilinear x^T y, no conjugation), columns independent."""
    x = torch.zeros_like(b)
    r = b.clone()
    z = r / diag[:, None]
    p = z.clone()
    rho = (r * z).sum(0)
    nb = torch.linalg.vector_norm(b, dim=0)
    for it in range(maxit):
        q = mv(p)
        alpha = rho / (p * q).sum(0)
        x += alpha * p
        r -= alpha * q
        if float(torch.max(torch.linalg.vector_norm(r, dim=0) / nb)) < tol:
            break
        z = r / diag[:, None]
        rho_new = (r * z).sum(0)
        p = z + (rho_new / rho) * p
        rho = rho_new
    res = float(torch.max(torch.linalg.vector_norm(mv(x) - b, dim=0) / nb))
    return x, res, it + 1


@pytest.fixture(scope="module")
def c5_full():
    """C5 at 64^3 with its 8 distinct shifts, factored on the GPU, in the
    configuration bench.py times (level schedule, relax 0.05)."""
    from paper_1604_02528_amd import SelInv

    w = workload("C5")
    print("full-size case C5 64^3, 8 distinct shifts (device factorization)", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128", batch=w.batch, cap=w.cap, relax=0.05,
               sched="levels")
    S._alloc(False)
    S.panels_view("x").zero_()
    S.factor(w.values, on_device=True)
    S.run()
    S.sync()
    xa = S.extract()
    S.sync()
    yield w, S, xa
    S.close()
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_c5_full_size_row_identity_every_shift(c5_full):
    w, S, xa = c5_full
    errs = _row_identity(w, xa)
    print(f"  C5 row identity per shift: {' '.join(f'{e:.1e}' for e in errs)}", flush=True)
    assert max(errs) <= 1e-10


@pytest.mark.gpu
def test_c5_full_size_diagonal_blocks_symmetric(c5_full):
    """Every X_KK of every shift equals its (plain) transpose."""
    w, S, xa = c5_full
    sym = S.symbolic()
    s_all = np.diff(sym["xsuper"])
    c_all = np.diff(sym["rowptr"])
    ij, ji = [], []
    for K in range(sym["nsuper"]):
        s, ld, off = int(s_all[K]), int(s_all[K] + c_all[K]), int(sym["panel_off"][K])
        if s < 2:
            continue
        i, j = np.tril_indices(s, -1)
        ij.append(off + j * ld + i)
        ji.append(off + i * ld + j)
    ij = torch.from_numpy(np.concatenate(ij)).cuda()
    ji = torch.from_numpy(np.concatenate(ji)).cuda()
    X = S.panels_view("x")
    for l in range(w.batch):
        d = float(torch.max(torch.abs(X[l][ij] - X[l][ji])))
        assert d == 0.0, (l, d)


@pytest.mark.gpu
def test_c5_full_size_columns_vs_krylov(c5_full):
    """16 columns of A_l^{-1} in every one of the 8 slots from Jacobi-
    preconditioned COCG (relative residual checked below 1e-13), compared
    with the selected entries of those panel columns: the first, the middle
    and the last column of B, the first column of the supernode with the
    largest C(K), and 12 seeded random columns."""
    w, S, xa = c5_full
    sym = S.symbolic()
    n = w.n
    xs, rowptr, rl, poff = sym["xsuper"], sym["rowptr"], sym["rowind_L"], sym["panel_off"]
    c_all = np.diff(rowptr)
    kbig = int(np.argmax(c_all))
    rng = np.random.default_rng(55)
    jbs = [0, n // 2, n - 1, int(xs[kbig])] + [int(j) for j in rng.choice(n, size=12, replace=False)]
    col2super = np.repeat(np.arange(sym["nsuper"]), np.diff(xs))
    perm = torch.from_numpy(np.asarray(w.perm)).cuda()
    X = S.panels_view("x")
    for l in range(w.batch):
        mv, diag = _c5_matvec_factory(w, l)
        b = torch.zeros((n, len(jbs)), dtype=torch.complex128, device="cuda")
        for q, jb in enumerate(jbs):
            b[int(w.perm[jb]), q] = 1.0
        x, res, its = _cocg(mv, diag, b)
        assert res < 1e-13, res
        worst = 0.0
        for q, jb in enumerate(jbs):
            K = int(col2super[jb])
            f, s = int(xs[K]), int(xs[K + 1] - xs[K])
            rows = np.concatenate([np.arange(f, f + s), rl[rowptr[K]:rowptr[K + 1]]])
            ref = x[perm[torch.from_numpy(rows).cuda()], q]
            lo = int(poff[K]) + (jb - f) * len(rows)
            got = X[l][lo: lo + len(rows)]
            err = float(torch.max(torch.abs(got - ref)) / torch.max(torch.abs(ref)))
            worst = max(worst, err)
        print(f"  C5 slot {l}: 16 columns vs COCG ({its} its, residual {res:.1e}): worst rel err {worst:.3e}",
              flush=True)
        assert worst <= 1e-9


@pytest.mark.gpu
@pytest.mark.parametrize("l", [2, 5])
def test_c5_full_size_slot_equals_single_shift_run(c5_full, l):
    """Shift l factored and inverted alone (batch 1) equals slot l of the
    8-shift run to 1e-13 over every selected entry."""
    from paper_1604_02528_amd import SelInv

    w, S, xa = c5_full
    S1 = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128", batch=1, cap=w.cap, relax=0.05, sched="levels")
    S1._alloc(False)
    S1.panels_view("x").zero_()
    S1.factor(w.values[l:l + 1], on_device=True)
    S1.run()
    S1.sync()
    a = S1.panels_view("x")[0]
    b = S.panels_view("x")[l]
    err = float(torch.max(torch.abs(a - b)) / torch.max(torch.abs(b)))
    print(f"  C5 shift {l} alone vs slot {l} of the batch: max-norm rel err {err:.3e}", flush=True)
    assert err <= 1e-13
    S1.close()
    torch.cuda.empty_cache()


@pytest.mark.gpu
@pytest.mark.parametrize("name", EDGE)
def test_edge_cases_push_schedule(name):
    from paper_1604_02528_amd import SelInv

    w = _edge(name)
    print(f"edge case {name} n={w.n} sched=push", flush=True)
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=0.0)
    ref = _dense_panels(sym, np.linalg.inv(selinv.permuted_dense(sym, w.values[0])))
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=1, cap=w.cap,
               relax=0.0, sched="push")
    S.factor(w.values)
    S.run()
    S.sync()
    err = maxrel(S.to_host("x")[0], ref)
    print(f"  max-norm rel err {err:.3e}", flush=True)
    assert err <= (1e-9 if w.is_complex else 1e-10)
    S.close()
