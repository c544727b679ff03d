"""Pins of the oracle's factorization and selected inversion.

What fixes the answer (none of it retypes the oracle's formulas):
  * the definition: (P A P^T)^{-1} restricted to the pattern of L (dense inverse);
  * closed-form traces of shifted Dirichlet Laplacians (tests/golden, written by
    tests/golden/make_closed_forms.py from the eigenvalues);
  * the identity sum_k A_ik X_ki = 1, which uses selected entries only because
    the pattern of A lies inside the pattern of L;
  * columns of A^{-1} from scipy's sparse LU (splu);
  * Cholesky of the SPD cases (L D^{1/2} = chol(B));
  * Alg. 1 and Alg. 2 of the paper computing the same selected entries.
"""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import factor, selinv, symbolic
from workloads import config, random_pattern, weighted_laplacian_3d, nested_dissection

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def run_oracle(w, l=0, relax=0.0, cap=256):
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=cap, relax=relax)
    P = factor.factor(sym, w.values[l])
    lh, dt = factor.normalize(sym, P)
    return sym, P, lh, dt


def maxrel(A, B):
    num = max(float(np.max(np.abs(a - b))) if a.size else 0.0 for a, b in zip(A, B))
    den = max(float(np.max(np.abs(b))) if b.size else 0.0 for b in B)
    return num / den


def trace(sym, X):
    return sum(np.trace(X[K][:sym.width(K), :]) for K in range(sym.nsuper))


CASES = [("C1", None, None), ("C4s", None, None), ("C2", 9, None), ("C3", 7, 3), ("C5", 5, 2)]


@pytest.mark.parametrize("relax", [0.0, 0.2])
@pytest.mark.parametrize("name,scale,batch", CASES)
def test_alg1_alg2_equal_dense_inverse(name, scale, batch, relax):
    w = config(name, scale=scale, batch=batch)
    for l in range(w.batch):
        sym, P, lh, dt = run_oracle(w, l, relax=relax, cap=32)
        X1 = selinv.alg1(sym, lh, dt)
        X2 = selinv.alg2(sym, lh, dt)
        Xd = selinv.dense_selected(sym, selinv.permuted_dense(sym, w.values[l]))
        assert maxrel(X1, Xd) < 1e-12
        assert maxrel(X2, X1) < 1e-13
        # diagonal blocks are symmetric (plain transpose, also for complex)
        for K in range(sym.nsuper):
            s = sym.width(K)
            assert np.array_equal(X1[K][:s, :], X1[K][:s, :].T)


@pytest.mark.parametrize("seed", range(12))
def test_random_patterns_vs_dense(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(10, 120))
    cplx = bool(seed % 2)
    colptr, rowind, vals = random_pattern(n, float(rng.uniform(0.02, 0.2)), rng, complex_values=cplx)
    perm = rng.permutation(n).astype(np.int64)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=int(rng.integers(1, 20)), relax=float(rng.choice([0.0, 0.1])))
    P = factor.factor(sym, vals[0])
    lh, dt = factor.normalize(sym, P)
    X1 = selinv.alg1(sym, lh, dt)
    Xd = selinv.dense_selected(sym, selinv.permuted_dense(sym, vals[0]))
    assert maxrel(X1, Xd) < 1e-12
    assert maxrel(selinv.alg2(sym, lh, dt), X1) < 1e-13


def test_c1_closed_form_trace():
    w = config("C1")
    sym, P, lh, dt = run_oracle(w)
    tr = trace(sym, selinv.alg1(sym, lh, dt))
    ref = float(GOLD["C1_2d_m31_sigma0.1"]["trace"])
    assert abs(tr - ref) / ref < 1e-13


@pytest.mark.parametrize("key,m", [("3d_m10_sigma0.05", 10), ("3d_m14_sigma0.05", 14)])
def test_3d_unit_laplacian_closed_form_trace(key, m):
    colptr, rowind, vals = weighted_laplacian_3d((m, m, m), 0.05, None)
    perm = nested_dissection((m, m, m))
    sym = symbolic.analyze(m ** 3, colptr, rowind, perm, relax=0.05)
    P = factor.factor(sym, vals[0])
    lh, dt = factor.normalize(sym, P)
    tr = trace(sym, selinv.alg1(sym, lh, dt))
    ref = float(GOLD[key]["trace"])
    assert abs(tr - ref) / ref < 1e-12


def test_cholesky_pin_spd():
    for name, scale in [("C1", None), ("C2", 8), ("C4s", None)]:
        w = config(name, scale=scale)
        sym, P, lh, dt = run_oracle(w)
        L, D = factor.to_dense_L(sym, P)
        Bd = selinv.permuted_dense(sym, w.values[0])
        Lc = np.linalg.cholesky(Bd)
        assert np.all(D > 0)
        assert np.max(np.abs(L * np.sqrt(D)[None, :] - Lc)) / np.max(np.abs(Lc)) < 1e-12


def test_complex_reconstruction_and_pivot_signs():
    w = config("C3", scale=6, batch=4)
    for l in range(w.batch):
        sym, P, lh, dt = run_oracle(w, l)
        L, D = factor.to_dense_L(sym, P)
        Bd = selinv.permuted_dense(sym, w.values[l])
        assert np.max(np.abs((L * D[None, :]) @ L.T - Bd)) / np.max(np.abs(Bd)) < 1e-13
        # -eta S is negative definite and the Schur complements inherit it
        assert np.all(D.imag < 0)
    w5 = config("C5", scale=5, batch=2)
    for l in range(w5.batch):
        sym, P, lh, dt = run_oracle(w5, l)
        _, D = factor.to_dense_L(sym, P)
        assert np.all(np.abs(D) >= 1.0)


def test_row_identity_on_selected_entries():
    """sum_k A_ik X_ki = 1 for every i (pattern of A inside the pattern of L)."""
    w = config("C2", scale=14)
    sym, P, lh, dt = run_oracle(w, relax=0.05)
    X = selinv.alg1(sym, lh, dt)
    xa = selinv.on_pattern_of_A(sym, X, w.colptr, w.rowind)
    A = sp.csc_matrix((w.values[0], w.rowind, w.colptr), shape=(w.n, w.n))
    Xs = sp.csc_matrix((xa, w.rowind, w.colptr), shape=(w.n, w.n))
    Af = A + sp.tril(A, -1).T
    Xf = Xs + sp.tril(Xs, -1).T
    diag = np.asarray(Af.multiply(Xf).sum(axis=0)).ravel()  # (A X)_ii, X symmetric
    assert np.max(np.abs(diag - 1.0)) < 1e-12


def test_columns_vs_sparse_lu():
    w = config("C2", scale=16)
    sym, P, lh, dt = run_oracle(w, relax=0.05)
    X = selinv.alg1(sym, lh, dt)
    n = w.n
    A = sp.csc_matrix((w.values[0], w.rowind, w.colptr), shape=(n, n))
    Af = (A + sp.tril(A, -1).T).tocsc()
    Bf = Af[w.perm][:, w.perm].tocsc()
    lu = spla.splu(Bf)
    rng = np.random.default_rng(7)
    xs = sym.xsuper
    for j in rng.choice(n, size=25, replace=False):
        e = np.zeros(n)
        e[j] = 1.0
        col = lu.solve(e)
        K = int(sym.col2super[j])
        f = int(xs[K])
        rows = np.concatenate([np.arange(f, xs[K + 1]), sym.rows[K]])
        got = X[K][:, j - f]
        assert np.max(np.abs(got - col[rows])) / np.max(np.abs(col)) < 1e-12


def test_zero_pivot_is_reported():
    w = config("C1")
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm)
    vals = w.values[0].copy()
    j_old = int(w.perm[0])  # first pivot of B is A[perm[0], perm[0]]
    vals[w.colptr[j_old]] = 0.0
    with pytest.raises(factor.ZeroPivot) as ei:
        factor.factor(sym, vals)
    assert ei.value.column == 0


# --------------------------------------------------------------------------
# log det B from the pivots (det B = prod_j D_jj for B = L D L^T, Section 2.3).
# Branch convention: the sum of the principal logarithms of the pivots.  Pinned
# against numpy's slogdet / det of the dense matrix (LU with partial pivoting,
# an independent route), and against the inertia from the eigenvalues.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,scale", [("C1", None), ("C4s", None), ("C2", 8)])
def test_logdet_real_spd_vs_slogdet(name, scale):
    w = config(name, scale=scale)
    sym, P, lh, dt = run_oracle(w)
    ld = factor.logdet(sym, P)
    sign, la = np.linalg.slogdet(selinv.permuted_dense(sym, w.values[0]))
    assert isinstance(ld, float) and sign == 1.0
    assert abs(ld - la) <= 1e-12 * max(1.0, abs(la))


@pytest.mark.parametrize("seed", range(4))
def test_logdet_real_indefinite_vs_slogdet_and_inertia(seed):
    """Mixed-sign strictly diagonally dominant matrices: no zero pivot without
    pivoting; the number of negative pivots is the number of negative
    eigenvalues (Sylvester's law of inertia)."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(30, 150))
    colptr, rowind, vals = random_pattern(n, 0.08, rng)
    v = vals[0].copy()
    flip = rng.random(n) < 0.4
    v[colptr[:-1][flip]] *= -1.0  # diagonal opens every column
    perm = rng.permutation(n).astype(np.int64)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=16)
    P = factor.factor(sym, v)
    ld = factor.logdet(sym, P)
    Bd = selinv.permuted_dense(sym, v)
    sign, la = np.linalg.slogdet(Bd)
    nneg = int(np.sum(np.linalg.eigvalsh(Bd) < 0))
    assert nneg > 0 and isinstance(ld, complex)
    assert abs(ld.real - la) <= 1e-12 * max(1.0, abs(la))
    assert abs(ld.imag - np.pi * nneg) <= 1e-12 * np.pi * n
    assert abs(np.exp(1j * ld.imag) - sign) < 1e-12


@pytest.mark.parametrize("name,scale,batch", [("C3", 6, 3), ("C5", 5, 2)])
def test_logdet_complex_vs_det(name, scale, batch):
    w = config(name, scale=scale, batch=batch)
    for l in range(w.batch):
        sym, P, lh, dt = run_oracle(w, l)
        ld = factor.logdet(sym, P)
        Bd = selinv.permuted_dense(sym, w.values[l])
        sign, la = np.linalg.slogdet(Bd)
        assert abs(ld.real - la) <= 1e-12 * max(1.0, abs(la))
        assert abs(np.exp(1j * ld.imag) - sign) < 1e-11
        if name == "C3":  # Im(pivot) < 0: every argument lies in (-pi, 0)
            assert -np.pi * w.n < ld.imag < 0.0


def test_logdet_complex_small_vs_det_value():
    """exp(log det) against numpy's det itself where it does not overflow."""
    rng = np.random.default_rng(77)
    for n in (12, 40, 90):
        colptr, rowind, vals = random_pattern(n, 0.1, rng, complex_values=True)
        v = vals[0] / np.abs(vals[0][colptr[:-1]]).mean()  # |det| of order one
        sym = symbolic.analyze(n, colptr, rowind, rng.permutation(n).astype(np.int64), cap=8)
        ld = factor.logdet(sym, factor.factor(sym, v))
        d = np.linalg.det(selinv.permuted_dense(sym, v))
        assert abs(np.exp(ld) - d) <= 1e-11 * abs(d)
