"""Pins of the oracle's Hermitian variant (conjugate transposes, Section 2.3).

What fixes the answer (none of it retypes the oracle's formulas):
  * the definition: A^{-1} from numpy's dense inverse of A assembled in the
    original indexing (A[r, c] = a, A[c, r] = conj(a)), permuted afterwards,
    so that neither the permutation map nor the conjugation of entries that
    the permutation moves to the upper triangle comes from the oracle;
  * tr(A^{-1}) = sum 1 / lambda from numpy's Hermitian eigensolver;
  * the reconstruction L D L^H = B with a real D, and log det from slogdet;
  * Alg. 1 and Alg. 2 computing the same entries.
The symmetric (plain transpose) route is checked to fail these pins, so they
do see a missing conjugation.
"""

import numpy as np
import pytest

from oracle import factor, selinv, symbolic
from workloads import config, random_pattern


def dense_original(n, colptr, rowind, vals):
    """Dense Hermitian A in the original indexing from its stored lower values."""
    A = np.zeros((n, n), dtype=np.complex128)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    A[cols, rowind] = np.conj(vals)
    A[rowind, cols] = vals
    return A


def selected_from_dense(sym, Ainv):
    """The entries of (P A P^T)^{-1} on the pattern of L, in panel layout."""
    Binv = Ainv[np.ix_(sym.perm, sym.perm)]
    out = []
    for K in range(sym.nsuper):
        f, l1 = int(sym.xsuper[K]), int(sym.xsuper[K + 1])
        rowsK = np.concatenate([np.arange(f, l1), sym.rows[K]])
        out.append(Binv[np.ix_(rowsK, np.arange(f, l1))])
    return out


def maxrel(A, B):
    num = max(float(np.max(np.abs(a - b))) if a.size else 0.0 for a, b in zip(A, B))
    den = max(float(np.max(np.abs(b))) if b.size else 0.0 for b in B)
    return num / den


def hermitian_random(n, dens, rng, indefinite=False):
    """Strictly diagonally dominant Hermitian matrix on a random pattern
    (unpivoted LDL^H exists); ``indefinite``: diagonal signs drawn at random."""
    colptr, rowind, vals = random_pattern(n, dens, rng, complex_values=True)
    v = vals[0].copy()
    diag = colptr[:-1]
    d = np.abs(v[diag].real)
    if indefinite:
        d = d * rng.choice([-1.0, 1.0], size=n)
    v[diag] = d
    return colptr, rowind, v


def run(sym, vals, herm=True):
    P = factor.factor(sym, vals, herm=herm)
    lh, dt = factor.normalize(sym, P, herm=herm)
    return P, lh, dt, selinv.alg1(sym, lh, dt, herm=herm)


@pytest.mark.parametrize("relax", [0.0, 0.1])
@pytest.mark.parametrize("scale", [4, 6])
def test_h3_alg1_alg2_vs_dense_inverse(scale, relax):
    w = config("H3", scale=scale, batch=3)
    assert w.is_hermitian
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=24, relax=relax)
    for l in range(w.batch):
        A = dense_original(w.n, w.colptr, w.rowind, w.values[l])
        assert np.array_equal(A, A.conj().T)
        ref = selected_from_dense(sym, np.linalg.inv(A))
        P, lh, dt, X = run(sym, w.values[l])
        assert maxrel(X, ref) < 1e-12
        assert maxrel(selinv.alg2(sym, lh, dt, herm=True), X) < 1e-13
        for K in range(sym.nsuper):
            s = sym.width(K)
            assert np.array_equal(X[K][:s, :], X[K][:s, :].conj().T)  # Hermitian diagonal blocks
        # trace of the inverse from the eigenvalues
        tr = sum(np.trace(X[K][:sym.width(K), :]) for K in range(sym.nsuper))
        lam = np.linalg.eigvalsh(A)
        assert abs(tr - np.sum(1.0 / lam)) <= 1e-12 * abs(np.sum(1.0 / lam))
        # the symmetric route misses the conjugations
        _, _, _, Xs = run(sym, w.values[l], herm=False)
        assert maxrel(Xs, ref) > 1e-3


@pytest.mark.parametrize("seed", range(8))
def test_random_hermitian_patterns_vs_dense(seed):
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(10, 110))
    colptr, rowind, v = hermitian_random(n, float(rng.uniform(0.03, 0.2)), rng, indefinite=bool(seed % 2))
    perm = rng.permutation(n).astype(np.int64)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=int(rng.integers(1, 20)),
                           relax=float(rng.choice([0.0, 0.1])))
    A = dense_original(n, colptr, rowind, v)
    ref = selected_from_dense(sym, np.linalg.inv(A))
    P, lh, dt, X = run(sym, v)
    assert maxrel(X, ref) < 1e-12
    assert maxrel(selinv.alg2(sym, lh, dt, herm=True), X) < 1e-13
    # on A's own pattern, original indexing (conjugated where the permutation flips an entry)
    xa = selinv.on_pattern_of_A(sym, X, colptr, rowind, herm=True)
    Ainv = np.linalg.inv(A)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    want = Ainv[rowind, cols]
    assert np.max(np.abs(xa - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.any(sym.aflip)  # the random permutation does flip entries


@pytest.mark.parametrize("seed", range(4))
def test_ldlh_reconstruction_real_pivots_and_logdet(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(20, 90))
    colptr, rowind, v = hermitian_random(n, 0.1, rng, indefinite=bool(seed % 2))
    perm = rng.permutation(n).astype(np.int64)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=8)
    P = factor.factor(sym, v, herm=True)
    L, D = factor.to_dense_L(sym, P)
    B = dense_original(n, colptr, rowind, v)[np.ix_(perm, perm)]
    assert np.max(np.abs(L @ np.diag(D) @ L.conj().T - B)) <= 1e-13 * np.max(np.abs(B))
    assert np.max(np.abs(D.imag)) <= 1e-14 * np.max(np.abs(D.real))
    sign, lad = np.linalg.slogdet(B)
    ld = factor.logdet(sym, P)
    assert abs(np.real(ld) - lad) <= 1e-12 * max(1.0, abs(lad))
    # the imaginary part is pi per negative pivot: exp(i Im) is the sign of det B
    assert abs(np.exp(1j * np.imag(ld)) - sign) <= 1e-12
