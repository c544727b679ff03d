"""Pins of the oracle's LU form (Alg. 1 and Alg. 2 with their U parts):
unsymmetric A with a symmetric pattern.

What fixes the answer (none of it retypes the oracle's formulas):
  * the definition: numpy's dense inverse of A assembled in the original
    indexing from the lower values and their mirrors, permuted afterwards;
  * the reconstruction L D U = B;
  * log det from slogdet;
  * Alg. 1 and Alg. 2 computing the same entries;
  * the symmetric special case: with mirrors equal to the lower values the LU
    route reduces to the LDL^T route.
Swapping the lower values and their mirrors is checked to fail the pins.
"""

import numpy as np
import pytest

from oracle import factor, selinv, symbolic
from workloads import config, random_pattern


def dense_original_lu(n, colptr, rowind, lo, up):
    A = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(colptr))
    A[cols, rowind] = up
    A[rowind, cols] = lo
    return A


def selected_from_dense_lu(sym, Ainv):
    """(X on the pattern of L, X^T on the pattern of L) of B = P A P^T, in panel layout."""
    Binv = Ainv[np.ix_(sym.perm, sym.perm)]
    outs = []
    for M in (Binv, Binv.T):
        out = []
        for K in range(sym.nsuper):
            f, l1 = int(sym.xsuper[K]), int(sym.xsuper[K + 1])
            rowsK = np.concatenate([np.arange(f, l1), sym.rows[K]])
            out.append(M[np.ix_(rowsK, np.arange(f, l1))])
        outs.append(out)
    return outs


def maxrel(A, B):
    num = max(float(np.max(np.abs(a - b))) if a.size else 0.0 for a, b in zip(A, B))
    den = max(float(np.max(np.abs(b))) if b.size else 0.0 for b in B)
    return num / den


def unsymmetric_random(n, dens, rng):
    """Random symmetric pattern, unsymmetric values, strictly diagonally
    dominant by rows and columns (unpivoted LU exists and is stable)."""
    colptr, rowind, vals = random_pattern(n, dens, rng)
    lo = vals[0].copy()
    cols = np.repeat(np.arange(n), np.diff(colptr))
    off = rowind != cols
    up = lo.copy()
    up[off] = lo[off] * rng.uniform(-1.5, 1.5, size=int(off.sum()))
    absum = np.zeros(n)
    np.add.at(absum, rowind[off], np.abs(lo[off]) + np.abs(up[off]))
    np.add.at(absum, cols[off], np.abs(lo[off]) + np.abs(up[off]))
    diag = colptr[:-1]
    lo[diag] = up[diag] = absum + 1.0
    return colptr, rowind, lo, up


def run_lu(sym, lo, up):
    PL, PU = factor.factor_lu(sym, lo, up)
    lh, ut, dt = factor.normalize_lu(sym, PL, PU)
    return PL, PU, lh, ut, dt, selinv.alg1_lu(sym, lh, ut, dt)


@pytest.mark.parametrize("seed", range(10))
def test_random_unsymmetric_vs_dense_inverse(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(10, 120))
    colptr, rowind, lo, up = unsymmetric_random(n, float(rng.uniform(0.02, 0.2)), rng)
    perm = rng.permutation(n).astype(np.int64)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=int(rng.integers(1, 20)), relax=float(rng.choice([0.0, 0.1])))
    A = dense_original_lu(n, colptr, rowind, lo, up)
    RL, RU = selected_from_dense_lu(sym, np.linalg.inv(A))
    PL, PU, lh, ut, dt, (XL, XU) = run_lu(sym, lo, up)
    assert maxrel(XL, RL) < 1e-12 and maxrel(XU, RU) < 1e-12
    YL, YU = selinv.alg2_lu(sym, lh, ut, dt)
    assert maxrel(YL, XL) < 1e-13 and maxrel(YU, XU) < 1e-13
    # reconstruction and log det
    L, D, U = factor.to_dense_ldu(sym, PL, PU)
    B = A[np.ix_(perm, perm)]
    assert np.max(np.abs(L @ np.diag(D) @ U - B)) <= 1e-13 * np.max(np.abs(B))
    sign, lad = np.linalg.slogdet(B)
    ld = factor.logdet(sym, PL)
    assert abs(np.real(ld) - lad) <= 1e-12 * max(1.0, abs(lad))
    assert abs(np.exp(1j * np.imag(ld)) - sign) <= 1e-12
    # the lower values and their mirrors swapped: the inverse of A^T, not of A
    _, _, _, _, _, (SL, SU) = run_lu(sym, up, lo)
    assert maxrel(SL, RL) > 1e-3


@pytest.mark.parametrize("relax", [0.0, 0.1])
@pytest.mark.parametrize("scale", [4, 6])
def test_u3_vs_dense_inverse(scale, relax):
    w = config("U3", scale=scale, batch=2)
    assert w.is_lu
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=24, relax=relax)
    for l in range(w.batch):
        lo, up = w.lower_values[l], w.upper_values[l]
        A = dense_original_lu(w.n, w.colptr, w.rowind, lo, up)
        assert np.max(np.abs(A - A.T)) > 0.1  # genuinely unsymmetric
        RL, RU = selected_from_dense_lu(sym, np.linalg.inv(A))
        _, _, lh, ut, dt, (XL, XU) = run_lu(sym, lo, up)
        assert maxrel(XL, RL) < 1e-12 and maxrel(XU, RU) < 1e-12


def test_symmetric_values_reduce_to_ldlt():
    """Mirrors equal to the lower values: XL = XU = the LDL^T route's X."""
    w = config("C2", scale=6)
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=16, relax=0.05)
    v = w.values[0]
    _, _, _, _, _, (XL, XU) = run_lu(sym, v, v)
    lh, dt = factor.normalize(sym, factor.factor(sym, v))
    X = selinv.alg1(sym, lh, dt)
    assert maxrel(XL, X) < 1e-13 and maxrel(XU, X) < 1e-13
