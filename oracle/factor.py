"""Oracle supernodal LDL^T and normalized factors (test infrastructure only).

The paper takes the factorization from an external solver that does no
dynamic pivoting and permutes symmetrically without looking at values
(Section 4).  Its LDL^T specialization (Section 2.3, the paragraph after
Alg. 2) makes U = D L^T, so the normalized factors of Alg. 1 steps 1-2 become

    Lhat_{C,K} = L_{C,K} L_{K,K}^{-1}          (U-hat_{K,C} = Lhat_{C,K}^T)
    Dt_K^{-1}  = U_{K,K}^{-1} L_{K,K}^{-1} = (L_KK D_K L_KK^T)^{-1}.

The factorization here is plain right-looking supernodal LDL^T with scalar
pivots: for every supernode in increasing order, factor the dense diagonal
block, solve for L_{C,K}, and subtract L_{C,K} D_K L_{C,K}^T from the
ancestors' panels (the fill property guarantees every target lies in F).

Panel layout: supernode K has a dense (s + c) x s array whose rows are K's own
columns followed by C(K).  After ``factor`` the strict lower part of the top
s x s block holds L_KK, its diagonal holds D_K and the bottom c x s block
holds L_{C,K}.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class ZeroPivot(Exception):
    def __init__(self, column, value):
        super().__init__(f"zero or non-finite pivot at column {column}: {value}")
        self.column = column
        self.value = value


def assemble(sym, bvals):
    """Scatter B's lower values into zeroed panels."""
    dtype = np.complex128 if np.iscomplexobj(bvals) else np.float64
    panels = []
    for K in range(sym.nsuper):
        s = sym.width(K)
        c = sym.rows[K].shape[0]
        panels.append(np.zeros((s + c, s), dtype=dtype))
    n = sym.n
    xs = sym.xsuper
    for j in range(n):
        K = int(sym.col2super[j])
        f, l = int(xs[K]), int(xs[K + 1] - 1)
        lo, hi = sym.Bcolptr[j], sym.Bcolptr[j + 1]
        r = sym.Browind[lo:hi]
        pos = np.where(r <= l, r - f, (l - f + 1) + np.searchsorted(sym.rows[K], r))
        panels[K][pos, j - f] = bvals[lo:hi]
    return panels


def factor(sym, avals):
    """Unpivoted supernodal LDL^T of B = P A P^T from A's stored lower values.

    ``avals`` is one matrix's values in A's CSC order.  Raises ZeroPivot on an
    exactly zero or non-finite pivot (no perturbation, no pivoting).
    """
    avals = np.asarray(avals)
    bvals = np.empty_like(avals)
    bvals[sym.amap] = avals
    return factor_panels(sym, assemble(sym, bvals))


def factor_panels(sym, panels):
    """Factor in place panels that already hold B's lower values on the pattern of L.

    Entries of the pattern of L that are not in A are allowed to be nonzero:
    the pattern of L is chordal, so such a matrix factors with no new fill.
    """
    xs = sym.xsuper
    for K in range(sym.nsuper):
        P = panels[K]
        s = sym.width(K)
        f = int(xs[K])
        # dense right-looking LDL^T of the panel's columns (scalar pivots)
        for jj in range(s):
            d = P[jj, jj]
            if d == 0 or not np.isfinite(d):
                raise ZeroPivot(f + jj, d)
            col = P[jj + 1:, jj] / d
            # trailing update of the remaining panel columns (lower part suffices)
            P[jj + 1:, jj + 1:] -= np.outer(col, P[jj + 1:s, jj])
            P[jj + 1:, jj] = col
        C = sym.rows[K]
        c = C.shape[0]
        if c == 0:
            continue
        Lc = P[s:, :]
        Dk = np.diag(P[:s, :s]).copy()
        U = (Lc * Dk[None, :]) @ Lc.T  # c x c, symmetric (plain transpose)
        g0, g1 = sym.seg_ptr[K], sym.seg_ptr[K + 1]
        for g in range(g0, g1):
            J = int(sym.seg_super[g])
            st = int(sym.seg_start[g])
            en = int(sym.seg_start[g + 1]) if g + 1 < g1 else c
            pos = sym.posarr[sym.seg_posoff[g]: sym.seg_posoff[g] + (c - st)]
            fJ = int(xs[J])
            # rows a >= b of the columns C[b], b in [st, en) (lower triangle only)
            aa, bb = np.nonzero(np.arange(st, c)[:, None] >= np.arange(st, en)[None, :])
            panels[J][pos[aa], C[st + bb] - fJ] -= U[st + aa, st + bb]
    return panels


def normalize(sym, panels):
    """Alg. 1 steps 1-2 for LDL^T: returns (Lhat list, Dtinv list).

    Lhat_{C,K} = L_{C,K} L_KK^{-1}; Dt_K^{-1} = L_KK^{-T} D_K^{-1} L_KK^{-1}.
    """
    lhat, dtinv = [], []
    for K in range(sym.nsuper):
        P = panels[K]
        s = sym.width(K)
        Lkk = np.tril(P[:s, :s], -1) + np.eye(s, dtype=P.dtype)
        d = np.diag(P[:s, :s]).copy()
        Linv = sla.solve_triangular(Lkk, np.eye(s, dtype=P.dtype), lower=True, unit_diagonal=True)
        dtinv.append(Linv.T @ (Linv / d[:, None]))
        Lc = P[s:, :]
        # Lhat = Lc Lkk^{-1}  <=>  Lhat^T = Lkk^{-T} Lc^T
        lhat.append(Lc @ Linv)
    return lhat, dtinv


def dtilde(sym, panels):
    """Dt_K = L_KK D_K L_KK^T (the pivot block of the block LDL^T)."""
    out = []
    for K in range(sym.nsuper):
        P = panels[K]
        s = sym.width(K)
        Lkk = np.tril(P[:s, :s], -1) + np.eye(s, dtype=P.dtype)
        d = np.diag(P[:s, :s]).copy()
        out.append((Lkk * d[None, :]) @ Lkk.T)
    return out


def logdet(sym, panels):
    """log det B from the pivots: B = L D L^T with L unit lower triangular
    (Section 2.3), so det B = prod_j D_jj.

    Branch convention: the sum over j of the principal logarithm of D_jj
    (not reduced to one branch afterwards).  Its real part is log|det B| and
    its exponential is det B.  A real B with positive pivots gives a float; a
    real B with negative pivots gives a complex value whose imaginary part is
    pi times the number of negative pivots (the inertia), and a complex B the
    sum of the pivots' arguments.
    """
    tot = 0.0 + 0.0j
    neg = False
    for K in range(sym.nsuper):
        s = sym.width(K)
        d = np.diag(panels[K][:s, :s])
        if not np.iscomplexobj(d):
            neg = neg or bool(np.any(d < 0))
        tot = tot + np.sum(np.log(d.astype(np.complex128)))
    if not np.iscomplexobj(panels[0]) and not neg:
        return float(tot.real)
    return complex(tot)


def to_dense_L(sym, panels):
    """Dense unit-lower L and diagonal D (small problems only)."""
    n = sym.n
    dtype = panels[0].dtype
    L = np.eye(n, dtype=dtype)
    D = np.zeros(n, dtype=dtype)
    for K in range(sym.nsuper):
        f, l1 = int(sym.xsuper[K]), int(sym.xsuper[K + 1])
        s = l1 - f
        P = panels[K]
        D[f:l1] = np.diag(P[:s, :s])
        L[f:l1, f:l1] = np.tril(P[:s, :s], -1) + np.eye(s, dtype=dtype)
        L[np.ix_(sym.rows[K], np.arange(f, l1))] = P[s:, :]
    return L, D
