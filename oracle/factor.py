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

Hermitian A (``herm=True``): the same with conjugate transposes wherever a
transpose appears (Section 2.3, after Alg. 2): B = L D L^H with real D,
U = D L^H, Dt_K^{-1} = L_KK^{-H} D_K^{-1} L_KK^{-1}.  A stored lower value of
A that the permutation moves into B's upper triangle enters B's lower
triangle conjugated.

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


def b_lower_values(sym, avals, herm=False):
    """B's lower values in B's CSC order from A's stored lower values."""
    avals = np.asarray(avals)
    if herm:
        avals = np.where(sym.aflip, np.conj(avals), avals)
    bvals = np.empty_like(avals)
    bvals[sym.amap] = avals
    return bvals


def factor(sym, avals, herm=False):
    """Unpivoted supernodal LDL^T (LDL^H for ``herm``) of B = P A P^T from A's
    stored lower values.

    ``avals`` is one matrix's values in A's CSC order.  Raises ZeroPivot on an
    exactly zero or non-finite pivot (no perturbation, no pivoting).
    """
    return factor_panels(sym, assemble(sym, b_lower_values(sym, avals, herm)), herm)


def _tr(M, herm):
    """Transpose, conjugate transpose for a Hermitian matrix."""
    return M.conj().T if herm else M.T


def factor_panels(sym, panels, herm=False):
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
            # trailing update of the remaining panel columns (lower part
            # suffices): entry (i, k) loses L_i d L_k, L_i d conj(L_k) if Hermitian
            row = P[jj + 1:s, jj]
            P[jj + 1:, jj + 1:] -= np.outer(col, np.conj(row) if herm else row)
            P[jj + 1:, jj] = col
        C = sym.rows[K]
        c = C.shape[0]
        if c == 0:
            continue
        Lc = P[s:, :]
        Dk = np.diag(P[:s, :s]).copy()
        U = (Lc * Dk[None, :]) @ _tr(Lc, herm)  # c x c: L_C D L_C^T (L_C D L_C^H if Hermitian)
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


def normalize(sym, panels, herm=False):
    """Alg. 1 steps 1-2 for LDL^T: returns (Lhat list, Dtinv list).

    Lhat_{C,K} = L_{C,K} L_KK^{-1}; Dt_K^{-1} = L_KK^{-T} D_K^{-1} L_KK^{-1}
    (L_KK^{-H} for ``herm``).
    """
    lhat, dtinv = [], []
    for K in range(sym.nsuper):
        P = panels[K]
        s = sym.width(K)
        Lkk = np.tril(P[:s, :s], -1) + np.eye(s, dtype=P.dtype)
        d = np.diag(P[:s, :s]).copy()
        Linv = sla.solve_triangular(Lkk, np.eye(s, dtype=P.dtype), lower=True, unit_diagonal=True)
        dtinv.append(_tr(Linv, herm) @ (Linv / d[:, None]))
        Lc = P[s:, :]
        # Lhat = Lc Lkk^{-1}  <=>  Lhat^T = Lkk^{-T} Lc^T
        lhat.append(Lc @ Linv)
    return lhat, dtinv


def dtilde(sym, panels, herm=False):
    """Dt_K = L_KK D_K L_KK^T (L_KK^H for ``herm``; the pivot block of the block LDL^T)."""
    out = []
    for K in range(sym.nsuper):
        P = panels[K]
        s = sym.width(K)
        Lkk = np.tril(P[:s, :s], -1) + np.eye(s, dtype=P.dtype)
        d = np.diag(P[:s, :s]).copy()
        out.append((Lkk * d[None, :]) @ _tr(Lkk, herm))
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


# ---------------------------------------------------------------------------
# Unsymmetric A with a symmetric pattern: B = L D U (Alg. 1 and Alg. 2 in
# their LU form).  Two panel sets share the layout of L: ``PL`` holds L (strict
# lower top block, D on the diagonal, L_{C,K} below) and ``PU`` holds U^T the
# same way (U unit upper, so U^T is unit lower; D again on the diagonal, and
# U_{K,C}^T below).  A's values come as the stored lower values a_lo[e] =
# A(r, c) and their mirrors a_up[e] = A(c, r) (r >= c, equal on the diagonal).
# ---------------------------------------------------------------------------

def b_values_lu(sym, a_lo, a_up):
    """(B's lower values, B's upper values transposed) in B's lower CSC order:
    an A entry the permutation moves into B's upper triangle swaps roles."""
    a_lo, a_up = np.asarray(a_lo), np.asarray(a_up)
    low = np.where(sym.aflip, a_up, a_lo)
    up = np.where(sym.aflip, a_lo, a_up)
    bl, bu = np.empty_like(low), np.empty_like(up)
    bl[sym.amap] = low
    bu[sym.amap] = up
    return bl, bu


def factor_lu(sym, a_lo, a_up):
    """Unpivoted supernodal LDU of B = P A P^T: returns (PL, PU)."""
    bl, bu = b_values_lu(sym, a_lo, a_up)
    PL, PU = assemble(sym, bl), assemble(sym, bu)
    xs = sym.xsuper
    for K in range(sym.nsuper):
        L, U = PL[K], PU[K]
        s = sym.width(K)
        f = int(xs[K])
        for jj in range(s):
            d = L[jj, jj]
            if d == 0 or not np.isfinite(d):
                raise ZeroPivot(f + jj, d)
            lrow = L[jj + 1:s, jj].copy()  # L_k d, k in the block
            urow = U[jj + 1:s, jj].copy()  # d U_k
            lcol = L[jj + 1:, jj] / d
            ucol = U[jj + 1:, jj] / d
            # B(i, k) -= L_i d U_k: the lower part in PL, the upper part (transposed) in PU
            L[jj + 1:, jj + 1:] -= np.outer(lcol, urow)
            U[jj + 1:, jj + 1:] -= np.outer(ucol, lrow)
            L[jj + 1:, jj] = lcol
            U[jj + 1:, jj] = ucol
            U[jj, jj] = d
        C = sym.rows[K]
        c = C.shape[0]
        if c == 0:
            continue
        Dk = np.diag(L[:s, :s]).copy()
        Lc, Uc = L[s:, :], U[s:, :]
        SL = (Lc * Dk[None, :]) @ Uc.T   # S(a, b) = sum_j L_a D_j U_b, lower part into PL
        SU = (Uc * Dk[None, :]) @ Lc.T   # S(b, a) for a >= b, transposed into PU
        g0, g1 = sym.seg_ptr[K], sym.seg_ptr[K + 1]
        for g in range(g0, g1):
            J = int(sym.seg_super[g])
            st = int(sym.seg_start[g])
            en = int(sym.seg_start[g + 1]) if g + 1 < g1 else c
            pos = sym.posarr[sym.seg_posoff[g]: sym.seg_posoff[g] + (c - st)]
            fJ = int(xs[J])
            aa, bb = np.nonzero(np.arange(st, c)[:, None] >= np.arange(st, en)[None, :])
            PL[J][pos[aa], C[st + bb] - fJ] -= SL[st + aa, st + bb]
            PU[J][pos[aa], C[st + bb] - fJ] -= SU[st + aa, st + bb]
    return PL, PU


def normalize_lu(sym, PL, PU):
    """Alg. 1 steps 1-2 in LU form: (Lhat, Uhat^T, Dt^{-1}) per supernode with
    Lhat = L_{C,K} L_KK^{-1}, Uhat^T = (U_KK^{-1} U_{K,C})^T and
    Dt^{-1} = U_KK^{-1} D_K^{-1} L_KK^{-1}."""
    lhat, uhat_t, dtinv = [], [], []
    for K in range(sym.nsuper):
        s = sym.width(K)
        L, U = PL[K], PU[K]
        eye = np.eye(s, dtype=L.dtype)
        Li = sla.solve_triangular(np.tril(L[:s, :s], -1) + eye, eye, lower=True, unit_diagonal=True)
        Ui_t = sla.solve_triangular(np.tril(U[:s, :s], -1) + eye, eye, lower=True, unit_diagonal=True)  # U_KK^{-T}
        d = np.diag(L[:s, :s]).copy()
        lhat.append(L[s:, :] @ Li)
        uhat_t.append(U[s:, :] @ Ui_t)
        dtinv.append(Ui_t.T @ (Li / d[:, None]))
    return lhat, uhat_t, dtinv


def to_dense_ldu(sym, PL, PU):
    """Dense unit lower L, diagonal D and unit upper U (small problems only)."""
    L, D = to_dense_L(sym, PL)
    Ut, _ = to_dense_L(sym, PU)
    return L, D, Ut.T
