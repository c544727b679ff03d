"""Oracle selected inversion (test infrastructure only).

Output convention: X is stored in panels with the layout of the factor panels
(rows = K's columns then C(K)); the top s x s block holds the full symmetric
A^{-1}_{K,K} and the bottom c x s block holds A^{-1}_{C,K}.  Together they are
every selected entry of the lower triangle: (i, j) with L_ij != 0 (Alg. 1 and
Alg. 2 output lines).  The upper triangle is the transpose (LDL^T
specialization, Section 2.3).  Transposes are plain transposes, also for
complex-symmetric matrices; with ``herm=True`` (Hermitian A, the variant of
Section 2.3 after Alg. 2) every transpose is a conjugate transpose, so the
upper triangle is the conjugate transpose of the lower one.

Three independent formulations:
  dense_selected  the definition: (P A P^T)^{-1} restricted to the pattern of L.
  alg1            Alg. 1, second loop (steps 3-4 with the LDL^T specialization
                  Uhat = Lhat^T), plus the diagonal-block symmetrization
                  described after Alg. 2.
  alg2            Alg. 2, the left-looking form: the diagonal update, then the
                  outer-product update Eq. (outerprod) and the inner-product
                  update Eq. (innerprod) pushed into the descendants C'(K)
                  (Eq. (newset)), split as the D, O, I and ID tasks of Section 3.1.
"""

from __future__ import annotations

import numpy as np


def _tr(M, herm):
    return M.conj().T if herm else M.T


def gather_cc(sym, X, K, herm=False):
    """Dense A^{-1}_{C,C} for C = C(K) from ancestor panels (lower part + its
    transpose, or conjugate transpose for ``herm``)."""
    C = sym.rows[K]
    c = C.shape[0]
    dtype = np.result_type(*[X[int(J)].dtype for J in sym.seg_super[sym.seg_ptr[K]:sym.seg_ptr[K + 1]]]) if c else np.float64
    G = np.zeros((c, c), dtype=dtype)
    g0, g1 = sym.seg_ptr[K], sym.seg_ptr[K + 1]
    for g in range(g0, g1):
        J = int(sym.seg_super[g])
        st = int(sym.seg_start[g])
        en = int(sym.seg_start[g + 1]) if g + 1 < g1 else c
        pos = sym.posarr[sym.seg_posoff[g]: sym.seg_posoff[g] + (c - st)]
        cols = C[st:en] - sym.xsuper[J]
        # column b of G (b in this segment), rows a >= st: X_J[pos[a - st], C[b] - first(J)]
        G[st:, st:en] = X[J][np.ix_(pos, cols)]
    lower = np.tril(G)
    return lower + _tr(np.tril(G, -1), herm)


def alg1(sym, lhat, dtinv, stop_after=None, herm=False):
    """Alg. 1 second loop, K = N..1 (root first), pull form.

    A^{-1}_{C,K} = -A^{-1}_{C,C} Lhat_{C,K}                   (step 3)
    A^{-1}_{K,K} = Dt_K^{-1} - Lhat_{C,K}^T A^{-1}_{C,K}        (step 4, Uhat = Lhat^T)
    A^{-1}_{K,K} <- (A^{-1}_{K,K} + A^{-T}_{K,K}) / 2            (symmetrization)
    (``herm``: ^H in place of ^T.)

    ``stop_after``: process only that many supernodes of the loop (the
    highest-numbered ones, which need no others; for timing a sample).
    """
    X = [None] * sym.nsuper
    order = list(reversed(range(sym.nsuper)))
    if stop_after is not None:
        order = order[:stop_after]
    for K in order:
        s = sym.width(K)
        c = sym.rows[K].shape[0]
        dtype = dtinv[K].dtype
        P = np.zeros((s + c, s), dtype=dtype)
        if c:
            G = gather_cc(sym, X, K, herm)
            Y = -G @ lhat[K]
            T = dtinv[K] - _tr(lhat[K], herm) @ Y
            P[s:, :] = Y
        else:
            T = dtinv[K].copy()
        P[:s, :] = 0.5 * (T + _tr(T, herm))
        X[K] = P
    return X


def descendants(sym):
    """C'(K) = {I' < K : L_{K,I'} != 0} for every K (Eq. (newset))."""
    out = [[] for _ in range(sym.nsuper)]
    for I in range(sym.nsuper):
        for g in range(sym.seg_ptr[I], sym.seg_ptr[I + 1]):
            out[int(sym.seg_super[g])].append((I, g))
    return out


def alg2(sym, lhat, dtinv, herm=False):
    """Alg. 2 (left-looking selected inversion), LDL^T specialization
    (``herm``: conjugate transposes in the D and I tasks).

    X starts at zero on the pattern of L.  For K = N..1:
      D   : X_KK = Dt_K^{-1} - Lhat_{C,K}^T X_{C,K}, then symmetrize.
      for each descendant I' in C'(K), with R_K = C(I') inside K's columns and
      R_> = C(I') above K (all of which lie in C(K)):
      O   : X[R_>, I'] -= X[R_>, R_K] Lhat[R_K, I']                  Eq. (outerprod)
      I   : X[R_K, I'] -= X[R_>, R_K]^T Lhat[R_>, I']                 Eq. (innerprod), I in C
      ID  : X[R_K, I'] -= X_KK[R_K, R_K] Lhat[R_K, I']                Eq. (innerprod), I = K
    X[*, I'] is stored in I''s panel, rows s_I' + (index in C(I')).
    """
    xs = sym.xsuper
    X = []
    for K in range(sym.nsuper):
        s = sym.width(K)
        c = sym.rows[K].shape[0]
        X.append(np.zeros((s + c, s), dtype=dtinv[K].dtype))
    desc = descendants(sym)
    for K in reversed(range(sym.nsuper)):
        s = sym.width(K)
        fK = int(xs[K])
        PK = X[K]
        # D task
        T = dtinv[K] - _tr(lhat[K], herm) @ PK[s:, :]
        PK[:s, :] = 0.5 * (T + _tr(T, herm))
        XKK = PK[:s, :]
        for (I, g) in desc[K]:
            sI = sym.width(I)
            CI = sym.rows[I]
            cI = CI.shape[0]
            st = int(sym.seg_start[g])
            g1 = sym.seg_ptr[I + 1]
            en = int(sym.seg_start[g + 1]) if g + 1 < g1 else cI
            pos = sym.posarr[sym.seg_posoff[g]: sym.seg_posoff[g] + (cI - st)]
            rk = np.arange(st, en)          # indices into C(I) of R_K
            ra = np.arange(en, cI)          # indices into C(I) of R_>
            colsK = CI[rk] - fK             # columns of K's panel
            posA = pos[en - st:]            # rows of K's panel holding R_>
            XI = X[I]
            Lh = lhat[I]
            X_a_k = PK[np.ix_(posA, colsK)]  # X[R_>, R_K], part of X_{C(K),K}
            # O task
            if ra.size:
                XI[sI + ra, :] -= X_a_k @ Lh[rk, :]
            # I task
            if ra.size:
                XI[sI + rk, :] -= _tr(X_a_k, herm) @ Lh[ra, :]
            # ID task
            XI[sI + rk, :] -= XKK[np.ix_(colsK, colsK)] @ Lh[rk, :]
    return X


def dense_selected(sym, bdense):
    """The definition: (P A P^T)^{-1} on the pattern of L, in panel layout."""
    Xd = np.linalg.inv(bdense)
    X = []
    for K in range(sym.nsuper):
        f, l1 = int(sym.xsuper[K]), int(sym.xsuper[K + 1])
        rowsK = np.concatenate([np.arange(f, l1), sym.rows[K]])
        X.append(Xd[np.ix_(rowsK, np.arange(f, l1))].copy())
    return X


def permuted_dense(sym, avals, herm=False):
    """Dense B = P A P^T from A's stored lower values (small problems); the
    upper triangle mirrors the lower one, conjugated for ``herm``."""
    n = sym.n
    avals = np.asarray(avals)
    if herm:
        avals = np.where(sym.aflip, np.conj(avals), avals)
    bvals = np.empty_like(avals)
    bvals[sym.amap] = avals
    Bd = np.zeros((n, n), dtype=avals.dtype)
    cols = np.repeat(np.arange(n), np.diff(sym.Bcolptr))
    Bd[cols, sym.Browind] = np.conj(bvals) if herm else bvals
    Bd[sym.Browind, cols] = bvals
    return Bd


def flatten(sym, X):
    """Concatenate panels column-major into one vector (the device layout)."""
    return np.concatenate([P.reshape(-1, order="F") for P in X]) if X else np.zeros(0)


def unflatten(sym, vec):
    out = []
    off = 0
    for K in range(sym.nsuper):
        s = sym.width(K)
        r = s + sym.rows[K].shape[0]
        out.append(np.asarray(vec[off: off + r * s]).reshape((r, s), order="F"))
        off += r * s
    return out


def on_pattern_of_A(sym, X, colptr, rowind, herm=False):
    """Selected entries at A's stored lower positions, original indexing.

    A entry (r, c) reads X at (max(ip[r], ip[c]), min(...)) of B, conjugated
    for ``herm`` when ip[r] < ip[c] (the entry lies in B's upper triangle).
    """
    n = sym.n
    ip = np.empty(n, dtype=np.int64)
    ip[sym.perm] = np.arange(n)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    i = ip[np.asarray(rowind)]
    j = ip[cols]
    hi, lo = np.maximum(i, j), np.minimum(i, j)
    out = np.empty(hi.shape[0], dtype=X[0].dtype)
    K = sym.col2super[lo]
    for e in range(hi.shape[0]):
        k = int(K[e])
        f, l = int(sym.xsuper[k]), int(sym.xsuper[k + 1] - 1)
        r = int(hi[e])
        if r <= l:
            pr = r - f
        else:
            pr = (l - f + 1) + int(np.searchsorted(sym.rows[k], r))
        out[e] = X[k][pr, int(lo[e]) - f]
    if herm:
        out = np.where(i < j, np.conj(out), out)
    return out


# ---------------------------------------------------------------------------
# LU form (unsymmetric A, symmetric pattern).  XL holds X on the pattern of L
# (the lower part and the full diagonal blocks), XU holds X^T the same way
# (entry (r, q) of XU is X(q, r)), both in the panel layout.
# ---------------------------------------------------------------------------

def gather_cc_lu(sym, XL, XU, K):
    """Dense A^{-1}_{C,C}: the lower part from XL, the upper part from XU."""
    GL = gather_cc(sym, XL, K)
    GU = gather_cc(sym, XU, K)
    return np.tril(GL) + np.triu(GU.T, 1)


def alg1_lu(sym, lhat, uhat_t, dtinv):
    """Alg. 1 (LU), K = N..1, pull form:
    A^{-1}_{C,K} = -A^{-1}_{C,C} Lhat_{C,K};  A^{-1}_{K,C} = -Uhat_{K,C} A^{-1}_{C,C};
    A^{-1}_{K,K} = U_KK^{-1} L_KK^{-1} - Uhat_{K,C} A^{-1}_{C,K}  (no symmetrization)."""
    XL, XU = [None] * sym.nsuper, [None] * sym.nsuper
    for K in reversed(range(sym.nsuper)):
        s = sym.width(K)
        c = sym.rows[K].shape[0]
        PL = np.zeros((s + c, s), dtype=dtinv[K].dtype)
        PU = np.zeros_like(PL)
        T = dtinv[K].copy()
        if c:
            G = gather_cc_lu(sym, XL, XU, K)
            YL = -G @ lhat[K]
            YU = -G.T @ uhat_t[K]       # A^{-1}_{K,C} transposed
            T = T - uhat_t[K].T @ YL
            PL[s:, :] = YL
            PU[s:, :] = YU
        PL[:s, :] = T
        PU[:s, :] = T.T
        XL[K], XU[K] = PL, PU
    return XL, XU


def alg2_lu(sym, lhat, uhat_t, dtinv):
    """Alg. 2 (LU), left-looking: the D task, then the outer- and
    inner-product updates of the lower part (Eqs. (outerprod), (innerprod))
    and of the upper part (the last two steps of Alg. 2), pushed into the
    descendants."""
    xs = sym.xsuper
    XL, XU = [], []
    for K in range(sym.nsuper):
        s = sym.width(K)
        c = sym.rows[K].shape[0]
        XL.append(np.zeros((s + c, s), dtype=dtinv[K].dtype))
        XU.append(np.zeros((s + c, s), dtype=dtinv[K].dtype))
    desc = descendants(sym)
    for K in reversed(range(sym.nsuper)):
        s = sym.width(K)
        fK = int(xs[K])
        PL, PU = XL[K], XU[K]
        T = dtinv[K] - uhat_t[K].T @ PL[s:, :]
        PL[:s, :] = T
        PU[:s, :] = T.T
        for (I, g) in desc[K]:
            sI = sym.width(I)
            CI = sym.rows[I]
            cI = CI.shape[0]
            st = int(sym.seg_start[g])
            g1 = sym.seg_ptr[I + 1]
            en = int(sym.seg_start[g + 1]) if g + 1 < g1 else cI
            pos = sym.posarr[sym.seg_posoff[g]: sym.seg_posoff[g] + (cI - st)]
            rk = np.arange(st, en)
            ra = np.arange(en, cI)
            colsK = CI[rk] - fK
            posA = pos[en - st:]
            XLa_k = PL[np.ix_(posA, colsK)]   # X[R_>, R_K]
            XUa_k = PU[np.ix_(posA, colsK)]   # X[R_K, R_>] transposed
            Lh, Ut = lhat[I], uhat_t[I]
            if ra.size:
                XL[I][sI + ra, :] -= XLa_k @ Lh[rk, :]          # lower, outer product
                XL[I][sI + rk, :] -= XUa_k.T @ Lh[ra, :]        # lower, inner product (I in C)
                XU[I][sI + ra, :] -= XUa_k @ Ut[rk, :]          # upper, outer product
                XU[I][sI + rk, :] -= XLa_k.T @ Ut[ra, :]        # upper, inner product (I in C)
            XL[I][sI + rk, :] -= PL[:s, :][np.ix_(colsK, colsK)] @ Lh[rk, :]   # lower, I = K
            XU[I][sI + rk, :] -= PU[:s, :][np.ix_(colsK, colsK)] @ Ut[rk, :]   # upper, I = K
    return XL, XU


def permuted_dense_lu(sym, a_lo, a_up):
    """Dense B = P A P^T from A's stored lower values and their mirrors."""
    n = sym.n
    a_lo, a_up = np.asarray(a_lo), np.asarray(a_up)
    low = np.where(sym.aflip, a_up, a_lo)
    up = np.where(sym.aflip, a_lo, a_up)
    bl, bu = np.empty_like(low), np.empty_like(up)
    bl[sym.amap] = low
    bu[sym.amap] = up
    Bd = np.zeros((n, n), dtype=np.result_type(bl, bu))
    cols = np.repeat(np.arange(n), np.diff(sym.Bcolptr))
    Bd[cols, sym.Browind] = bu
    Bd[sym.Browind, cols] = bl
    return Bd


def dense_selected_lu(sym, bdense):
    """The definition: (P A P^T)^{-1} on the pattern of L (XL), and its
    transpose, the inverse of B^T, on the same pattern (XU)."""
    return dense_selected(sym, bdense), dense_selected(sym, bdense.T)
