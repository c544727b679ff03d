"""Oracle adjoint of selected inversion (test infrastructure only).

Not in the paper.  Let a loss depend on the stored lower selected entries
x_pq = (A^{-1})_pq, (p, q) in the pattern of L, p >= q, and let W hold
dloss/dx_pq.  With W_s = (W + W^T)/2 (off-diagonal halved and mirrored) and
X = A^{-1}:

    dloss = <W_s, dX> = -<W_s, X dA X> = <G, dA>,   G = -X W_s X.

A stored lower value a_ij stands for both (i, j) and (j, i), so

    dloss/da_ij = 2 G_ij (i != j),   dloss/da_ii = G_ii      (stored-value convention).

``dense_abar`` is that definition.  ``complex_step_abar`` obtains G on the
pattern of L from the forward selected inversion alone: for real symmetric A,
Im(sel((A + i h W_s)^{-1})) / h = -X W_s X + O(h^2) (the chordal pattern of L
is unchanged by the perturbation).  ``reverse_mode`` is the node-by-node
reverse sweep the device implements (R1 leaves to root through Alg. 1, R2 per
node, R3 root to leaves through the block LDL^T); it is pinned against the two
definitions above, never the other way round.

Conventions inside ``reverse_mode``: "full" adjoints Xi satisfy
dloss = sum over all (i, j) of Xi_ij dM_ij for a symmetric matrix M; a stored
lower value's gradient is Xi_ij + Xi_ji = 2 Xi_ij off the diagonal.
"""

from __future__ import annotations

import numpy as np

from . import selinv as _sel
from . import factor as _fac


def xbar_full_from_stored(sym, W):
    """Full-convention panels from stored-value gradients W (panel layout).

    The top block's lower triangle (diagonal included) and the bottom block
    are the stored values; the top block's strict upper triangle is ignored.
    """
    out = []
    for K in range(sym.nsuper):
        s = sym.width(K)
        P = np.array(W[K], copy=True)
        top = np.tril(P[:s, :])
        full = 0.5 * (top + top.T)  # diagonal kept, off-diagonal halved & mirrored
        P[:s, :] = full
        P[s:, :] = 0.5 * P[s:, :]
        out.append(P)
    return out


def _lower_to_full_dense(sym, panels):
    """Dense symmetric matrix (B indexing) from panels whose top block is full."""
    n = sym.n
    M = np.zeros((n, n), dtype=panels[0].dtype)
    for K in range(sym.nsuper):
        f, l1 = int(sym.xsuper[K]), int(sym.xsuper[K + 1])
        s = l1 - f
        P = panels[K]
        M[f:l1, f:l1] = P[:s, :]
        C = sym.rows[K]
        if C.shape[0]:
            M[np.ix_(C, np.arange(f, l1))] = P[s:, :]
            M[np.ix_(np.arange(f, l1), C)] = P[s:, :].T
    return M


def dense_abar(sym, avals, W, colptr, rowind):
    """Definition: stored-value gradient on A's pattern, G = -X W_s X."""
    Bd = _sel.permuted_dense(sym, avals)
    X = np.linalg.inv(Bd)
    Ws = _lower_to_full_dense(sym, xbar_full_from_stored(sym, W))
    G = -X @ Ws @ X
    return g_on_pattern_of_A(sym, G, colptr, rowind)


def g_on_pattern_of_A(sym, G, colptr, rowind):
    """Stored-value convention on A's lower pattern from a dense full-convention G (B indexing)."""
    n = sym.n
    ip = np.empty(n, dtype=np.int64)
    ip[sym.perm] = np.arange(n)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    i = ip[np.asarray(rowind)]
    j = ip[cols]
    g = G[i, j]
    return np.where(i == j, g, 2.0 * g)


def complex_step_abar(sym, avals, W, colptr, rowind, h=1e-30):
    """Stored-value gradient from one complex-step forward selected inversion.

    Perturb B = P A P^T by i h W_s on the pattern of L (the pattern is chordal,
    so the perturbed matrix has the same symbolic factorization), run the
    forward oracle (factor + Alg. 1) in complex arithmetic and read
    G = Im(X(h)) / h = -X W_s X + O(h^2) on the pattern of L.
    """
    Wfull = xbar_full_from_stored(sym, W)
    avals = np.asarray(avals)
    bvals = np.empty(avals.shape[0], dtype=np.complex128)
    bvals[sym.amap] = avals
    panels = _fac.assemble(sym, bvals)
    for K in range(sym.nsuper):
        s = sym.width(K)
        pert = np.array(Wfull[K], dtype=np.complex128)
        pert[:s, :] = np.tril(pert[:s, :])
        panels[K] = panels[K] + 1j * h * pert
    panels = _fac.factor_panels(sym, panels)
    lhat, dtinv = _fac.normalize(sym, panels)
    X = _sel.alg1(sym, lhat, dtinv)
    G_panels = [np.imag(P) / h for P in X]
    # G is known on the pattern of L, which contains A's pattern
    return abar_from_sbar(sym, G_panels, colptr, rowind)


def reverse_mode(sym, lhat, dtinv, dtil, X, W):
    """Reverse sweep through Alg. 1 and the block LDL^T (full conventions).

    R1, K = 1..N (leaves first; every descendant of K has pushed into K):
        Tbar = Xi_KK,  Ybar = 2 Xi_{C,K},  Zbar = Ybar - Lhat Tbar
        Lhatbar_K = -X_{C,C} Zbar - X_{C,K} Tbar,  Ebar_K = Tbar
        Xi_{C,C} += -sym(Zbar Lhat^T)          (into the ancestors)
    R2: Dtbar_K = -E Ebar_K E,   E = Dt^{-1}
    R3, K = N..1 (root first), Sbar the adjoint of the Schur complements:
        Lhatbar_K += -2 Sbar_{C,C} Lhat Dt,   Dtbar_K += -Lhat^T Sbar_{C,C} Lhat
        Sbar_{C,K} = (Lhatbar_K E) / 2 (full convention),
        Dtbar_K += -Lhat^T Lhatbar_K E,   Sbar_KK = sym(Dtbar_K)
    Returns the Sbar panels (full convention; top block full symmetric).
    """
    Xi = xbar_full_from_stored(sym, W)
    # keep only the lower triangle of top blocks while accumulating
    acc = []
    for K in range(sym.nsuper):
        s = sym.width(K)
        P = Xi[K].copy()
        P[:s, :] = np.tril(P[:s, :])
        acc.append(P)
    lbar = [None] * sym.nsuper
    ebar = [None] * sym.nsuper
    xs = sym.xsuper
    for K in range(sym.nsuper):
        s = sym.width(K)
        C = sym.rows[K]
        c = C.shape[0]
        top = acc[K][:s, :]
        Tbar = top + np.tril(top, -1).T
        ebar[K] = Tbar
        if c == 0:
            lbar[K] = np.zeros((0, s), dtype=Tbar.dtype)
            continue
        Ybar = 2.0 * acc[K][s:, :]
        L = lhat[K]
        Y = X[K][s:, :]
        Zbar = Ybar - L @ Tbar
        G = _sel.gather_cc(sym, X, K)
        lbar[K] = -G @ Zbar - Y @ Tbar
        Gbar = -Zbar @ L.T
        Gs = 0.5 * (Gbar + Gbar.T)
        for g in range(sym.seg_ptr[K], sym.seg_ptr[K + 1]):
            J = int(sym.seg_super[g])
            st = int(sym.seg_start[g])
            en = int(sym.seg_start[g + 1]) if g + 1 < sym.seg_ptr[K + 1] else c
            pos = sym.posarr[sym.seg_posoff[g]: sym.seg_posoff[g] + (c - st)]
            aa, bb = np.nonzero(np.arange(st, c)[:, None] >= np.arange(st, en)[None, :])
            acc[J][pos[aa], C[st + bb] - xs[J]] += Gs[st + aa, st + bb]
    S = [None] * sym.nsuper
    for K in reversed(range(sym.nsuper)):
        s = sym.width(K)
        C = sym.rows[K]
        c = C.shape[0]
        E = dtinv[K]
        Dt = dtil[K]
        L = lhat[K]
        Dtbar = -E @ ebar[K] @ E
        P = np.zeros((s + c, s), dtype=E.dtype)
        if c:
            Sb = _sel.gather_cc(sym, S, K)
            Lb = lbar[K] - 2.0 * Sb @ L @ Dt
            Dtbar = Dtbar - L.T @ Sb @ L - L.T @ Lb @ E
            P[s:, :] = 0.5 * (Lb @ E)
        P[:s, :] = 0.5 * (Dtbar + Dtbar.T)
        S[K] = P
    return S


def abar_from_sbar(sym, S, colptr, rowind):
    """Stored-value gradient on A's pattern from full-convention Sbar panels."""
    vals = _sel.on_pattern_of_A(sym, S, colptr, rowind)
    n = sym.n
    ip = np.empty(n, dtype=np.int64)
    ip[sym.perm] = np.arange(n)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    i = ip[np.asarray(rowind)]
    j = ip[cols]
    return np.where(i == j, vals, 2.0 * vals)


def w_diag(sym, cvec):
    """Stored-value W for the loss sum_i c_i (A^{-1})_ii (original index i)."""
    W = []
    ip = np.empty(sym.n, dtype=np.int64)
    ip[sym.perm] = np.arange(sym.n)
    cB = np.empty(sym.n)
    cB[ip] = cvec
    for K in range(sym.nsuper):
        f, l1 = int(sym.xsuper[K]), int(sym.xsuper[K + 1])
        s = l1 - f
        P = np.zeros((s + sym.rows[K].shape[0], s))
        P[np.arange(s), np.arange(s)] = cB[f:l1]
        W.append(P)
    return W
