"""Pins of the oracle's adjoint (not in the paper; plain matrix calculus).

dloss/dA for a loss on the selected entries: G = -X W_s X, stored-value
convention (x2 off the diagonal).  Pinned by three independent routes:
the dense formula, a complex-step forward selected inversion, and central
finite differences of the C4 GMRF loss in kappa and the edge log-weights.
The node-by-node reverse sweep is pinned against them.
"""

import numpy as np
import pytest

from oracle import adjoint, factor, selinv, symbolic
from workloads import config, gmrf_2d


def setup(name="C4s", scale=None, relax=0.0):
    w = config(name, scale=scale)
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, relax=relax, cap=24)
    P = factor.factor(sym, w.values[0])
    lh, dt = factor.normalize(sym, P)
    X = selinv.alg1(sym, lh, dt)
    return w, sym, P, lh, dt, X


def random_w(sym, X, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(p.shape) for p in X]


@pytest.mark.parametrize("relax", [0.0, 0.1])
@pytest.mark.parametrize("which", ["diag", "random"])
def test_three_routes_agree(which, relax):
    w, sym, P, lh, dt, X = setup(relax=relax)
    W = adjoint.w_diag(sym, w.meta["c"]) if which == "diag" else random_w(sym, X, 3)
    g_dense = adjoint.dense_abar(sym, w.values[0], W, w.colptr, w.rowind)
    g_cs = adjoint.complex_step_abar(sym, w.values[0], W, w.colptr, w.rowind)
    S = adjoint.reverse_mode(sym, lh, dt, factor.dtilde(sym, P), X, W)
    g_rev = adjoint.abar_from_sbar(sym, S, w.colptr, w.rowind)
    scale = np.max(np.abs(g_dense))
    assert np.max(np.abs(g_cs - g_dense)) / scale < 1e-12
    assert np.max(np.abs(g_rev - g_dense)) / scale < 1e-12


def loss_theta(m, kappa, wlog, cvec):
    """The C4 loss through the oracle's forward path (factor, Alg. 1, log det)."""
    colptr, rowind, vals, edges = gmrf_2d(m, m, kappa, wlog)
    from workloads import nested_dissection
    perm = nested_dissection((m, m))
    sym = symbolic.analyze(m * m, colptr, rowind, perm)
    P = factor.factor(sym, vals[0])
    lh, dt = factor.normalize(sym, P)
    X = selinv.alg1(sym, lh, dt)
    xa = selinv.on_pattern_of_A(sym, X, colptr, rowind)
    diag_pos = colptr[:-1]
    return float(np.dot(cvec, xa[diag_pos]) + factor.logdet(sym, P))


def oracle_theta_gradient(m, kappa, wlog, cvec):
    """dloss/dkappa and dloss/dw_e from the oracle's reverse sweep plus the
    log det term (d log det Q / dQ = Q^{-1}), chained through dQ/dkappa = 2
    kappa I and dQ/dw_e = e^{w_e} (e_a - e_b)(e_a - e_b)^T."""
    colptr, rowind, vals, edges = gmrf_2d(m, m, kappa, wlog)
    from workloads import nested_dissection
    perm = nested_dissection((m, m))
    sym = symbolic.analyze(m * m, colptr, rowind, perm)
    P = factor.factor(sym, vals[0])
    lh, dt = factor.normalize(sym, P)
    X = selinv.alg1(sym, lh, dt)
    W = adjoint.w_diag(sym, cvec)
    S = adjoint.reverse_mode(sym, lh, dt, factor.dtilde(sym, P), X, W)
    gA = adjoint.abar_from_sbar(sym, S, colptr, rowind)
    xa = selinv.on_pattern_of_A(sym, X, colptr, rowind)
    cols = np.repeat(np.arange(m * m), np.diff(colptr))
    gA = gA + np.where(rowind == cols, xa, 2.0 * xa)
    diag_pos = colptr[:-1]
    g_kappa = 2.0 * kappa * np.sum(gA[diag_pos])
    pos = {(int(rowind[p]), int(cols[p])): p for p in range(rowind.shape[0])}
    g_w = np.array([np.exp(wlog[e]) * (gA[diag_pos[a]] + gA[diag_pos[b]] - gA[pos[(max(a, b), min(a, b))]])
                    for e, (a, b) in enumerate(edges)])
    return g_kappa, g_w, (colptr, rowind, vals, edges)


def test_c4s_gradient_vs_finite_differences_every_parameter():
    """The 30 x 30 GMRF of C4 (kappa = 0.5, its seeded w_e and c_i):
    loss = sum_i c_i (Q^{-1})_ii + log det Q, central differences in kappa and
    in every one of the 1,740 edge log-weights.

    The perturbed losses for w_e come from exact rank-one identities on the
    dense inverse (numpy), independent of the oracle: Q' = Q + d u u^T with
    u = e_a - e_b and d = e^{w_e +- h} - e^{w_e} gives
    diag(Q'^{-1}) = diag(X) - d (X u)^2 / (1 + d q), q = u^T X u
    (Sherman-Morrison) and log det Q' = log det Q + log(1 + d q) (matrix
    determinant lemma), so each difference loss(+h) - loss(-h) is formed
    without cancellation.  kappa and ten random edges also go through the
    oracle's own forward path."""
    w = config("C4s")
    m = w.meta["grid"][0]
    kappa, wlog, cvec = w.meta["kappa"], np.asarray(w.meta["w"]), np.asarray(w.meta["c"])
    g_kappa, g_w, (colptr, rowind, vals, edges) = oracle_theta_gradient(m, kappa, wlog, cvec)
    n = m * m
    Lq = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(colptr))
    Lq[rowind, cols] = vals[0]
    Lq[cols, rowind] = vals[0]
    X = np.linalg.inv(Lq)
    h = 1e-4
    a, b = edges[:, 0], edges[:, 1]
    XU = X[:, a] - X[:, b]                      # columns X u_e
    q = XU[a, np.arange(len(a))] - XU[b, np.arange(len(a))]
    cq = (cvec[:, None] * XU * XU).sum(axis=0)  # sum_i c_i (X u)_i^2
    we = np.exp(wlog)
    dp, dm = np.exp(wlog + h) - we, np.exp(wlog - h) - we
    diff = (-dp / (1 + dp * q) + dm / (1 + dm * q)) * cq + np.log1p(dp * q) - np.log1p(dm * q)
    fd_w = diff / (2 * h)
    err_w = np.abs(fd_w - g_w) / np.maximum(1.0, np.abs(g_w))
    assert np.max(err_w) < 1e-8, (int(np.argmax(err_w)), float(np.max(err_w)))
    hk = 1e-5
    fd_k = (loss_theta(m, kappa + hk, wlog, cvec) - loss_theta(m, kappa - hk, wlog, cvec)) / (2 * hk)
    assert abs(fd_k - g_kappa) / abs(g_kappa) < 1e-7
    rng = np.random.default_rng(4)
    for e in rng.choice(len(wlog), size=10, replace=False):
        wp, wm = wlog.copy(), wlog.copy()
        wp[e] += hk
        wm[e] -= hk
        fd = (loss_theta(m, kappa, wp, cvec) - loss_theta(m, kappa, wm, cvec)) / (2 * hk)
        assert abs(fd - g_w[e]) <= 1e-6 * max(1.0, abs(g_w[e]))


def test_c4s_gradient_vs_dense_gradient():
    """The same gradient from the dense definition G = -X diag(c) X + X."""
    w = config("C4s")
    m = w.meta["grid"][0]
    kappa, wlog, cvec = w.meta["kappa"], np.asarray(w.meta["w"]), np.asarray(w.meta["c"])
    g_kappa, g_w, (colptr, rowind, vals, edges) = oracle_theta_gradient(m, kappa, wlog, cvec)
    n = m * m
    Q = np.zeros((n, n))
    cols = np.repeat(np.arange(n), np.diff(colptr))
    Q[rowind, cols] = vals[0]
    Q[cols, rowind] = vals[0]
    X = np.linalg.inv(Q)
    G = -(X * cvec[None, :]) @ X + X
    assert abs(2 * kappa * np.trace(G) - g_kappa) <= 1e-10 * abs(g_kappa)
    a, b = edges[:, 0], edges[:, 1]
    ref = np.exp(wlog) * (G[a, a] + G[b, b] - 2 * G[a, b])
    assert np.max(np.abs(ref - g_w)) <= 1e-10 * np.max(np.abs(ref))


def _complex_setup(scale=5, relax=0.0, shift=0):
    """A small complex-symmetric shifted matrix H - z S of the C3 family."""
    w = config("C3", scale=scale, batch=4)
    vals = np.asarray(w.values[shift])
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, relax=relax, cap=24)
    return w, sym, vals


def _stored_lower_w(sym, rng):
    """Random complex stored-value gradients (top blocks: lower triangle only)."""
    W = []
    for K in range(sym.nsuper):
        s = sym.width(K)
        P = rng.standard_normal((s + sym.rows[K].shape[0], s)) + 1j * rng.standard_normal(
            (s + sym.rows[K].shape[0], s))
        P[:s, :] = np.tril(P[:s, :])
        W.append(P)
    return W


def _bilinear_loss(sym, vals, W):
    """loss(a) = sum over the stored selected entries of W * x (no conjugation:
    a holomorphic function of A's values), through the oracle's forward path."""
    P = factor.factor(sym, vals)
    lh, dt = factor.normalize(sym, P)
    X = selinv.alg1(sym, lh, dt)
    tot = 0.0 + 0.0j
    for K in range(sym.nsuper):
        s = sym.width(K)
        tot += np.sum(W[K][:s, :] * np.tril(X[K][:s, :])) + np.sum(W[K][s:, :] * X[K][s:, :])
    return tot


def test_complex_dense_abar_vs_finite_differences_real_and_imaginary():
    """Complex-symmetric A: the dense definition G = -X W_s X (plain
    transposes) is the holomorphic derivative of a bilinear loss in the
    selected entries.  Central differences of the oracle's forward path along
    a real step h and along an imaginary step i h of single stored values must
    both equal it (a holomorphic function has one complex derivative in every
    direction); a conjugated X or W_s fails the imaginary direction."""
    w, sym, vals = _complex_setup()
    rng = np.random.default_rng(11)
    W = _stored_lower_w(sym, rng)
    g = adjoint.dense_abar(sym, vals, W, w.colptr, w.rowind)
    h = 1e-6
    cols = np.repeat(np.arange(w.n), np.diff(w.colptr))
    picks = list(rng.choice(len(vals), size=6, replace=False))
    picks += [int(np.flatnonzero(w.rowind == cols)[0])]  # a diagonal value too
    for e in picks:
        for step in (h, 1j * h):
            vp, vm = vals.copy(), vals.copy()
            vp[e] += step
            vm[e] -= step
            fd = (_bilinear_loss(sym, vp, W) - _bilinear_loss(sym, vm, W)) / (2 * step)
            assert abs(fd - g[e]) <= 1e-6 * max(1.0, abs(g[e])), (e, step, fd, g[e])


@pytest.mark.parametrize("relax", [0.0, 0.1])
def test_complex_reverse_sweep_matches_dense(relax):
    """The node-by-node reverse sweep in complex arithmetic against the dense
    definition, with random complex W on every stored entry."""
    w, sym, vals = _complex_setup(scale=6, relax=relax, shift=2)
    P = factor.factor(sym, vals)
    lh, dt = factor.normalize(sym, P)
    X = selinv.alg1(sym, lh, dt)
    W = _stored_lower_w(sym, np.random.default_rng(5))
    g_dense = adjoint.dense_abar(sym, vals, W, w.colptr, w.rowind)
    S = adjoint.reverse_mode(sym, lh, dt, factor.dtilde(sym, P), X, W)
    g_rev = adjoint.abar_from_sbar(sym, S, w.colptr, w.rowind)
    assert np.iscomplexobj(g_rev)
    assert np.max(np.abs(g_rev - g_dense)) / np.max(np.abs(g_dense)) < 1e-12
