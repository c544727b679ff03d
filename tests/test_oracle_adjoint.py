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


def test_c4_gradient_vs_finite_differences():
    """loss = sum_i c_i (Q^{-1})_ii + log det Q; dQ/dkappa = 2 kappa I, dQ/dw_e = e^{w_e} L_e."""
    m = 12
    rng = np.random.default_rng(4)
    nedge = 2 * m * (m - 1)
    wlog = rng.normal(0.0, 0.3, size=nedge)
    cvec = rng.uniform(0.0, 1.0, size=m * m)
    kappa = 0.5
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
    # log det Q contributes X (stored convention: x2 off the diagonal)
    xa = selinv.on_pattern_of_A(sym, X, colptr, rowind)
    cols = np.repeat(np.arange(m * m), np.diff(colptr))
    gA = gA + np.where(rowind == cols, xa, 2.0 * xa)
    # chain rule to theta (stored values: diagonal entries and one entry per edge)
    diag_pos = colptr[:-1]
    g_kappa = 2.0 * kappa * np.sum(gA[diag_pos])
    pos = {}
    for p in range(rowind.shape[0]):
        pos[(int(rowind[p]), int(cols[p]))] = p
    g_w = np.empty(nedge)
    for e, (a, b) in enumerate(edges):
        hi, lo = max(a, b), min(a, b)
        we = np.exp(wlog[e])
        g_w[e] = we * (gA[diag_pos[a]] + gA[diag_pos[b]] - gA[pos[(hi, lo)]])
    h = 1e-5
    fd_k = (loss_theta(m, kappa + h, wlog, cvec) - loss_theta(m, kappa - h, wlog, cvec)) / (2 * h)
    assert abs(fd_k - g_kappa) / abs(g_kappa) < 1e-7
    for e in rng.choice(nedge, size=12, replace=False):
        wp, wm = wlog.copy(), wlog.copy()
        wp[e] += h
        wm[e] -= h
        fd = (loss_theta(m, kappa, wp, cvec) - loss_theta(m, kappa, wm, cvec)) / (2 * h)
        assert abs(fd - g_w[e]) <= 1e-6 * max(1.0, abs(g_w[e]))
