"""GPU adjoint (selinv_backward) against the oracle's gradient.

The reference for small cases is the plain definition dloss/dA = G on A's
pattern (stored-value convention), G = -X W_s X with a dense inverse; for the
full C4 GMRF it is the oracle's reverse sweep, itself pinned against the dense
definition, a complex-step derivative and finite differences (CPU tests).
"""

import numpy as np
import pytest
import torch

from oracle import adjoint, factor, selinv
from tests._ref import maxrel, oracle_sym, workload

TOL = 1e-9


def random_w(sym, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((sym.width(K) + sym.rows[K].shape[0], sym.width(K))) for K in range(sym.nsuper)]


def gpu_abar(w, relax, W_panels, sym, dense=0, split=0):
    from paper_1604_02528_amd import SelInv

    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=1, cap=w.cap, relax=relax, sched="levels",
               dense_min_c=dense, split_min_k=split)
    S.factor(w.values, want_dtilde=True)
    S.run()
    xbar = torch.zeros((1, S.panel_elems), dtype=torch.float64)
    xbar[0, torch.from_numpy(S.packed_index())] = torch.from_numpy(selinv.flatten(sym, W_panels))
    xbar = xbar.to("cuda")
    abar = S.backward(xbar)
    S.sync()
    return abar.cpu().numpy()[0]


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,dense", [("C4s", None, 0), ("C1", None, 0), ("C2", 8, 0), ("C2", 12, 0),
                                              ("C2", 12, 65)], ids=["C4s", "C1", "C2_8", "C2_12", "C2_12_dense"])
def test_backward_matches_dense_gradient(name, scale, dense):
    w = workload(name, scale, None)
    print(f"adjoint case {name} scale={scale} dense={dense}", flush=True)
    sym = oracle_sym(name, scale, None, 0.0)
    W = random_w(sym, 11)
    got = gpu_abar(w, 0.0, W, sym, dense=dense)
    ref = adjoint.dense_abar(sym, w.values[0], W, w.colptr, w.rowind)
    err = maxrel(got, ref)
    print(f"  max-norm rel err {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.gpu
def test_backward_c4_loss_vs_oracle_reverse_sweep():
    """C4 (200 x 200 GMRF): loss = sum_i c_i (Q^{-1})_ii."""
    w = workload("C4", None, None)
    print("adjoint case C4 (full) diag loss", flush=True)
    sym = oracle_sym("C4", None, None, 0.0)
    P = factor.factor(sym, w.values[0])
    lh, dt = factor.normalize(sym, P)
    X = selinv.alg1(sym, lh, dt)
    W = adjoint.w_diag(sym, w.meta["c"])
    S = adjoint.reverse_mode(sym, lh, dt, factor.dtilde(sym, P), X, W)
    ref = adjoint.abar_from_sbar(sym, S, w.colptr, w.rowind)
    got = gpu_abar(w, 0.0, W, sym)
    err = maxrel(got, ref)
    print(f"  max-norm rel err {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.gpu
def test_autograd_function_c4s_loss():
    """torch.autograd through SelInvFunction: loss = sum c_i X_ii + log det Q on
    the 30 x 30 GMRF, against the dense definition of both gradients."""
    from paper_1604_02528_amd import SelInv, SelInvFunction

    w = workload("C4s", None, None)
    sym = oracle_sym("C4s", None, None, 0.0)
    c = torch.from_numpy(np.asarray(w.meta["c"], dtype=np.float64)).to("cuda")
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=1, cap=w.cap, sched="levels")
    vals = torch.from_numpy(np.ascontiguousarray(w.values)).to("cuda").requires_grad_(True)
    x, logdet = SelInvFunction.apply(vals, S)
    diag = torch.from_numpy(np.asarray(w.colptr[:-1], dtype=np.int64)).to("cuda")  # diagonal first in each column
    loss = (c * x[0, diag]).sum() + logdet.sum()
    loss.backward()
    got = vals.grad.cpu().numpy()[0]
    # dense definition: W = diag(c) for the trace part, plus d logdet/da = X (x2 off the diagonal)
    Wd = adjoint.w_diag(sym, w.meta["c"])
    ref = adjoint.dense_abar(sym, w.values[0], Wd, w.colptr, w.rowind)
    Xd = np.linalg.inv(selinv.permuted_dense(sym, w.values[0]))
    ref = ref + adjoint.g_on_pattern_of_A(sym, Xd, w.colptr, w.rowind)
    err = maxrel(got, ref)
    print(f"autograd C4s: max-norm rel err {err:.3e}", flush=True)
    assert err <= TOL
