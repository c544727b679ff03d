"""Device numeric factorization (selinv_factor_device) against the oracle's
supernodal LDL^T, element by element on the lower part of every panel, its
log det against the oracle's, and the whole path (device factor, normalize,
selected inversion) against the oracle's selected inverse."""

import numpy as np
import pytest
import torch

from oracle import factor, selinv, symbolic
from tests._ref import maxrel, oracle_sym, oracle_x, workload
from tests.test_gpu_edge_full import _edge

CASES = [
    # (name, scale, batch, relax)
    ("C1", None, None, 0.0),
    ("C4s", None, None, 0.05),
    ("C2", 12, None, 0.0),
    ("C2", 20, None, 0.05),
    ("C3", 8, 2, 0.05),
    ("C3", 14, 2, 0.0),
    ("C5", 6, 2, 0.05),
]


def _lower_mask(sym):
    return np.concatenate([np.tril(np.ones((sym.width(K) + sym.rows[K].shape[0], sym.width(K)), bool)).reshape(-1, order="F")
                           for K in range(sym.nsuper)])


def _check_factor(w, sym, S, ldlt_dev):
    """Element-wise parity with the oracle's LDL^T to 1e-13 times the
    sensitivity of the factors: rounding differences (here the order of the
    Schur-update sums) move them by about eps * cond(B), so the bound is
    1e-13 * max(1, cond(B) / 100) (cond from numpy for n <= 3000, else the
    ratio of the largest to the smallest pivot modulus).  For n <= 3000 the
    device factors must also reproduce B: max |L D L^T - B| <= 1e-13 max |B|."""
    P = ldlt_dev.cpu().numpy()[:, S.packed_index()]
    mask = _lower_mask(sym)
    S.sync()
    ld = S.logdet()
    for l in range(w.batch):
        ref = factor.factor(sym, w.values[l])
        rf = selinv.flatten(sym, ref)
        err = np.max(np.abs(P[l][mask] - rf[mask])) / np.max(np.abs(rf[mask]))
        if w.n <= 3000:
            Bd = selinv.permuted_dense(sym, w.values[l])
            kappa = float(np.linalg.cond(Bd))
            L, D = factor.to_dense_L(sym, selinv.unflatten(sym, P[l]))
            bwd = np.max(np.abs((L * D[None, :]) @ L.T - Bd)) / np.max(np.abs(Bd))
            assert bwd <= 1e-13, bwd
        else:
            D = np.concatenate([np.diag(ref[K][:sym.width(K), :]) for K in range(sym.nsuper)])
            kappa = float(np.max(np.abs(D)) / np.min(np.abs(D)))
            bwd = float("nan")
        tol = 1e-13 * max(1.0, kappa / 100.0)
        print(f"  matrix {l}: LDL^T max-norm rel err {err:.3e} (bound {tol:.1e}, cond {kappa:.1e}); "
              f"backward error {bwd:.1e}", flush=True)
        assert err <= tol
        ref_ld = factor.logdet(sym, ref)
        if w.is_complex:
            assert abs(ld[l].real - ref_ld.real) <= 1e-11 * max(1.0, abs(ref_ld.real))
            assert abs(np.exp(1j * (ld[l].imag - ref_ld.imag)) - 1.0) < 1e-11
        else:
            assert abs(ld[l] - ref_ld) <= 1e-11 * max(1.0, abs(ref_ld))


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,batch,relax", CASES)
def test_device_factor_matches_oracle(name, scale, batch, relax):
    from paper_1604_02528_amd import SelInv

    w = workload(name, scale, batch)
    print(f"device factor case {name} scale={scale} batch={batch} relax={relax}", flush=True)
    sym = oracle_sym(name, scale, batch, relax)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
               cap=w.cap, relax=relax)
    ldlt = S.factor_device(w.values)
    _check_factor(w, sym, S, ldlt)
    # the whole path from the device factor
    S.factor(w.values, on_device=True)
    S.run()
    S.sync()
    X = S.to_host("x")
    ref = oracle_x(name, scale, batch, relax)
    for l in range(w.batch):
        err = maxrel(X[l], ref[l])
        print(f"  matrix {l}: selected inverse from the device factor, max-norm rel err {err:.3e}", flush=True)
        assert err <= (1e-9 if w.is_complex else 1e-10)
    S.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["n1", "diagonal", "dense40", "dense300", "dense70_c128", "arrow", "random_c128"])
def test_device_factor_edge_cases(name):
    """Degenerate shapes: one column, no off-diagonal rows, one dense
    supernode, a node wider than one diagonal block of the kernel (300 > 256
    columns: two supernodes), every leaf with |C(K)| = 1, a random complex
    pattern under a random permutation."""
    from paper_1604_02528_amd import SelInv

    w = _edge(name)
    print(f"device factor edge case {name} n={w.n}", flush=True)
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=0.0)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=1, cap=w.cap,
               relax=0.0)
    ldlt = S.factor_device(w.values)
    _check_factor(w, sym, S, ldlt)
    S.close()


@pytest.mark.gpu
def test_device_factor_zero_pivot_reports_column_and_batch():
    """ESINGULAR at the next selinv_sync with the first bad column of B and
    the batch index (the first pivot of the third matrix set to zero)."""
    from paper_1604_02528_amd import SelInv
    from paper_1604_02528_amd.capi import SelinvError

    w = workload("C1")
    vals = np.repeat(w.values, 3, axis=0)
    vals[2, w.colptr[int(w.perm[0])]] = 0.0
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=3, relax=0.0)
    S.factor_device(vals)
    with pytest.raises(SelinvError) as ei:
        S.sync()
    assert ei.value.status == 3 and ei.value.info == (0, 2)
    # the context recovers: a good factorization afterwards succeeds
    S.factor_device(np.repeat(w.values, 3, axis=0))
    S.sync()
    S.close()
