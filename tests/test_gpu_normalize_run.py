"""selinv_normalize_run (normalization in depth-range chunks on a second
stream, each chunk's traversal waiting for that chunk) against
selinv_normalize followed by selinv_run: the same kernels on the same inputs,
so the normalized panels, the D-tilde output and X must agree bit for bit; and
X against the oracle."""

import numpy as np
import pytest
import torch

from tests._ref import maxrel, oracle_x, workload

CASES = [("C2", None, "levels"), ("C2", 12, "levels"), ("C3", 8, "levels"), ("C4", None, "levels"),
         ("C2", 12, "persistent"), ("C3", None, "levels")]


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,sched", CASES)
def test_normalize_run_matches_separate_calls(name, scale, sched):
    """The full C3 (32 shifts) plan has five normalization chunks; the oracle
    check runs on the smaller cases (the full C3 is checked against the oracle
    in test_gpu_edge_full.py)."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale)
    print(f"normalize_run case {name} scale={scale} sched={sched} batch={w.batch}", flush=True)
    dt = "c128" if w.is_complex else "f64"
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=w.batch, cap=w.cap, relax=0.05, sched=sched)
    full = name == "C3" and scale is None
    if full:
        assert len(capi.selinv_items(S.h, 3)) >= 3
    ldlt = torch.from_numpy(S.factor_host(w.values)).to("cuda")
    S._alloc(True)
    st = torch.cuda.current_stream().cuda_stream
    b = S._bufs
    for t in (b["panels"], b["x"], S.dtilde):  # alignment gaps between panels are never written
        t.zero_()
    capi.selinv_normalize(S.h, ldlt, b["panels"], b["work"], S.dtilde, st)
    capi.selinv_run(S.h, b["panels"], b["x"], b["work"], st)
    S.sync()
    ref_p, ref_x, ref_d = b["panels"].clone(), b["x"].clone(), S.dtilde.clone()
    for rep in range(2):  # the second call reuses the context's stream and events
        for t in (b["panels"], b["x"], S.dtilde):
            t.zero_()
        capi.selinv_normalize_run(S.h, ldlt, b["panels"], b["x"], b["work"], S.dtilde, st)
        S.sync()
        torch.cuda.synchronize()
        for what, got, ref in (("panels", b["panels"], ref_p), ("x", b["x"], ref_x), ("dtilde", S.dtilde, ref_d)):
            if not torch.equal(got, ref):
                g64, r64 = got.view(torch.float64), ref.view(torch.float64)
                bad = torch.nonzero(g64 != r64).flatten()
                d = (g64 - r64).abs().max().item()
                pytest.fail(f"{what} differ in call {rep}: {bad.numel()} of {g64.numel()} doubles, max |diff| {d:.3e}, "
                            f"first at {bad[:8].tolist()}, nan in got {int(torch.isnan(g64).sum())}")
    if not full:
        err = maxrel(S.to_host("x"), oracle_x(name, scale, None, 0.05))
        print(f"  max-norm rel err vs oracle {err:.3e}", flush=True)
        assert err <= (1e-9 if w.is_complex else 1e-10)
    S.close()


def _poison_lds():
    """Leave inf / NaN in the LDS of every CU: a device factorization whose
    first pivot is zero (its diagonal-block, L_{C,K} and Schur-update kernels
    stage non-finite values through LDS), 16 matrices at once."""
    from paper_1604_02528_amd import SelInv
    from paper_1604_02528_amd.capi import SelinvError

    w = workload("C2", 20)
    vals = np.repeat(w.values, 16, axis=0)
    vals[:, w.colptr[int(w.perm[0])]] = 0.0
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=16, cap=w.cap, relax=0.05)
    S.factor_device(vals)
    with pytest.raises(SelinvError):
        S.sync()
    S.close()


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,batch", [("C2", None, None), ("C4", None, None), ("C3", 14, 2)])
def test_stale_lds_contents_do_not_reach_results(name, scale, batch):
    """Kernels leave their LDS contents behind for the next kernel on the CU.
    After a launch that leaves inf / NaN there, normalize + run and the
    overlapped normalize_run (many s = 1 nodes, normalized by the
    single-wavefront kernel) must still match the oracle: no kernel may read
    an LDS word it did not write, not even to multiply it by zero."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale, batch)
    print(f"stale-LDS case {name} scale={scale} batch={batch}", flush=True)
    ref = oracle_x(name, scale, batch, 0.05)
    dt = "c128" if w.is_complex else "f64"
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=w.batch, cap=w.cap, relax=0.05)
    ldlt = torch.from_numpy(S.factor_host(w.values)).to("cuda")
    S._alloc(True)
    st = torch.cuda.current_stream().cuda_stream
    b = S._bufs
    for call in ("separate", "overlapped"):
        _poison_lds()
        if call == "separate":
            capi.selinv_normalize(S.h, ldlt, b["panels"], b["work"], S.dtilde, st)
            capi.selinv_run(S.h, b["panels"], b["x"], b["work"], st)
        else:
            capi.selinv_normalize_run(S.h, ldlt, b["panels"], b["x"], b["work"], S.dtilde, st)
        S.sync()
        err = maxrel(S.to_host("x"), ref)
        print(f"  {call}: max-norm rel err vs oracle {err:.3e}", flush=True)
        assert err <= (1e-9 if w.is_complex else 1e-10)
    S.close()
