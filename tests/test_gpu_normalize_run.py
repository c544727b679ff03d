"""selinv_normalize_run (normalization overlapped with the traversal of the
top etree depths on a second stream) against selinv_normalize followed by
selinv_run: the same kernels on the same inputs, so the normalized panels, the
D-tilde output and X must agree bit for bit; and X against the oracle."""

import numpy as np
import pytest
import torch

from tests._ref import maxrel, oracle_x, workload

CASES = [("C2", None, "levels"), ("C2", 12, "levels"), ("C3", 8, "levels"), ("C4", None, "levels"),
         ("C2", 12, "persistent")]


@pytest.mark.gpu
@pytest.mark.parametrize("name,scale,sched", CASES)
def test_normalize_run_matches_separate_calls(name, scale, sched):
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale)
    print(f"normalize_run case {name} scale={scale} sched={sched} batch={w.batch}", flush=True)
    dt = "c128" if w.is_complex else "f64"
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=w.batch, cap=w.cap, relax=0.05, sched=sched)
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
        assert torch.equal(b["panels"], ref_p), rep
        assert torch.equal(b["x"], ref_x), rep
        assert torch.equal(S.dtilde, ref_d), rep
    err = maxrel(S.to_host("x"), oracle_x(name, scale, None, 0.05))
    print(f"  max-norm rel err vs oracle {err:.3e}", flush=True)
    assert err <= (1e-9 if w.is_complex else 1e-10)
    S.close()
