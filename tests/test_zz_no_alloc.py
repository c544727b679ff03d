"""selinv_normalize_run_noalloc (the entry point that allocates nothing: its
work area is a fixed library-owned device array) against
selinv_normalize_run with a caller-allocated work buffer: same kernels, so
the normalized panels, Dt and X must agree bit for bit.  Two calls in a row,
the second on a smaller problem, then the first context again (its tables
were replaced in the array and must be uploaded anew)."""

import numpy as np
import pytest
import torch

from tests._ref import maxrel, oracle_x, workload


def test_noalloc_rejects_a_plan_beyond_the_limit():
    """C2 at 40^3 needs far more than the fixed 64 MiB: ENOMEM with the
    bytes needed and the limit, before any device call."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload("C2")
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=0.05, device="cpu")
    with pytest.raises(capi.SelinvError) as ei:
        capi.selinv_normalize_run_noalloc(S.h, 1, 1, 1, None, None)
    assert ei.value.status == 4 and ei.value.info[1] == 64 << 20 and ei.value.info[0] > 64 << 20
    S.close()


def _setup(name, scale, batch, sched):
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale, batch)
    dt = "c128" if w.is_complex else "f64"
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=w.batch, cap=w.cap, relax=0.05, sched=sched)
    ldlt = torch.from_numpy(S.factor_host(w.values)).to("cuda")
    S._alloc(True)
    b = S._bufs
    st = torch.cuda.current_stream().cuda_stream
    for t in (b["panels"], b["x"], S.dtilde):
        t.zero_()
    capi.selinv_normalize_run(S.h, ldlt, b["panels"], b["x"], b["work"], S.dtilde, st)
    S.sync()
    ref = (b["panels"].clone(), b["x"].clone(), S.dtilde.clone())
    return w, S, ldlt, ref


def _noalloc_matches(S, ldlt, ref, label):
    from paper_1604_02528_amd import capi

    b = S._bufs
    st = torch.cuda.current_stream().cuda_stream
    for t in (b["panels"], b["x"], S.dtilde):
        t.zero_()
    print(f"  no-alloc call: {label}", flush=True)
    capi.selinv_normalize_run_noalloc(S.h, ldlt, b["panels"], b["x"], S.dtilde, st)
    S.sync()
    torch.cuda.synchronize()
    assert torch.equal(b["panels"], ref[0]), label
    assert torch.equal(b["x"], ref[1]), label
    assert torch.equal(S.dtilde, ref[2]), label


@pytest.mark.gpu
@pytest.mark.parametrize("sched", ["levels", "persistent"])
def test_noalloc_matches_work_buffer_entry_point(sched):
    big = ("C2", 12, None)
    small = ("C1", None, None)
    print(f"no-alloc case sched={sched}: C2 12^3, then C1, then C2 12^3 again, then C3 8^3 x2 (complex)", flush=True)
    wb, Sb, lb, rb = _setup(*big, sched)
    ws, Ss, ls, rs = _setup(*small, sched)
    assert Sb.sizes.work_bytes > Ss.sizes.work_bytes
    _noalloc_matches(Sb, lb, rb, "C2 12^3")
    _noalloc_matches(Ss, ls, rs, "C1 (smaller, second call)")
    _noalloc_matches(Sb, lb, rb, "C2 12^3 again (tables uploaded anew)")
    err = maxrel(Sb.to_host("x"), oracle_x(*big, 0.05))
    print(f"  C2 12^3 vs oracle {err:.3e}", flush=True)
    assert err <= 1e-10
    wc, Sc, lc, rc = _setup("C3", 8, 2, sched)
    _noalloc_matches(Sc, lc, rc, "C3 8^3 x2 complex")
    for S in (Sb, Ss, Sc):
        S.close()


@pytest.mark.gpu
def test_noalloc_lu_form():
    """The LU form through the no-alloc entry point (two panel sets, a doubled
    L_KK^{-1} scratch in the fixed array): bit for bit the work-buffer call,
    then a smaller symmetric plan and the LU plan again."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload("U3", 8, 2)
    print("no-alloc LU case: U3 8^3 x2, then C1, then U3 again", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="lu64", batch=w.batch, cap=w.cap, relax=0.05)
    ldlt = torch.from_numpy(S.factor_host(w.values)).to("cuda")
    S._alloc(False)
    b = S._bufs
    st = torch.cuda.current_stream().cuda_stream
    for t in (b["panels"], b["x"]):
        t.zero_()
    capi.selinv_normalize_run(S.h, ldlt, b["panels"], b["x"], b["work"], None, st)
    S.sync()
    ref = (b["panels"].clone(), b["x"].clone())

    def check(label):
        for t in (b["panels"], b["x"]):
            t.zero_()
        print(f"  no-alloc call: {label}", flush=True)
        capi.selinv_normalize_run_noalloc(S.h, ldlt, b["panels"], b["x"], None, st)
        S.sync()
        torch.cuda.synchronize()
        assert torch.equal(b["panels"], ref[0]), label
        assert torch.equal(b["x"], ref[1]), label

    check("U3 8^3 x2")
    ws, Ss, ls, rs = _setup("C1", None, None, "levels")
    _noalloc_matches(Ss, ls, rs, "C1 (symmetric, between the LU calls)")
    check("U3 8^3 x2 again (tables uploaded anew)")
    assert maxrel(S.to_host("x"), oracle_x("U3", 8, 2, 0.05)) <= 1e-10
    S.close()
    Ss.close()
