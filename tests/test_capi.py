"""C ABI: every declared symbol is exported; host-only entry points and error paths."""

import os
import re

import numpy as np
import pytest

from tests._ref import oracle_sym, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "selinv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(selinv_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1604_02528_amd import capi

    lib = capi.load()
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(capi.EXPORTED) <= set(names)


def _ctx(w, relax=0.0, **kw):
    from paper_1604_02528_amd import SelInv

    return SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
                  cap=w.cap, relax=relax, device="cpu", **kw)


def test_malformed_pattern_is_rejected():
    from paper_1604_02528_amd.capi import SelinvError

    w = workload("C1")
    rowind = w.rowind.copy()
    j = 5
    rowind[w.colptr[j] + 1], rowind[w.colptr[j] + 2] = rowind[w.colptr[j] + 2], rowind[w.colptr[j] + 1]
    from paper_1604_02528_amd import SelInv

    with pytest.raises(SelinvError) as ei:
        SelInv(w.n, w.colptr, rowind, w.perm, device="cpu")
    assert ei.value.status == 2 and ei.value.info[0] == j
    bad_perm = w.perm.copy()
    bad_perm[3] = bad_perm[4]
    with pytest.raises(SelinvError) as ei:
        SelInv(w.n, w.colptr, w.rowind, bad_perm, device="cpu")
    assert ei.value.status == 2
    with pytest.raises(SelinvError) as ei:
        SelInv(w.n, w.colptr, w.rowind, w.perm, cap=300, device="cpu")
    assert ei.value.status == 1


def test_zero_pivot_reports_column_and_batch():
    from paper_1604_02528_amd.capi import SelinvError

    w = workload("C1")
    vals = np.repeat(w.values, 3, axis=0)
    vals[2, w.colptr[int(w.perm[0])]] = 0.0  # first pivot of the third matrix
    from paper_1604_02528_amd import SelInv

    S = SelInv(w.n, w.colptr, w.rowind, w.perm, batch=3, device="cpu")
    with pytest.raises(SelinvError) as ei:
        S.factor_host(vals)
    assert ei.value.status == 3 and ei.value.info == (0, 2)
    vals[2, w.colptr[int(w.perm[0])]] = np.nan
    with pytest.raises(SelinvError):
        S.factor_host(vals)


def test_run_before_factor_is_a_state_error():
    from paper_1604_02528_amd import capi

    w = workload("C1")
    S = _ctx(w)
    with pytest.raises(capi.SelinvError) as ei:
        capi.selinv_run(S.h, 1, 1, 1, None)
    assert ei.value.status == 6


def test_sizes_are_consistent():
    w = workload("C3", 6, 3)
    S = _ctx(w, relax=0.05)
    s = S.sizes
    sym = S.symbolic()
    assert s.panels_bytes >= 3 * sym["panel_elems"] * 16 and s.panels_bytes % 256 == 0
    assert s.abar_bytes >= 3 * w.nnz * 16
    assert s.work_bytes > 0


def test_backward_before_factor_is_a_state_error():
    from paper_1604_02528_amd import capi

    w = workload("C1")
    S = _ctx(w)
    with pytest.raises(capi.SelinvError) as ei:
        capi.selinv_backward(S.h, 1, 1, 1, 1, 1, 1, None)
    assert ei.value.status == 6


def test_adjoint_items_cover_every_node_once_per_sweep():
    """Host plan of the reverse sweep: R1 visits depths deepest first, R3 root
    first; every node gets its diagonal-block items once in each sweep."""
    from paper_1604_02528_amd import capi

    w = workload("C2", 10)
    S = _ctx(w, relax=0.05)
    it = capi.selinv_items(S.h)  # forward items, for the node count
    sym = S.symbolic()
    ns = sym["nsuper"]
    assert it.shape[1] == 4 and it[:, 0].max() == ns - 1
