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


def test_normalize_run_rejects_null_buffers():
    """EINVAL (status 1) for a missing buffer, before any device work."""
    from paper_1604_02528_amd import capi

    w = workload("C1")
    S = _ctx(w, sched="levels")
    for args in [(None, 1, 1, 1), (1, None, 1, 1), (1, 1, None, 1), (1, 1, 1, None)]:
        with pytest.raises(capi.SelinvError) as ei:
            capi.selinv_normalize_run(S.h, *args, None, None)
        assert ei.value.status == 1


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


@pytest.mark.parametrize("name,scale", [("C2", None), ("C3", 14), ("C4", None)])
def test_forward_items_cover_every_tile_once(name, scale):
    """Host plan of the forward traversal: per node, the GEMM-1 items cover
    every (row tile, column tile, part) once; the R items, where present,
    cover every tile once per share and their 64-row blocks of P partition
    [0, ceil(s/64)); the D items cover the lower block pairs (in slabs for
    nodes with many row tiles); nodes with c, s <= 64 are one S item."""
    from paper_1604_02528_amd import capi

    w = workload(name, scale)
    S = _ctx(w, relax=0.05)
    it = capi.selinv_items(S.h)
    sym = S.symbolic()
    s_all = np.diff(sym["xsuper"]).astype(int)
    c_all = np.diff(sym["rowptr"]).astype(int)
    ITEM_Y, ITEM_D, ITEM_S, ITEM_G, ITEM_R = 0, 1, 2, 3, 4
    order = np.argsort(it[:, 0], kind="stable")
    bounds = np.searchsorted(it[order, 0], np.arange(len(s_all) + 1))
    n_rsplit = 0
    for K in range(len(s_all)):
        rows = it[order[bounds[K]:bounds[K + 1]]]
        s, c = int(s_all[K]), int(c_all[K])
        nr, nb = -(-c // 64), -(-s // 64)
        types = rows[:, 1]
        if c <= 64 and s <= 64:
            assert list(types[types != ITEM_G]) == [ITEM_S]
            continue
        y = rows[types == ITEM_Y]
        parts = len(y) // (nr * nb)
        assert parts >= 1 and len(y) == nr * nb * parts
        keys = {(int(a), int(b) & 0xFFFF, int(b) >> 16) for _, _, a, b in y}
        assert keys == {(a, b, p) for a in range(nr) for b in range(nb) for p in range(parts)}
        r = rows[types == ITEM_R]
        if len(r):
            rq = max(1, int(r[0, 3]) >> 24)
            nq = nb
            assert 1 <= rq <= nq and len(r) == nr * nb * rq
            got = sorted((int(a), int(b) & 0xFFFF, (int(b) >> 16) & 0xFF, max(1, int(b) >> 24)) for _, _, a, b in r)
            assert got == sorted((a, b, q, rq) for a in range(nr) for b in range(nb) for q in range(rq))
            cover = sorted(x for q in range(rq) for x in range(q * nq // rq, (q + 1) * nq // rq))
            assert cover == list(range(nq))
            n_rsplit += rq > 1
        else:
            assert parts == 1
        d = rows[types == ITEM_D]
        nsl = 4 if nr >= 4 else 1
        assert len(d) == nb * (nb + 1) // 2 * nsl
    if name == "C2":
        assert n_rsplit > 0  # the top separator chain cuts its GEMM-2 shares
