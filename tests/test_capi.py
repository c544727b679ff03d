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
        capi.selinv_backward(S.h, 1, 1, 1, 1, None, 1, 1, None)
    assert ei.value.status == 6


@pytest.mark.parametrize("name,scale,relax,dense", [("C2", 10, 0.05, 0), ("C2", 12, 0.0, 65), ("C4s", None, 0.0, 0),
                                                   ("C4", None, 0.05, 0)])
def test_adjoint_items_cover_every_node_once_per_sweep(name, scale, relax, dense):
    """Host plan of the reverse sweep (selinv_items(which=1), launch order):
    every node is visited exactly once in R1 and once in R3, either as the
    whole-node small kernel or as a full set of tile items (T, Z, L, F, D0
    over its s x s / c x s blocks, SC over the lower block pairs of c x c, G
    iff it has a dense X_{C,C} buffer; M, LB, N, DF, SG likewise in R3); R1
    visits a node only after all of its children are complete and R3 only
    after its parent is complete."""
    from paper_1604_02528_amd import capi

    w = workload(name, scale)
    S = _ctx(w, relax=relax, dense_min_c=dense)
    seq = capi.selinv_items(S.h, 1)
    sym = S.symbolic()
    ns = sym["nsuper"]
    s_all = np.diff(sym["xsuper"]).astype(int)
    c_all = np.diff(sym["rowptr"]).astype(int)
    sparent = sym["sparent"]
    R1 = {0: "T", 1: "G", 2: "Z", 3: "L", 4: "SC", 5: "F", 6: "D0"}
    R3 = {7: "SG", 8: "M", 9: "LB", 10: "N", 11: "DF"}
    # split the sequence into the two sweeps: R1 types / tiny R1 first, then R3
    is_r1 = np.isin(seq[:, 1], list(R1) + [12])
    n1 = int(is_r1.sum())
    assert is_r1[:n1].all() and not is_r1[n1:].any()
    for sweep, types, tiny in ((seq[:n1], R1, 12), (seq[n1:], R3, 13)):
        first, last = np.full(ns, -1), np.full(ns, -1)
        for pos, (K, t, a, b) in enumerate(sweep):
            if first[K] < 0:
                first[K] = pos
            last[K] = pos
        assert (first >= 0).all(), "a node is missing from a sweep"
        for K in range(ns):
            rows = sweep[first[K]:last[K] + 1]
            rows = rows[rows[:, 0] == K]
            s, c = int(s_all[K]), int(c_all[K])
            nb, nr = -(-s // 64), -(-c // 64)
            got = sorted(map(tuple, rows[:, 1:].tolist()))
            if (rows[:, 1] == tiny).any():
                assert got == [(tiny, 0, 0)]
                continue
            want = []
            sq = [(a, b) for a in range(nb) for b in range(nb)]
            tiles = [(a, b) for b in range(nb) for a in range(nr)]
            lower_c = [(a, b) for a in range(nr) for b in range(a + 1)]
            lower_s = [(a, b) for a in range(nb) for b in range(a + 1)]
            dense_buf = sum(1 for r in rows if r[1] in (1, 7)) > 0
            if types is R1:
                want += [(0,) + p for p in sq] + [(5,) + p for p in sq] + [(6,) + p for p in sq]
                want += [(2,) + p for p in tiles] + [(3,) + p for p in tiles] + [(4,) + p for p in lower_c]
                if dense_buf:
                    want += [(1,) + p for p in lower_c]
            else:
                want += [(8,) + p for p in tiles] + [(9,) + p for p in tiles] + [(10,) + p for p in tiles]
                want += [(11,) + p for p in lower_s]
                if dense_buf:
                    want += [(7,) + p for p in lower_c]
            assert got == sorted(want), (K, s, c)
        # order: R1 after every child is complete, R3 after the parent is complete
        for K in range(ns):
            P = int(sparent[K])
            if P < 0:
                continue
            if types is R1:
                assert last[K] < first[P]
            else:
                assert last[P] < first[K]


def test_adjoint_items_which_is_checked():
    from paper_1604_02528_amd import capi

    S = _ctx(workload("C1"))
    with pytest.raises(capi.SelinvError) as ei:
        capi.selinv_items(S.h, 5)
    assert ei.value.status == 1


@pytest.mark.parametrize("name,scale", [("C2", None), ("C3", 14)])
def test_level_launch_list(name, scale):
    """selinv_items(which = 2): the level schedule's launches run the etree
    depths root first, each depth's phases in order (gathers, GEMM-1 tiles,
    GEMM-2 and split sums, diagonal blocks, then the single-wavefront nodes),
    and together hold every work item once."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
               cap=w.cap, relax=0.05, device="cpu", adjoint=False)
    L = capi.selinv_items(S.h, 2)
    items = capi.selinv_items(S.h, 0)
    assert L[:, 1].sum() == len(items)
    assert np.all(np.diff(L[:, 3]) >= 0) and L[0, 3] == 0 and L[-1, 3] == S.symbolic()["depth"] - 1
    phase = {3: 0, 0: 1, 4: 2, 5: 2, 1: 3, 2: 3}  # item type -> phase
    for d in np.unique(L[:, 3]):
        rows = L[L[:, 3] == d]
        ph = [4 if k == 1 else phase[t] for k, t in zip(rows[:, 0], rows[:, 2])]
        assert ph == sorted(ph), (d, rows)
        assert set(rows[:, 0]) <= {0, 1, 2, 5, 6}
        # each launch runs the kernel of its phase: gathers (5), GEMM-2 shares (6)
        for k, t in zip(rows[:, 0], rows[:, 2]):
            if k == 5:
                assert t == 3
            if k == 6:
                assert t in (4, 5)
            if t == 3:
                assert k == 5
            if t in (4, 5):
                assert k == 6


def _drop_entry(colptr, rowind, vals, j, k):
    """The pattern without entry k of column j."""
    p = colptr[j] + k
    cp = colptr.copy()
    cp[j + 1:] -= 1
    return cp, np.delete(rowind, p), np.delete(vals, p, axis=1)


def test_pattern_errors_report_the_column():
    """EPATTERN (status 2) with the offending column in error_info(0): a
    duplicate row, a row index out of range, a missing diagonal, an entry
    above the diagonal, a colptr that is not monotone."""
    from paper_1604_02528_amd import SelInv
    from paper_1604_02528_amd.capi import SelinvError

    w = workload("C1")
    n = w.n
    j = 17
    cases = {}
    r = w.rowind.copy()
    r[w.colptr[j] + 2] = r[w.colptr[j] + 1]  # duplicate
    cases["duplicate"] = (w.colptr, r, j)
    r = w.rowind.copy()
    r[w.colptr[n - 40 + 1] - 1] = n  # last entry of a column past the matrix
    cases["out_of_range"] = (w.colptr, r, n - 40)
    cp, r, _ = _drop_entry(w.colptr, w.rowind, w.values, j, 0)  # the diagonal
    cases["missing_diagonal"] = (cp, r, j)
    r = w.rowind.copy()
    r[w.colptr[j]] = j - 1  # an upper-triangle entry in front of the diagonal
    cases["upper_entry"] = (w.colptr, r, j)
    cp = w.colptr.copy()
    cp[j + 1] = cp[j]  # empty column
    cases["empty_column"] = (cp, w.rowind, j)
    for what, (cp, r, col) in cases.items():
        with pytest.raises(SelinvError) as ei:
            SelInv(n, cp, r, w.perm, device="cpu")
        assert ei.value.status == 2 and ei.value.info[0] == col, what


def test_absurd_batch_is_enomem_and_unknown_dtype_unsupported():
    """ENOMEM (4) before anything of the batch's size is allocated: the item
    ids of the whole batch must fit in int32.  EUNSUPPORTED (7) for a dtype
    the library does not have."""
    from paper_1604_02528_amd import capi

    w = workload("C1")
    o = capi.selinv_default_opts()
    o.batch = 1 << 30
    with pytest.raises(capi.SelinvError) as ei:
        capi.selinv_analyze(w.n, w.colptr, w.rowind, w.perm, o)
    assert ei.value.status == 4
    o = capi.selinv_default_opts()
    o.dtype = 5
    with pytest.raises(capi.SelinvError) as ei:
        capi.selinv_analyze(w.n, w.colptr, w.rowind, w.perm, o)
    assert ei.value.status == 7


def test_adjoint_scratch_is_optional():
    """opts.adjoint < 0 leaves the adjoint's three panel-layout and three
    s x s arrays per matrix out of the work area; nothing before them moves
    (the forward path's part of the work area is the same)."""
    from paper_1604_02528_amd import SelInv

    for name, scale, dt in [("C1", None, "f64"), ("C3", 8, "c128")]:
        w = workload(name, scale)
        sb = 16 if dt == "c128" else 8
        a = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=w.batch, device="cpu")
        b = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=dt, batch=w.batch, device="cpu", adjoint=False)
        assert a.sizes.tables_bytes == b.sizes.tables_bytes
        extra = a.sizes.work_bytes - b.sizes.work_bytes
        pan = sb * w.batch * a.panel_elems
        sq = int(a.sizes.dtilde_bytes)  # the Dt blocks: batch * sum of s^2 scalars, padded
        assert 3 * pan + 2 * sq < extra <= 3 * pan + 3 * sq + 6 * 256
        a.close()
        b.close()


def test_default_options_are_the_measured_fastest():
    from paper_1604_02528_amd import capi

    o = capi.selinv_default_opts()
    assert o.sched == capi.SCHED_LEVELS and o.relax == 0.05 and o.max_super == 256


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
    ITEM_Y, ITEM_D, ITEM_S, ITEM_G, ITEM_R, ITEM_P = 0, 1, 2, 3, 4, 5
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
        r = rows[(types == ITEM_R) | (types == ITEM_P)]
        assert not ((types == ITEM_R).any() and (types == ITEM_P).any())
        if (types == ITEM_P).any():  # GEMM-2 deferred: dense buffer, unsplit
            assert (types == ITEM_G).any() and parts == 1
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


# --------------------------------------------------------------------------
# tune tables (selinv_opts.tune_cache)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("choice", ["gather", "dense_fused", "dense_ydense", "dense_ydense128"])
def test_tune_table_choices_shape_the_plan(choice):
    """A table forcing one choice on every bucket: 'gather' leaves no dense
    X_{C,C} buffer (no G items); 'dense_fused' gives every node with c > 64 a
    buffer and keeps GEMM-2 in the GEMM-1 tiles of the general item kernel;
    'dense_ydense' runs them in the GEMM-1 kernel of the dense nodes, with the
    GEMM-2 share still fused (no P items); 'dense_ydense128' moves the GEMM-2
    of unsplit dense nodes into P items (the 128 x 128 tiles have none).
    Every supernode is covered by an entry."""
    from paper_1604_02528_amd import capi
    from tests._tune import forced_table, remove

    w = workload("C2", 16)
    path = forced_table(choice, "f64")
    try:
        S = _ctx(w, relax=0.05, tune_cache=path)
        sym = S.symbolic()
        it = capi_items(S)
        assert sym["tuned_nodes"] == sym["nsuper"]
        c_all = np.diff(sym["rowptr"])
        types = it[:, 1]
        dense_nodes = set(it[types == 3, 0].tolist())
        big = {K for K in range(sym["nsuper"]) if c_all[K] > 64}
        if choice == "gather":
            assert not dense_nodes and not (types == 5).any()
        else:
            assert dense_nodes == big
            assert (types == 5).any() == (choice == "dense_ydense128")
        # the 128 x 128 tiles replace the 64 x 64 dense-buffer launches (kind 4 for kind 2)
        kinds = set(capi.selinv_items(S.h, 2)[:, 0].tolist())
        assert (4 in kinds) == (choice == "dense_ydense128")
        assert (2 in kinds) == (choice == "dense_ydense")
    finally:
        remove(path)


def capi_items(S):
    from paper_1604_02528_amd import capi

    return capi.selinv_items(S.h, 0)


def test_tune_table_other_keys_are_ignored_and_split_follows_the_table():
    from tests._tune import forced_table, remove

    w = workload("C2", 16)
    for kw in ({"arch": "gfx000"}, {"rocm": "0.0.0"}):
        path = forced_table("gather", "f64", **kw)
        try:
            assert _ctx(w, relax=0.05, tune_cache=path).symbolic()["tuned_nodes"] == 0
        finally:
            remove(path)
    path = forced_table("gather", "c128")  # another dtype
    try:
        assert _ctx(w, relax=0.05, tune_cache=path).symbolic()["tuned_nodes"] == 0
    finally:
        remove(path)
    path = forced_table("dense_ydense", "f64", split_min_k=-1)  # never split
    try:
        it = capi_items(_ctx(w, relax=0.05, tune_cache=path))
        y = it[it[:, 1] == 0]
        assert (y[:, 3] >> 16 == 0).all()
    finally:
        remove(path)


def test_malformed_tune_table_is_einval(tmp_path):
    from paper_1604_02528_amd.capi import SelinvError

    w = workload("C1")
    cases = {"not_json.json": "{entries: [", "no_format.json": '{"entries": []}',
             "bad_format.json": '{"format": "other", "entries": []}',
             "bad_tile.json": '{"format": "selinv-tune-1", "entries": [{"tile": 96}]}'}
    for name, text in cases.items():
        p = tmp_path / name
        p.write_text(text)
        with pytest.raises(SelinvError) as ei:
            _ctx(w, tune_cache=str(p))
        assert ei.value.status == 1, name
    with pytest.raises(SelinvError) as ei:
        _ctx(w, tune_cache=str(tmp_path / "missing.json"))
    assert ei.value.status == 1


def test_tune_key_names_this_build():
    from paper_1604_02528_amd import capi

    k = capi.selinv_tune_key()
    assert k.startswith("arch=gfx950 rocm=")


@pytest.mark.parametrize("name,scale,chunks", [("C2", None, 2), ("C3", None, 3), ("C5", 16, 2)])
def test_normalization_chunks(name, scale, chunks):
    """selinv_items(which = 3): selinv_normalize_run's normalization chunks
    start at the first level launch, then at increasing level launches and
    etree depths, and together hold every normalization work entry; the
    pipelined plan of the full C3 (32 shifts) has more than the two chunks
    (top depths, rest) of a small plan."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=w.dtype, batch=w.batch, cap=w.cap, relax=0.05,
               device="cpu", adjoint=False)
    N = capi.selinv_items(S.h, 3)
    L = capi.selinv_items(S.h, 2)
    assert len(N) >= chunks
    assert N[0, 0] == 0 and N[0, 1] == 0
    assert np.all(np.diff(N[:, 0]) > 0) and np.all(np.diff(N[:, 1]) > 0)
    assert np.all(N[:, 0] < len(L))
    assert np.all(L[N[:, 0], 3] == N[:, 1])  # a chunk starts at the first launch of its depth
    assert np.all(N[:, 2] >= 0)
    capi.selinv_check_plan(S.h)
    with pytest.raises(capi.SelinvError):
        capi.selinv_items(S.h, 5)
