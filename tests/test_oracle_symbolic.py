"""Pins of the oracle's symbolic analysis against brute force and definitions.

Section 2.1: supernodes are maximal sets of contiguous columns of L with the
same structure below the block and a dense lower-triangular diagonal block,
optionally capped; Eq. (newset): C(K) = {I > K : L_{I,K} != 0}.
"""

import numpy as np
import pytest

from oracle import symbolic
from workloads import config, random_pattern


def dense_pattern(n, colptr, rowind, perm):
    P = np.zeros((n, n), dtype=bool)
    ip = np.empty(n, dtype=np.int64)
    ip[perm] = np.arange(n)
    cols = np.repeat(np.arange(n), np.diff(colptr))
    i, j = ip[rowind], ip[cols]
    P[i, j] = True
    P[j, i] = True
    return P


def random_case(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 61))
    dens = float(rng.uniform(0.03, 0.3))
    colptr, rowind, vals = random_pattern(n, dens, rng)
    perm = rng.permutation(n).astype(np.int64)
    return n, colptr, rowind, perm


@pytest.mark.parametrize("seed", range(40))
@pytest.mark.parametrize("cap", [256, 3])
def test_etree_colcount_structure_vs_brute_force(seed, cap):
    n, colptr, rowind, perm = random_case(seed)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=cap)
    Ld = symbolic.dense_symbolic(dense_pattern(n, colptr, rowind, perm))
    # column counts and elimination tree by definition: parent(j) = min{i > j : L_ij != 0}
    assert np.array_equal(sym.colcount, Ld.sum(axis=0))
    for j in range(n):
        below = np.flatnonzero(Ld[j + 1:, j]) + j + 1
        assert sym.parent[j] == (below[0] if below.size else -1)
    xs = sym.xsuper
    for K in range(sym.nsuper):
        f, l = xs[K], xs[K + 1] - 1
        C = np.flatnonzero(Ld[l + 1:, l]) + l + 1
        assert np.array_equal(sym.rows[K], C)
        # supernode definition: every column has structure [j..l] U C(K)
        for j in range(f, l + 1):
            expect = np.concatenate([np.arange(j, l + 1), C])
            assert np.array_equal(np.flatnonzero(Ld[:, j]), expect)
        assert l - f + 1 <= cap
        # maximality: the next column could not have joined
        if l + 1 < n:
            s_next = np.flatnonzero(Ld[:, l + 1])
            same = (sym.parent[l] == l + 1 and np.array_equal(np.flatnonzero(Ld[:, l]), np.concatenate([[l], s_next])))
            assert (not same) or (l - f + 1 == cap)
        # supernodal etree: parent supernode owns min C(K)
        if C.size:
            assert sym.sparent[K] == sym.col2super[C[0]]
            # fill property: C(K) inside cols(P) U C(P)
            Pn = sym.sparent[K]
            allowed = set(range(xs[Pn], xs[Pn + 1])) | set(sym.rows[Pn].tolist())
            assert set(C.tolist()) <= allowed
        else:
            assert sym.sparent[K] == -1


@pytest.mark.parametrize("seed", range(25))
@pytest.mark.parametrize("relax", [0.0, 0.1])
def test_ancestor_maps_point_at_the_right_rows(seed, relax):
    n, colptr, rowind, perm = random_case(seed)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=8, relax=relax)
    xs = sym.xsuper
    for K in range(sym.nsuper):
        C = sym.rows[K]
        c = C.shape[0]
        segs = range(sym.seg_ptr[K], sym.seg_ptr[K + 1])
        owners = [int(sym.seg_super[g]) for g in segs]
        assert owners == sorted(set(sym.col2super[C].tolist()))
        for g in segs:
            J = int(sym.seg_super[g])
            st = int(sym.seg_start[g])
            assert sym.col2super[C[st]] == J and (st == 0 or sym.col2super[C[st - 1]] != J)
            pos = sym.posarr[sym.seg_posoff[g]: sym.seg_posoff[g] + c - st]
            panel_rows = np.concatenate([np.arange(xs[J], xs[J + 1]), sym.rows[J]])
            assert np.array_equal(panel_rows[pos], C[st:])


@pytest.mark.parametrize("seed", range(25))
@pytest.mark.parametrize("relax", [0.05, 0.3])
def test_relaxed_partition_respects_zero_budget(seed, relax):
    n, colptr, rowind, perm = random_case(seed)
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=16, relax=relax)
    Ld = symbolic.dense_symbolic(dense_pattern(n, colptr, rowind, perm))
    xs = sym.xsuper
    for K in range(sym.nsuper):
        f, l = xs[K], xs[K + 1] - 1
        C = sym.rows[K]
        assert np.array_equal(C, np.flatnonzero(Ld[l + 1:, l]) + l + 1)
        entries = 0
        nnz = 0
        for j in range(f, l + 1):
            trap = set(range(j, l + 1)) | set(C.tolist())
            struct = set(np.flatnonzero(Ld[:, j]).tolist())
            assert struct <= trap  # relaxed structure contains the true one
            entries += len(trap)
            nnz += len(struct)
        assert entries - nnz <= relax * entries + 1e-9
        for j in range(f, l):
            assert sym.parent[j] == j + 1  # merged only along etree chains


def test_relax_zero_is_the_maximal_partition():
    w = config("C2", scale=10)
    a = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, relax=0.0)
    b = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, relax=1e-12)
    assert np.array_equal(a.xsuper, b.xsuper)


def test_c1_top_separator():
    """C1: ND puts the x = 15 plane (31 points) last; the root supernode holds it.

    The plane's Schur complement is dense, so its 31 columns share one
    supernode (which also absorbs the chained columns of the y = 15 half-plane
    separator below it: 46 columns in all)."""
    w = config("C1")
    sym = symbolic.analyze(w.n, w.colptr, w.rowind, w.perm)
    last = w.perm[-31:]
    assert np.all(last % 31 == 15)
    assert sym.xsuper[-1] - sym.xsuper[-2] == 46
    assert sym.rows[-1].shape[0] == 0
