"""Oracle symbolic analysis (test infrastructure; never imported by the product).

Follows Section 2.1 of the paper: a structurally symmetric pattern, its
elimination tree, and the supernode partition ("a maximal set of contiguous
columns of L with the same nonzero structure below the last column and a dense
lower triangle in the diagonal block", optionally capped in size).  The sets
C(K) = {I > K : L_{I,K} != 0} are Eq. (newset).

Everything here works on the permuted matrix B = P A P^T (perm is new -> old),
lower triangle, CSC.

Parity pin: tests/test_oracle_symbolic.py compares against dense boolean
symbolic elimination on random patterns and checks the supernode definition
and the fill property directly.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Symbolic:
    n: int
    perm: np.ndarray          # new -> old
    Bcolptr: np.ndarray       # lower CSC of B = P A P^T
    Browind: np.ndarray
    amap: np.ndarray          # A entry e -> position of that entry in B's CSC arrays
    parent: np.ndarray        # column elimination tree (-1 = root)
    colcount: np.ndarray      # nnz of each column of L, diagonal included
    xsuper: np.ndarray        # supernode K owns columns xsuper[K] .. xsuper[K+1]-1
    col2super: np.ndarray
    sparent: np.ndarray       # supernodal etree (-1 = root)
    rows: list                # rows[K] = C(K), sorted, int64
    # canonical ancestor index maps (see ancestor_maps)
    seg_ptr: np.ndarray
    seg_super: np.ndarray
    seg_start: np.ndarray
    seg_posoff: np.ndarray
    posarr: np.ndarray
    aflip: np.ndarray = None  # A entry e lands in B's strict upper triangle (ip[row] < ip[col])

    @property
    def nsuper(self) -> int:
        return int(self.xsuper.shape[0] - 1)

    def width(self, K) -> int:
        return int(self.xsuper[K + 1] - self.xsuper[K])

    def nnzL(self) -> int:
        return int(self.colcount.sum())

    def flops(self, complex_values=False) -> float:
        """Selected-inversion work sum_K 2 c^2 s + 2 c s^2 (x4 for complex)."""
        tot = 0.0
        for K in range(self.nsuper):
            s = self.width(K)
            c = len(self.rows[K])
            tot += 2.0 * c * c * s + 2.0 * c * s * s
        return tot * (4.0 if complex_values else 1.0)


def permute_lower(n, colptr, rowind, perm):
    """Lower CSC of B = P A P^T and the map from A's entries to B's entries.

    B[i, j] = A[perm[i], perm[j]]; an A entry (r, c) lands at
    (max(ip[r], ip[c]), min(ip[r], ip[c])) with ip the inverse permutation.
    The last result flags the entries with ip[r] < ip[c]: their value is that
    of B's upper triangle, so B's lower entry there is its transpose
    (conjugated for a Hermitian A).
    """
    colptr = np.asarray(colptr, dtype=np.int64)
    rowind = np.asarray(rowind, dtype=np.int64)
    perm = np.asarray(perm, dtype=np.int64)
    ip = np.empty(n, dtype=np.int64)
    ip[perm] = np.arange(n, dtype=np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(colptr))
    i = ip[rowind]
    j = ip[cols]
    hi = np.maximum(i, j)
    lo = np.minimum(i, j)
    order = np.lexsort((hi, lo))
    Bcolptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(Bcolptr, lo + 1, 1)
    Bcolptr = np.cumsum(Bcolptr)
    Browind = hi[order]
    amap = np.empty_like(order)
    amap[order] = np.arange(order.shape[0], dtype=np.int64)
    return Bcolptr, Browind, amap, i < j


def analyze(n, colptr, rowind, perm=None, cap=256, relax=0.0):
    """Full symbolic analysis of the pattern (Section 2.1).

    ``relax`` is the explicit-zero budget of the supernode partition (see
    below); 0 gives the maximal supernodes of the definition, capped at
    ``cap`` columns.
    """
    if perm is None:
        perm = np.arange(n, dtype=np.int64)
    Bcolptr, Browind, amap, aflip = permute_lower(n, colptr, rowind, perm)

    # Column structures by the column-structure theorem: struct(L_j) is the
    # lower pattern of column j of B together with struct(L_c) \ {c} for every
    # child c of j in the elimination tree; parent(j) = min(struct(L_j) \ {j}).
    parent = np.full(n, -1, dtype=np.int64)
    colcount = np.zeros(n, dtype=np.int64)
    pending = {}
    # Supernodes are closed greedily from the lowest column.  Column j+1 joins
    # the open supernode [f, j] iff parent(j) = j+1, the merged supernode has
    # at most ``cap`` columns, and the merged block [f, j+1] x ([f, j+1] U
    # C(j+1)) holds at most relax * (its size) structural zeros.  With
    # relax = 0 this says colcount(i) = colcount(i+1) + 1 along the chain:
    # struct(L_j) = {j} U struct(L_{j+1}), identical structure below the block
    # and a dense diagonal triangle, i.e. the paper's (maximal, capped)
    # supernode.  With relax > 0 the partition is relaxed along etree chains;
    # the extra entries are exact zeros of L and exact entries of A^{-1}.
    starts = [0]
    rows = []
    prev_struct = None
    run_cc = 0  # sum of colcount over the open supernode
    for j in range(n):
        parts = [Browind[Bcolptr[j]:Bcolptr[j + 1]]]
        parts.extend(pending.pop(j, []))
        st = np.unique(np.concatenate(parts))
        if st[0] != j:
            raise ValueError(f"missing diagonal in column {j}")
        colcount[j] = st.shape[0]
        if st.shape[0] > 1:
            parent[j] = st[1]
            pending.setdefault(int(st[1]), []).append(st[1:])
        if j > 0:
            f = starts[-1]
            size = j - f + 1
            joins = parent[j - 1] == j and size <= cap
            if joins:
                entries = size * (size + 1) // 2 + size * (int(colcount[j]) - 1)
                zeros = entries - (run_cc + int(colcount[j]))
                joins = zeros <= relax * entries
            if not joins:
                rows.append(prev_struct[1:].copy())
                starts.append(j)
                run_cc = 0
        run_cc += int(colcount[j])
        prev_struct = st
    rows.append(prev_struct[1:].copy())
    xsuper = np.array(starts + [n], dtype=np.int64)
    nsuper = xsuper.shape[0] - 1
    col2super = np.repeat(np.arange(nsuper, dtype=np.int64), np.diff(xsuper))
    sparent = np.full(nsuper, -1, dtype=np.int64)
    for K in range(nsuper):
        if rows[K].shape[0] > 0:
            sparent[K] = col2super[rows[K][0]]
    maps = ancestor_maps(xsuper, col2super, rows)
    return Symbolic(n, np.asarray(perm, dtype=np.int64), Bcolptr, Browind, amap, parent,
                    colcount, xsuper, col2super, sparent, rows, *maps, aflip=aflip)


def panel_row(xsuper, rows, J, r):
    """Row position of global row r inside supernode J's panel.

    The panel of J has s_J + c_J rows: J's own columns first, then C(J).
    """
    f, l = xsuper[J], xsuper[J + 1] - 1
    if f <= r <= l:
        return int(r - f)
    k = int(np.searchsorted(rows[J], r))
    if k >= rows[J].shape[0] or rows[J][k] != r:
        raise AssertionError("row outside the structure of the ancestor")
    return int(l - f + 1 + k)


def ancestor_maps(xsuper, col2super, rows):
    """Canonical ancestor index maps.

    For supernode K with C = C(K) (sorted), the ancestors that own a column of
    C are visited in increasing order; J_t owns C[start_t .. end_t).  For each
    such J_t the map holds the panel-row positions, inside J_t's panel, of the
    rows C[start_t:], i.e. every row of C(K) at or above J_t's first column.
    These are exactly the entries of A^{-1}_{C,C} needed by step 3 of Alg. 1:
    the block of column segment t lives in J_t's panel, column C[b] - first(J_t).

    Flat layout: segments of K are seg_ptr[K] .. seg_ptr[K+1]-1; segment g has
    owner seg_super[g], start index seg_start[g] (into C(K)) and its positions
    at posarr[seg_posoff[g] : seg_posoff[g] + c_K - seg_start[g]].
    """
    nsuper = xsuper.shape[0] - 1
    seg_ptr = [0]
    seg_super, seg_start, seg_posoff = [], [], []
    pos_chunks = []
    off = 0
    for K in range(nsuper):
        C = rows[K]
        c = C.shape[0]
        if c:
            owners = col2super[C]
            brk = np.flatnonzero(np.diff(owners)) + 1
            starts = np.concatenate([[0], brk])
            for st in starts:
                J = int(owners[st])
                sub = C[st:]
                f, l = xsuper[J], xsuper[J + 1] - 1
                inblk = sub <= l
                pos = np.empty(sub.shape[0], dtype=np.int64)
                pos[inblk] = sub[inblk] - f
                above = sub[~inblk]
                k = np.searchsorted(rows[J], above)
                if above.shape[0] and (np.any(k >= rows[J].shape[0])
                                       or np.any(rows[J][np.minimum(k, rows[J].shape[0] - 1)] != above)):
                    raise AssertionError("fill property violated")
                pos[~inblk] = (l - f + 1) + k
                seg_super.append(J)
                seg_start.append(int(st))
                seg_posoff.append(off)
                pos_chunks.append(pos)
                off += pos.shape[0]
        seg_ptr.append(len(seg_super))
    posarr = (np.concatenate(pos_chunks) if pos_chunks else np.zeros(0, dtype=np.int64))
    return (np.array(seg_ptr, dtype=np.int64), np.array(seg_super, dtype=np.int64),
            np.array(seg_start, dtype=np.int64), np.array(seg_posoff, dtype=np.int64),
            posarr.astype(np.int64))


def dense_symbolic(Bdense_pattern):
    """Brute-force symbolic elimination on a dense boolean lower pattern.

    Eliminating column k fills (i, j) for every pair i > j > k with
    L_ik and L_jk nonzero.  Returns the boolean pattern of L.
    """
    P = np.array(Bdense_pattern, dtype=bool)
    P = np.tril(P | P.T)
    n = P.shape[0]
    for k in range(n):
        nz = np.flatnonzero(P[k + 1:, k]) + k + 1
        if nz.size:
            P[np.ix_(nz, nz)] |= True
            P = np.tril(P)
    np.fill_diagonal(P, True)
    return P
