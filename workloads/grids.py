"""Grid matrices, the nested-dissection permutation and the named workloads.

Conventions (shared by every consumer):

* A grid point (x, y[, z]) has original index p = x + nx*(y + ny*z), x fastest.
* Matrices are symmetric (real), complex-symmetric (A = A^T, no conjugation)
  or, for the H3 family, Hermitian (A = A^H; ``meta["dtype"] == "h128"``),
  or, for the U3 family, unsymmetric with a symmetric pattern
  (``meta["dtype"] == "lu64"``): ``values`` is then [B, 2 nnz], the stored
  lower values A(r, c) followed by their mirrors A(c, r).
  Only the lower triangle is stored: CSC with int64 ``colptr``/``rowind``,
  rows ascending in each column, so the diagonal entry opens every column.
* ``values`` has shape [B, nnz] (B matrices that share one pattern, the batched
  shifts of a pole expansion); B = 1 for a single matrix.
* ``perm`` maps new -> old: the analysed matrix is B = P A P^T with
  B[i, j] = A[perm[i], perm[j]].  The paper permutes symmetrically without
  looking at values (Section 4); the geometric nested dissection below is that
  permutation for grid problems.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C4s", "C5", "H3", "U3")


@dataclass
class Workload:
    name: str
    n: int
    colptr: np.ndarray
    rowind: np.ndarray
    values: np.ndarray
    perm: np.ndarray
    cap: int = 256
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowind.shape[0])

    @property
    def batch(self) -> int:
        return int(self.values.shape[0])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.values)

    @property
    def is_hermitian(self) -> bool:
        return self.meta.get("dtype") == "h128"

    @property
    def is_lu(self) -> bool:
        return self.meta.get("dtype") == "lu64"

    @property
    def lower_values(self):
        """[B, nnz] stored lower values (for LU workloads the first half)."""
        return self.values[:, :self.nnz] if self.is_lu else self.values

    @property
    def upper_values(self):
        """[B, nnz] their mirrors A(c, r) (LU workloads; the same as lower_values otherwise)."""
        return self.values[:, self.nnz:] if self.is_lu else self.values

    @property
    def dtype(self) -> str:
        """The library's dtype name: "f64", "c128" (complex-symmetric) or "h128" (Hermitian)."""
        if self.is_lu:
            return "lu64"
        return "h128" if self.is_hermitian else ("c128" if self.is_complex else "f64")


# --------------------------------------------------------------------------
# assembly helpers
# --------------------------------------------------------------------------

def _lower_csc(n, rows, cols, vals):
    """Sort (row, col, val) triplets with row >= col into lower CSC.

    ``vals`` is [B, m].  Triplets must be unique (the generators never emit a
    duplicate); this is checked.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if np.any(rows < cols):
        raise ValueError("triplets must lie in the lower triangle")
    order = np.lexsort((rows, cols))
    r, c = rows[order], cols[order]
    key = c * n + r
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate entries")
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(colptr, c + 1, 1)
    colptr = np.cumsum(colptr)
    vals = np.asarray(vals)
    if vals.ndim == 1:
        vals = vals[None, :]
    return colptr, r.copy(), np.ascontiguousarray(vals[:, order])


def _grid_index(shape):
    """Original index array of a grid, indexed [z][y][x] (x fastest)."""
    n = int(np.prod(shape))
    rev = tuple(reversed(shape))
    return np.arange(n, dtype=np.int64).reshape(rev)


def _axis_edges(shape, offset):
    """All (a, b) pairs with b = a + offset on the grid, a lexicographic.

    ``offset`` is a per-axis step tuple (dx, dy[, dz]); steps are -1, 0 or 1.
    """
    idx = _grid_index(shape)
    nd = len(shape)
    sl_a, sl_b = [], []
    for ax in reversed(range(nd)):  # array axes are (z, y, x)
        d = offset[ax]
        if d == 0:
            sl_a.append(slice(None))
            sl_b.append(slice(None))
        elif d > 0:
            sl_a.append(slice(0, shape[ax] - d))
            sl_b.append(slice(d, None))
        else:
            sl_a.append(slice(-d, None))
            sl_b.append(slice(0, shape[ax] + d))
    a = idx[tuple(sl_a)].ravel()
    b = idx[tuple(sl_b)].ravel()
    return a, b


def _unit_offsets(nd):
    out = []
    for ax in range(nd):
        off = [0] * nd
        off[ax] = 1
        out.append(tuple(off))
    return out


def _ghost_points(shape):
    """Points that miss a grid neighbour, one entry per missing neighbour.

    Enumerated axis by axis (x, y, z), low face then high face, points in
    lexicographic order inside a face.
    """
    idx = _grid_index(shape)
    nd = len(shape)
    pts = []
    for ax in range(nd):
        arr_ax = nd - 1 - ax
        for side in (0, shape[ax] - 1):
            sl = [slice(None)] * nd
            sl[arr_ax] = side
            pts.append(idx[tuple(sl)].ravel())
    return np.concatenate(pts)


def _weighted_graph_laplacian(n, a, b, w, ghost_pts=None, g=None, diag_extra=0.0):
    """sum_e w_e (e_a - e_b)(e_a - e_b)^T + sum_ghost g e_p e_p^T + diag_extra I.

    ``w`` and ``g`` are [B, m] arrays (B matrices with one pattern).
    """
    w = np.atleast_2d(w)
    B = w.shape[0]
    diag = np.zeros((B, n), dtype=w.dtype) + diag_extra
    for k in range(B):
        np.add.at(diag[k], a, w[k])
        np.add.at(diag[k], b, w[k])
        if ghost_pts is not None:
            np.add.at(diag[k], ghost_pts, np.atleast_2d(g)[k])
    hi = np.maximum(a, b)
    lo = np.minimum(a, b)
    rows = np.concatenate([np.arange(n, dtype=np.int64), hi])
    cols = np.concatenate([np.arange(n, dtype=np.int64), lo])
    vals = np.concatenate([diag, -w], axis=1)
    return _lower_csc(n, rows, cols, vals)


# --------------------------------------------------------------------------
# nested dissection
# --------------------------------------------------------------------------

def nested_dissection(shape):
    """Geometric nested-dissection permutation (new -> old) of a grid.

    Rule: a box whose longest extent is below 3 is a leaf and is numbered
    lexicographically (x fastest).  Otherwise split along the longest axis
    (lowest axis index on a tie) at the plane lo + len//2, number the first
    half, then the second half, then the separator plane (lexicographic).  One
    plane separates both 7-point and 27-point stencils.  No postorder.
    """
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    idx = _grid_index(shape)
    pieces = []

    def emit(lo, hi):
        sl = tuple(slice(lo[ax], hi[ax]) for ax in reversed(range(nd)))
        pieces.append(idx[sl].ravel())

    stack = [("box", tuple([0] * nd), shape)]
    # iterative post-order: (box) expands to [first, second, plane] emitted in
    # that order; a stack of pending actions keeps recursion depth bounded.
    while stack:
        kind, lo, hi = stack.pop()
        ext = [hi[ax] - lo[ax] for ax in range(nd)]
        if min(ext) <= 0:
            continue
        if kind == "plane":
            emit(lo, hi)
            continue
        m = max(ext)
        if m < 3:
            emit(lo, hi)
            continue
        d = ext.index(m)
        mid = lo[d] + ext[d] // 2
        first_hi = list(hi)
        first_hi[d] = mid
        second_lo = list(lo)
        second_lo[d] = mid + 1
        plane_lo = list(lo)
        plane_lo[d] = mid
        plane_hi = list(hi)
        plane_hi[d] = mid + 1
        # pushed in reverse so that they pop as first, second, plane
        stack.append(("plane", tuple(plane_lo), tuple(plane_hi)))
        stack.append(("box", tuple(second_lo), hi))
        stack.append(("box", lo, tuple(first_hi)))
    perm = np.concatenate(pieces).astype(np.int64)
    assert perm.shape[0] == int(np.prod(shape))
    return perm


# --------------------------------------------------------------------------
# matrix families
# --------------------------------------------------------------------------

def laplacian_2d_dirichlet(nx, ny, sigma):
    """Unscaled 5-point Dirichlet Laplacian (diagonal 4, off-diagonal -1) + sigma I."""
    shape = (nx, ny)
    n = nx * ny
    a_list, b_list = [], []
    for off in _unit_offsets(2):
        a, b = _axis_edges(shape, off)
        a_list.append(a)
        b_list.append(b)
    a = np.concatenate(a_list)
    b = np.concatenate(b_list)
    w = np.ones((1, a.shape[0]))
    ghost = _ghost_points(shape)
    g = np.ones((1, ghost.shape[0]))
    return _weighted_graph_laplacian(n, a, b, w, ghost, g, diag_extra=sigma)


def weighted_laplacian_3d(shape, sigma, rng=None, wlo=0.5, whi=1.5):
    """sum_e w_e (e_a-e_b)(e_a-e_b)^T + sum_ghost g e_a e_a^T + sigma I on a 3-D grid.

    7-point couplings.  Edge weights (axis x, y, z in turn, lexicographic) are
    drawn first from U[wlo, whi], then one ghost weight per missing neighbour
    from the same stream.  ``rng=None`` gives all weights 1 (the textbook
    Dirichlet Laplacian, which has a closed-form spectrum).
    """
    shape = tuple(shape)
    n = int(np.prod(shape))
    a_list, b_list = [], []
    for off in _unit_offsets(3):
        a, b = _axis_edges(shape, off)
        a_list.append(a)
        b_list.append(b)
    a = np.concatenate(a_list)
    b = np.concatenate(b_list)
    ghost = _ghost_points(shape)
    if rng is None:
        w = np.ones((1, a.shape[0]))
        g = np.ones((1, ghost.shape[0]))
    else:
        w = rng.uniform(wlo, whi, size=a.shape[0])[None, :]
        g = rng.uniform(wlo, whi, size=ghost.shape[0])[None, :]
    return _weighted_graph_laplacian(n, a, b, w, ghost, g, diag_extra=sigma)


def magnetic_laplacian_3d(shape, rng, wlo=0.5, whi=1.5):
    """Hermitian 7-point operator sum_e w_e u_e u_e^H + sum_ghost g e_a e_a^T,
    u_e = e_a - e^{-i theta_e} e_b, on a 3-D grid (a discrete magnetic
    Laplacian, positive semidefinite).

    Edges as in weighted_laplacian_3d (a < b, b = a + a unit step); the stored
    lower entry is A[b, a] = -w_e e^{-i theta_e} (so A[a, b] = -w_e e^{i theta_e}).
    Draw order: edge weights U[wlo, whi], ghost weights, then phases
    theta_e ~ U[-pi, pi].
    """
    shape = tuple(shape)
    n = int(np.prod(shape))
    a_list, b_list = [], []
    for off in _unit_offsets(3):
        a, b = _axis_edges(shape, off)
        a_list.append(a)
        b_list.append(b)
    a = np.concatenate(a_list)
    b = np.concatenate(b_list)
    ghost = _ghost_points(shape)
    w = rng.uniform(wlo, whi, size=a.shape[0])
    g = rng.uniform(wlo, whi, size=ghost.shape[0])
    theta = rng.uniform(-np.pi, np.pi, size=a.shape[0])
    diag = np.zeros(n)
    np.add.at(diag, a, w)
    np.add.at(diag, b, w)
    np.add.at(diag, ghost, g)
    hi = np.maximum(a, b)
    lo = np.minimum(a, b)
    off = -w * np.exp(-1j * theta)  # at (hi, lo) = (b, a)
    rows = np.concatenate([np.arange(n, dtype=np.int64), hi])
    cols = np.concatenate([np.arange(n, dtype=np.int64), lo])
    vals = np.concatenate([diag.astype(np.complex128), off])[None, :]
    return _lower_csc(n, rows, cols, vals)


def convection_diffusion_3d(shape, rng, wlo=0.5, whi=1.5, pmax=0.5):
    """Unsymmetric 7-point operator with a symmetric pattern: for each grid
    edge (a, b), b = a + a unit step, A(a, b) = -w_e (1 - p_e) and
    A(b, a) = -w_e (1 + p_e) (a diffusion weight w_e ~ U[wlo, whi] and a
    convection share p_e ~ U[-pmax, pmax], as a central difference gives);
    the diagonal is sum_e w_e (1 + |p_e|) over the point's edges plus one
    ghost weight per missing neighbour, so every row is strictly diagonally
    dominant.  Returns (colptr, rowind, lower, upper): the stored lower values
    A(r, c), r >= c, and their mirrors A(c, r).  Draw order: w, p, ghosts."""
    shape = tuple(shape)
    n = int(np.prod(shape))
    a_list, b_list = [], []
    for off in _unit_offsets(3):
        a, b = _axis_edges(shape, off)
        a_list.append(a)
        b_list.append(b)
    a = np.concatenate(a_list)
    b = np.concatenate(b_list)
    ghost = _ghost_points(shape)
    w = rng.uniform(wlo, whi, size=a.shape[0])
    p = rng.uniform(-pmax, pmax, size=a.shape[0])
    g = rng.uniform(wlo, whi, size=ghost.shape[0])
    diag = np.zeros(n)
    np.add.at(diag, a, w * (1 + np.abs(p)))
    np.add.at(diag, b, w * (1 + np.abs(p)))
    np.add.at(diag, ghost, g)
    rows = np.concatenate([np.arange(n, dtype=np.int64), b])  # b > a: (b, a) is the lower entry
    cols = np.concatenate([np.arange(n, dtype=np.int64), a])
    low = np.concatenate([diag, -w * (1 + p)])   # A(b, a)
    up = np.concatenate([diag, -w * (1 - p)])    # A(a, b)
    colptr, rowind, both = _lower_csc(n, rows, cols, np.stack([low, up]))
    return colptr, rowind, both[0], both[1]


def gmrf_2d(nx, ny, kappa, w):
    """GMRF precision kappa^2 I + sum_e exp(w_e)(e_a-e_b)(e_a-e_b)^T (Neumann, no ghosts).

    ``w`` holds one log-weight per edge (axis x edges, then axis y edges).
    Returns (colptr, rowind, values, edges) where ``edges`` is [m, 2] (a, b).
    """
    shape = (nx, ny)
    n = nx * ny
    a_list, b_list = [], []
    for off in _unit_offsets(2):
        a, b = _axis_edges(shape, off)
        a_list.append(a)
        b_list.append(b)
    a = np.concatenate(a_list)
    b = np.concatenate(b_list)
    we = np.exp(np.asarray(w, dtype=np.float64))[None, :]
    colptr, rowind, vals = _weighted_graph_laplacian(n, a, b, we, None, None,
                                                     diag_extra=kappa * kappa)
    return colptr, rowind, vals, np.stack([a, b], axis=1)


def stencil27_complex(shape, rng, margin=3.0):
    """Complex-symmetric 27-point operator with a diagonally dominant real part.

    Off-diagonal a_ab = a_ba: Re ~ U[-1, 0], Im ~ U[-0.1, 0.1] (one value per
    unordered neighbour pair; the 13 forward directions in lexicographic order
    of (dz, dy, dx), pairs lexicographic inside a direction).  Diagonal:
    Re = sum_b |a_ab| + margin, Im ~ U[-0.1, 0.1].  Draw order: all real
    parts, all imaginary parts, then the diagonal imaginary parts.
    """
    shape = tuple(shape)
    n = int(np.prod(shape))
    a_list, b_list = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dz, dy, dx) <= (0, 0, 0):
                    continue
                a, b = _axis_edges(shape, (dx, dy, dz))
                a_list.append(a)
                b_list.append(b)
    a = np.concatenate(a_list)
    b = np.concatenate(b_list)
    m = a.shape[0]
    re = rng.uniform(-1.0, 0.0, size=m)
    im = rng.uniform(-0.1, 0.1, size=m)
    off = re + 1j * im
    absum = np.zeros(n)
    np.add.at(absum, a, np.abs(off))
    np.add.at(absum, b, np.abs(off))
    dim = rng.uniform(-0.1, 0.1, size=n)
    diag = (absum + margin) + 1j * dim
    hi = np.maximum(a, b)
    lo = np.minimum(a, b)
    rows = np.concatenate([np.arange(n, dtype=np.int64), hi])
    cols = np.concatenate([np.arange(n, dtype=np.int64), lo])
    vals = np.concatenate([diag, off])[None, :]
    return _lower_csc(n, rows, cols, vals)


def shifted_batch(colptr, rowind, base_values, s_diag, z):
    """values_l = A - z_l S for a diagonal S: one pattern, B = len(z) matrices.

    ``base_values`` is [nnz] (real or complex), ``s_diag`` is [n] (the diagonal
    of S, or None for S = I), ``z`` is [B] complex.
    """
    n = colptr.shape[0] - 1
    base = np.asarray(base_values).reshape(-1).astype(np.complex128)
    diag_pos = colptr[:-1]  # diagonal opens every column
    if not np.all(rowind[diag_pos] == np.arange(n)):
        raise ValueError("diagonal missing")
    s = np.ones(n) if s_diag is None else np.asarray(s_diag, dtype=np.float64)
    out = np.repeat(base[None, :], len(z), axis=0)
    out[:, diag_pos] -= np.asarray(z, dtype=np.complex128)[:, None] * s[None, :]
    return out


def random_pattern(n, density, rng, complex_values=False):
    """Random symmetric pattern with a strictly diagonally dominant value set.

    Every off-diagonal lower pair is present with probability ``density``.
    """
    mask = np.tril(rng.random((n, n)) < density, -1)
    r, c = np.nonzero(mask)
    m = r.shape[0]
    off = rng.uniform(-1.0, 1.0, size=m)
    if complex_values:
        off = off + 1j * rng.uniform(-0.5, 0.5, size=m)
    absum = np.zeros(n)
    np.add.at(absum, r, np.abs(off))
    np.add.at(absum, c, np.abs(off))
    diag = absum + 1.0
    if complex_values:
        diag = diag + 1j * rng.uniform(-0.5, 0.5, size=n)
    rows = np.concatenate([np.arange(n), r]).astype(np.int64)
    cols = np.concatenate([np.arange(n), c]).astype(np.int64)
    vals = np.concatenate([diag, off])[None, :]
    return _lower_csc(n, rows, cols, vals)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def _shifts(rng, B):
    """z_l = E_l + i eta_l, E_l ~ U[-2, 2], log10(eta_l) ~ U[-3, 0]."""
    E = rng.uniform(-2.0, 2.0, size=B)
    eta = 10.0 ** rng.uniform(-3.0, 0.0, size=B)
    return E + 1j * eta


def config(name, scale=None, batch=None):
    """Build a named workload.

    C1  2-D 5-point Dirichlet Laplacian 31x31 + 0.1 I (diagonal 4.1), FP64.
    C2  3-D 7-point weighted Laplacian 40^3, weights U[0.5,1.5], sigma 0.05, FP64, seed 2.
    C3  32 complex-symmetric shifts H - z_l S, H from the C2 family on 30^3
        (sigma 0), S = diag(U[0.8,1.2]), seed 3.
    C4  GMRF 200x200, kappa 0.5, w_e ~ N(0, 0.3^2), c_i ~ U[0,1], seed 4.
    C4s the same generator on 30x30.
    C5  64^3 27-point complex-symmetric, 8 shifts A - z_l I, cap 256, seed 5.
    U3  unsymmetric (LU): the 7-point convection-diffusion operator on 30^3
        (convection_diffusion_3d) with 4 real shifts A_l = A + sigma_l I,
        log10(sigma_l) ~ U[-2, 0], seed 7.
    H3  Hermitian: the magnetic 7-point Laplacian H on 30^3 (weights
        U[0.5,1.5], phases U[-pi,pi]) with 16 real shifts A_l = H + sigma_l I,
        log10(sigma_l) ~ U[-2, 0], seed 6 (positive definite).

    ``scale`` replaces the grid edge length (smaller test instances of the
    same family); ``batch`` replaces the number of shifts.
    """
    if name == "C1":
        m = scale or 31
        colptr, rowind, vals = laplacian_2d_dirichlet(m, m, 0.1)
        return Workload("C1", m * m, colptr, rowind, vals, nested_dissection((m, m)),
                        meta={"grid": (m, m), "sigma": 0.1, "dtype": "f64"})
    if name == "C2":
        m = scale or 40
        rng = np.random.default_rng(2)
        colptr, rowind, vals = weighted_laplacian_3d((m, m, m), 0.05, rng)
        return Workload("C2", m ** 3, colptr, rowind, vals, nested_dissection((m, m, m)),
                        meta={"grid": (m, m, m), "sigma": 0.05, "dtype": "f64", "seed": 2})
    if name == "C3":
        m = scale or 30
        B = batch or 32
        rng = np.random.default_rng(3)
        colptr, rowind, hv = weighted_laplacian_3d((m, m, m), 0.0, rng)
        n = m ** 3
        s = rng.uniform(0.8, 1.2, size=n)
        z = _shifts(rng, B)
        vals = shifted_batch(colptr, rowind, hv[0], s, z)
        return Workload("C3", n, colptr, rowind, vals, nested_dissection((m, m, m)),
                        meta={"grid": (m, m, m), "dtype": "c128", "seed": 3, "z": z, "S": s})
    if name in ("C4", "C4s"):
        m = scale or (200 if name == "C4" else 30)
        rng = np.random.default_rng(4)
        nedge = 2 * m * (m - 1)
        w = rng.normal(0.0, 0.3, size=nedge)
        cvec = rng.uniform(0.0, 1.0, size=m * m)
        kappa = 0.5
        colptr, rowind, vals, edges = gmrf_2d(m, m, kappa, w)
        return Workload(name, m * m, colptr, rowind, vals, nested_dissection((m, m)),
                        meta={"grid": (m, m), "dtype": "f64", "seed": 4, "kappa": kappa,
                              "w": w, "c": cvec, "edges": edges})
    if name == "C5":
        m = scale or 64
        B = batch or 8
        rng = np.random.default_rng(5)
        colptr, rowind, av = stencil27_complex((m, m, m), rng)
        z = _shifts(rng, B)
        vals = shifted_batch(colptr, rowind, av[0], None, z)
        return Workload("C5", m ** 3, colptr, rowind, vals, nested_dissection((m, m, m)),
                        cap=256, meta={"grid": (m, m, m), "dtype": "c128", "seed": 5, "z": z})
    if name == "H3":
        m = scale or 30
        B = batch or 16
        rng = np.random.default_rng(6)
        colptr, rowind, hv = magnetic_laplacian_3d((m, m, m), rng)
        sig = 10.0 ** rng.uniform(-2.0, 0.0, size=B)
        vals = shifted_batch(colptr, rowind, hv[0], None, -sig.astype(np.complex128))
        return Workload("H3", m ** 3, colptr, rowind, vals, nested_dissection((m, m, m)),
                        meta={"grid": (m, m, m), "dtype": "h128", "seed": 6, "sigma": sig})
    if name == "U3":
        m = scale or 30
        B = batch or 4
        rng = np.random.default_rng(7)
        colptr, rowind, lo, up = convection_diffusion_3d((m, m, m), rng)
        sig = 10.0 ** rng.uniform(-2.0, 0.0, size=B)
        cols = np.repeat(np.arange(m ** 3), np.diff(colptr))
        dg = (rowind == cols).astype(np.float64)
        vals = np.concatenate([lo[None, :] + sig[:, None] * dg[None, :], up[None, :] + sig[:, None] * dg[None, :]],
                              axis=1)
        return Workload("U3", m ** 3, colptr, rowind, vals, nested_dissection((m, m, m)),
                        meta={"grid": (m, m, m), "dtype": "lu64", "seed": 7, "sigma": sig})
    raise KeyError(name)
