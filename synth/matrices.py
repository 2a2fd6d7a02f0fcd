"""Seeded sparse test matrices in CSR form (0-based, int32 indices, FP64 values).

Every generator returns a ``CSR`` tuple ``(n, rowptr, col, val)`` with columns
sorted ascending and unique within each row.  Nothing here multiplies,
reorders or schedules anything: the arithmetic under test lives elsewhere.
"""
from collections import namedtuple

import numpy as np

CSR = namedtuple("CSR", ["n", "rowptr", "col", "val"])


def _from_rows(n, cols_per_row, vals_per_row, mask):
    """Pack an (n, w) table of candidate entries into CSR, keeping ``mask``.

    Candidates must already be in ascending column order along each row.
    """
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols_per_row[mask].astype(np.int32)
    val = vals_per_row[mask].astype(np.float64)
    return CSR(int(n), rowptr.astype(np.int32), col, val)


def _from_coo(n, rows, cols, vals):
    """CSR from COO triplets with no duplicate (row, col) pairs."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate entries in COO input")
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(int(n), rowptr.astype(np.int32), cols.astype(np.int32), vals)


def laplacian_1d(n):
    """Dirichlet 1D Laplacian tridiag(-1, 2, -1) of order n."""
    i = np.arange(n, dtype=np.int64)[:, None]
    cols = i + np.array([-1, 0, 1], dtype=np.int64)[None, :]
    vals = np.broadcast_to(np.array([-1.0, 2.0, -1.0]), cols.shape)
    mask = (cols >= 0) & (cols < n)
    return _from_rows(n, cols, vals, mask)


def laplacian_2d(nx, ny=None):
    """Dirichlet 5-point Laplacian on an nx-by-ny grid (diagonal 4, neighbours -1).

    Row index of grid point (i, j) is i + nx*j (natural order).  The matrix is
    T_y (x) I + I (x) T_x with T the 1D Laplacian, so its eigenvalues are sums
    of 1D eigenvalues.
    """
    ny = nx if ny is None else ny
    n = nx * ny
    idx = np.arange(n, dtype=np.int64)
    i, j = idx % nx, idx // nx
    offs = np.array([-nx, -1, 0, 1, nx], dtype=np.int64)
    cols = idx[:, None] + offs[None, :]
    vals = np.broadcast_to(np.array([-1.0, -1.0, 4.0, -1.0, -1.0]), cols.shape)
    mask = np.ones(cols.shape, dtype=bool)
    mask[:, 0] = j > 0
    mask[:, 1] = i > 0
    mask[:, 3] = i < nx - 1
    mask[:, 4] = j < ny - 1
    return _from_rows(n, cols, vals, mask)


def laplacian_3d(nx, ny=None, nz=None):
    """Dirichlet 7-point Laplacian on an nx*ny*nz grid (diagonal 6, neighbours -1).

    Row index of (i, j, k) is i + nx*(j + ny*k).  At 160^3 this has
    N = 4,096,000 rows and 28,518,400 nonzeros.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    pl = nx * ny
    offs = np.array([-pl, -nx, -1, 0, 1, nx, pl], dtype=np.int64)
    cols = idx[:, None] + offs[None, :]
    vals = np.broadcast_to(np.array([-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0]), cols.shape)
    mask = np.ones(cols.shape, dtype=bool)
    mask[:, 0] = k > 0
    mask[:, 1] = j > 0
    mask[:, 2] = i > 0
    mask[:, 4] = i < nx - 1
    mask[:, 5] = j < ny - 1
    mask[:, 6] = k < nz - 1
    return _from_rows(n, cols, vals, mask)


def _morton_key(points, bits=21):
    q = np.minimum((points * (1 << bits)).astype(np.uint64), np.uint64((1 << bits) - 1))
    key = np.zeros(points.shape[0], dtype=np.uint64)
    for b in range(bits):
        for d in range(3):
            bit = (q[:, d] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(3 * b + d)
    return key


def knn_graph_laplacian(npts, k=26, shift=0.1, seed=0, morton=True, workers=-1):
    """Shifted graph Laplacian of a symmetrised k-nearest-neighbour graph.

    ``npts`` points are drawn uniformly in [0,1)^3 from ``default_rng(seed)``
    and, if ``morton`` is set, renumbered along a Morton (Z-order) curve so
    that nearby points get nearby indices.  Each point is joined to its ``k``
    nearest other points (exact Euclidean search); the adjacency is
    symmetrised by union, W = max(W, W^T), with unit weights.  The result is
    L = D - W + shift*I, symmetric positive definite with smallest eigenvalue
    exactly ``shift`` (the constant vector is an eigenvector of D - W).
    Every row has at least k+1 entries.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(int(npts), 3))
    if morton:
        pts = pts[np.argsort(_morton_key(pts), kind="stable")]
    tree = cKDTree(pts)
    _, nbr = tree.query(pts, k=k + 1, workers=workers)
    n = pts.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), k + 1)
    cols = nbr.reshape(-1).astype(np.int64)
    keep = rows != cols
    rows, cols = rows[keep], cols[keep]
    # each point is its own nearest neighbour; if duplicates pushed it out of
    # the list, a row may carry k+1 neighbours: trim to k per row
    key = np.unique(np.concatenate([rows * n + cols, cols * n + rows]))
    r, c = key // n, key % n
    deg = np.bincount(r, minlength=n).astype(np.float64)
    rows_all = np.concatenate([r, np.arange(n)])
    cols_all = np.concatenate([c, np.arange(n)])
    vals_all = np.concatenate([-np.ones(r.size), deg + shift])
    return _from_coo(n, rows_all, cols_all, vals_all)


def random_pattern(n, avg_nnz, seed, symmetric=False, diag=True, integer=False, value_range=1.0):
    """Seeded random sparse matrix for property tests.

    Each row receives ``Poisson(avg_nnz)`` distinct random columns (so empty
    rows occur).  ``symmetric`` mirrors the pattern (values stay random, so the
    matrix itself need not be symmetric).  ``integer`` draws small integer
    values in [-2, 2] instead of uniform floats.
    """
    rng = np.random.default_rng(seed)
    counts = np.minimum(rng.poisson(avg_nnz, size=n), n)
    rows = np.repeat(np.arange(n, dtype=np.int64), counts)
    cols = rng.integers(0, n, size=rows.size, dtype=np.int64)
    if diag:
        rows = np.concatenate([rows, np.arange(n)])
        cols = np.concatenate([cols, np.arange(n)])
    if symmetric:
        rows, cols = np.concatenate([rows, cols]), np.concatenate([cols, rows])
    key = np.unique(rows * n + cols)
    r, c = key // n, key % n
    if integer:
        v = rng.integers(-2, 3, size=r.size).astype(np.float64)
    else:
        v = rng.uniform(-value_range, value_range, size=r.size)
    return _from_coo(n, r, c, v)


def banded_random(n, avg_nnz, half_band, seed, symmetric=False, integer=False):
    """Seeded random pattern confined to a band |i - j| <= half_band, diagonal
    always present.  Off-diagonal entries are drawn independently per (row,
    column) with probability (avg_nnz - 1) / (2 half_band), so unless
    ``symmetric`` the pattern is nonsymmetric; the band keeps the graph's
    diameter near n / half_band (long BFS level structures), unlike
    ``random_pattern``.  Values uniform in [-1, 1] (integers in [-3, 3] with
    ``integer``), the diagonal 1 + |row sum| of the off-diagonal magnitudes.
    """
    rng = np.random.default_rng(seed)
    w = 2 * half_band + 1
    i = np.arange(n, dtype=np.int64)[:, None]
    cols = i + np.arange(-half_band, half_band + 1, dtype=np.int64)[None, :]
    prob = min(1.0, (avg_nnz - 1.0) / (2.0 * half_band))
    keep = rng.random((n, w)) < prob
    if integer:
        vals = rng.integers(-3, 4, size=(n, w)).astype(np.float64)
    else:
        vals = rng.uniform(-1.0, 1.0, size=(n, w))
    if symmetric:  # mirror the strictly upper half onto the lower half
        for d in range(1, half_band + 1):
            up_k, up_v = keep[:, half_band + d], vals[:, half_band + d]
            keep[d:, half_band - d] = up_k[:-d]
            vals[d:, half_band - d] = up_v[:-d]
    mask = keep & (cols >= 0) & (cols < n)
    mask[:, half_band] = False
    off = np.where(mask, np.abs(vals), 0.0).sum(axis=1)
    vals = vals.copy()
    vals[:, half_band] = 1.0 + (np.ceil(off) if integer else off)
    mask[:, half_band] = True
    return _from_rows(n, cols, vals, mask)


def block_diagonal(*mats):
    """Block-diagonal matrix from CSR blocks (a graph with several components)."""
    rows, cols, vals = [], [], []
    off = 0
    for m in mats:
        rp = np.asarray(m.rowptr, dtype=np.int64)
        rows.append(np.repeat(np.arange(m.n, dtype=np.int64), np.diff(rp)) + off)
        cols.append(np.asarray(m.col, dtype=np.int64) + off)
        vals.append(np.asarray(m.val, dtype=np.float64))
        off += m.n
    if not rows:
        return CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    return _from_coo(off, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def from_dense(a, keep_zeros=False):
    """CSR from a dense 2D array (explicit zeros dropped unless ``keep_zeros``)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix expected")
    mask = np.ones_like(a, dtype=bool) if keep_zeros else (a != 0)
    r, c = np.nonzero(mask)
    return _from_coo(n, r, c, a[r, c])


def identity(n):
    i = np.arange(n)
    return _from_coo(n, i, i, np.ones(n))


def diagonal(d):
    d = np.asarray(d, dtype=np.float64)
    i = np.arange(d.size)
    return _from_coo(d.size, i, i, d)


def cyclic_shift(n):
    """Permutation matrix with (A x)[i] = x[(i + 1) mod n]: a directed ring."""
    i = np.arange(n)
    return _from_coo(n, i, (i + 1) % n, np.ones(n))
