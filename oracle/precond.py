"""Block-Jacobi preconditioner of the probe and y solves, and the point order that
defines its blocks (test infrastructure).

The paper leaves the log-determinant method unnamed (Sec. 4.6, App. B.6 "LOGDET").
The estimators of ``oracle.estimators`` are written for any factor L of a
preconditioner M = L L^T; the diagonal (Jacobi) choice L = D^{1/2} is the special
case of one-point blocks. The block choice is:

* order the points by spatial bin: a grid of cells of side h >= r anchored at the
  lower corner of the points' bounding box, bins numbered with the first coordinate
  varying fastest (so that points closer than r fall in the same or neighbouring
  cells); inside a cell, by the Z-order (Morton) code of the point's offset from the
  cell's corner on a 2^10-step sub-grid per axis, then by user index (so that a run
  of consecutive points is compact even where one cell holds thousands of points);
* cut that order into runs of ``size`` consecutive points (the last run holds the
  remainder); a block of M is the principal submatrix of K on one run, and L is
  its Cholesky factor.

Every function states the quantity it returns in plain linear algebra.
"""
from __future__ import annotations

import numpy as np

BLOCK = 128            # points per block of a single matrix's preconditioner (the default)
BLOCK_SMALL = 64       # the smaller block a single matrix may use instead
BATCH_BLOCK = 64       # points per block inside each instance of a batch


def grid(x, radius, ell_bound=1.0, refine=1, min_cells=65536):
    """(origin, h, nb): the bin grid for points x (n, dim), support radius r (a scalar,
    or one radius per axis) and the bound of the length-scale field l(x) (1 for a
    stationary kernel). Along axis k, h_k = r_k (1 + 1e-6) / refine, times the bound
    when it is not 1; all h_k are widened by a common factor if needed so that the
    number of cells stays within max(4 n, min_cells); nb[k] = floor((hi_k - lo_k) / h_k)
    + 1. One matrix uses refine = 1 and min_cells = 65536; an instance of a batch uses
    the batch's bin refinement (1 or 2) and min_cells = 4096."""
    x = np.asarray(x, dtype=np.float64)
    n, dim = x.shape
    r = np.asarray(radius, dtype=np.float64).reshape(-1)
    radii = [float(r[0])] * dim if r.size == 1 else [float(v) for v in r]
    lo, hi = x.min(axis=0), x.max(axis=0)
    h = [rk * (1.0 + 1e-6) / refine for rk in radii]
    if ell_bound != 1.0:
        h = [hk * ell_bound for hk in h]
    max_bins = max(4.0 * n, float(min_cells))
    for _ in range(64):
        total = 1.0
        for k in range(dim):
            total *= np.floor((hi[k] - lo[k]) / h[k]) + 1.0
        if total <= max_bins:
            break
        f = (total / max_bins) ** (1.0 / dim) * 1.01
        h = [hk * f for hk in h]
    nb = [int(np.floor((hi[k] - lo[k]) / h[k]) + 1.0) for k in range(dim)]
    return lo, np.array(h), nb


def bin_coords(x, radius, ell_bound=1.0, refine=1, min_cells=65536):
    """(n, dim) integer cell coordinates floor((x_k - lo_k) (1 / h_k)), clamped to the grid."""
    x = np.asarray(x, dtype=np.float64)
    lo, h, nb = grid(x, radius, ell_bound, refine, min_cells)
    inv_h = 1.0 / h
    c = np.floor((x - lo[None, :]) * inv_h[None, :])
    return np.clip(c, 0, np.array(nb) - 1).astype(np.int64), nb


SUB_BITS = 10


def morton(f):
    """Z-order code of non-negative integer coordinates f (n, dim) below 2^SUB_BITS: bit b
    of coordinate k becomes bit dim * b + k of the code."""
    f = np.asarray(f, dtype=np.int64)
    n, dim = f.shape
    code = np.zeros(n, dtype=np.int64)
    for b in range(SUB_BITS):
        for k in range(dim):
            code |= ((f[:, k] >> b) & 1) << (dim * b + k)
    return code


def sub_cell_codes(x, radius, ell_bound=1.0, refine=1, min_cells=65536):
    """(n,) int64 position of each point inside its cell: with u_k = (x_k - lo_k)(1 / h_k)
    and c_k = floor(u_k) clamped to the grid, f_k = floor((u_k - c_k) 2^SUB_BITS) clamped
    to [0, 2^SUB_BITS - 1], and the code is morton(f)."""
    x = np.asarray(x, dtype=np.float64)
    lo, h, nb = grid(x, radius, ell_bound, refine, min_cells)
    inv_h = 1.0 / h
    u = (x - lo[None, :]) * inv_h[None, :]
    c = np.clip(np.floor(u), 0, np.array(nb) - 1)
    steps = float(1 << SUB_BITS)
    f = np.clip(np.floor((u - c) * steps), 0, steps - 1)
    return morton(f.astype(np.int64))


def bin_order(x, radius, ell_bound=1.0, refine=1, min_cells=65536):
    """perm (n,) int64: perm[p] is the user index of the point at position p when the
    points are sorted by cell number (first coordinate fastest), then by sub-cell code,
    then by user index."""
    c, nb = bin_coords(x, radius, ell_bound, refine, min_cells)
    key = np.zeros(c.shape[0], dtype=np.int64)
    for k in range(c.shape[1] - 1, -1, -1):
        key = key * nb[k] + c[:, k]
    code = sub_cell_codes(x, radius, ell_bound, refine, min_cells)
    return np.lexsort((np.arange(c.shape[0]), code, key)).astype(np.int64)


def block_partition(order, size=BLOCK):
    """Runs of `size` consecutive entries of `order` (the last one may be shorter)."""
    order = np.asarray(order, dtype=np.int64)
    return [order[s:s + size] for s in range(0, len(order), size)]


def jacobi_partition(n):
    """One-point blocks: M = diag(K)."""
    return [np.array([i], dtype=np.int64) for i in range(n)]


def block_factor(K, blocks):
    """(L, Linv, logdet_M) for M = the block diagonal of K over `blocks` (index sets
    of a partition of the points, in user indexing): L[b, b] = chol(K[b, b]) (lower
    within the block's own index order), zero elsewhere, so that M = L L^T; Linv is
    L^-1 with the same structure; logdet_M = ln|M| = sum over blocks of ln|K[b, b]|.
    Blocks of equal size are factored together (a batched library Cholesky)."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    L = np.zeros((n, n))
    Linv = np.zeros((n, n))
    logdet = 0.0
    by_size = {}
    for b in blocks:
        b = np.asarray(b, dtype=np.int64)
        by_size.setdefault(len(b), []).append(b)
    for size in sorted(by_size):
        idx = np.stack(by_size[size])                      # (m, size)
        Kb = K[idx[:, :, None], idx[:, None, :]]           # (m, size, size)
        Lb = np.linalg.cholesky(Kb)
        Lb_inv = np.linalg.inv(Lb)
        L[idx[:, :, None], idx[:, None, :]] = Lb
        Linv[idx[:, :, None], idx[:, None, :]] = Lb_inv
        logdet += 2.0 * float(np.sum(np.log(np.diagonal(Lb, axis1=1, axis2=2))))
    return L, Linv, logdet
