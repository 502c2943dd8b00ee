"""Sparsity pattern of the covariance matrix, by brute force and by a k-d tree.

The paper (Sec. 4.6) notes that its distributed implementation evaluates every
entry because the zeros are only known after evaluation. For the kernel used here
the zeros are known geometrically: k(x_i, x_j) vanishes when ||x_i - x_j|| >= r
(the Wendland factor, Eq. wendland has strict support) or when either point lies
outside every bump (the bump factor, Eq. bump has strict support). The pattern is
therefore defined structurally:

    (i, j) stored  <=>  i == j  or  ( ||x_i - x_j||^2 < r^2  and  gamma_i  and  gamma_j )

It depends on the points, r, the bump centres and the bump width only; entries in
the pattern may still evaluate to zero (a bump value that underflows).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def pairwise_sqdist(xa, xb):
    """||x_a - x_b||^2 from coordinate differences (no |a|^2 + |b|^2 - 2ab expansion)."""
    xa = np.asarray(xa, dtype=np.float64)
    xb = np.asarray(xb, dtype=np.float64)
    d2 = np.zeros((xa.shape[0], xb.shape[0]))
    for k in range(xa.shape[1]):
        diff = xa[:, k][:, None] - xb[:, k][None, :]
        d2 += diff * diff
    return d2


def sqdist_pairs(xa, xb):
    """Row-wise ||xa_k - xb_k||^2, summed over coordinates in order (the same
    rounding order as pairwise_sqdist)."""
    d2 = np.zeros(xa.shape[0])
    for k in range(xa.shape[1]):
        diff = xa[:, k] - xb[:, k]
        d2 += diff * diff
    return d2


def pattern_bruteforce(x, radius, gamma):
    """All stored (i, j), i, j in user order, by testing every pair. Returns a
    sorted (m, 2) int64 array (row-major order, columns ascending)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    r2 = float(radius) ** 2
    rows, cols = [], []
    block = max(1, (1 << 22) // max(n, 1))
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        d2 = pairwise_sqdist(x[lo:hi], x)
        keep = (d2 < r2) & gamma[lo:hi, None] & gamma[None, :]
        keep[np.arange(hi - lo), np.arange(lo, hi)] = True
        i, j = np.nonzero(keep)
        rows.append(i + lo)
        cols.append(j)
    out = np.stack([np.concatenate(rows), np.concatenate(cols)], axis=1).astype(np.int64)
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def pattern_kdtree(x, radius, gamma):
    """Same set as pattern_bruteforce, found with scipy's k-d tree (candidate pairs
    with distance <= r) followed by the exact strict test in float64."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    r2 = float(radius) ** 2
    tree = cKDTree(x)
    pairs = tree.query_pairs(float(radius), output_type="ndarray")
    if pairs.size:
        d2 = sqdist_pairs(x[pairs[:, 0]], x[pairs[:, 1]])
        keep = (d2 < r2) & gamma[pairs[:, 0]] & gamma[pairs[:, 1]]
        pairs = pairs[keep]
    diag = np.arange(n, dtype=np.int64)
    rows = np.concatenate([pairs[:, 0], pairs[:, 1], diag]).astype(np.int64)
    cols = np.concatenate([pairs[:, 1], pairs[:, 0], diag]).astype(np.int64)
    out = np.stack([rows, cols], axis=1)
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def mean_row_count(x, radius):
    """Mean over rows of #{j : ||x_i - x_j|| <= r}, diagonal included (the radius
    calibration target; ties at exactly r have probability zero for the synthetic
    inputs). Uses the k-d tree's dual-tree pair count."""
    x = np.asarray(x, dtype=np.float64)
    tree = cKDTree(x)
    return float(tree.count_neighbors(tree, float(radius))) / x.shape[0]


def boundary_exempt_pairs(x, radius, pairs, rel=1e-6):
    """Boolean mask over (m, 2) candidate pairs whose rho^2 lies within rel of 1:
    there float32 and float64 evaluations of the strict support test may differ."""
    x = np.asarray(x, dtype=np.float64)
    rho2 = sqdist_pairs(x[pairs[:, 0]], x[pairs[:, 1]]) / float(radius) ** 2
    return np.abs(rho2 - 1.0) <= rel


def boundary_exempt_points(x, centers, bump_width, rel=1e-6):
    """Boolean mask over points lying within rel (in s = ||x - c||^2 / w^2) of some
    bump's boundary: their bump-membership flag may differ between precisions."""
    x = np.asarray(x, dtype=np.float64)
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, x.shape[1])
    out = np.zeros(x.shape[0], dtype=bool)
    w2 = float(bump_width) ** 2
    for c in centers:
        d = x - c[None, :]
        s = np.einsum("ik,ik->i", d, d) / w2
        out |= np.abs(s - 1.0) <= rel
    return out
