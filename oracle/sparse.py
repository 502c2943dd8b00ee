"""Sparse float64 covariance (scipy CSR, user order) for sizes beyond the dense
oracle, plus a plain Jacobi-preconditioned conjugate-gradient solve.

The stored entries are exactly those of the structural pattern (oracle.pattern),
found with a k-d tree; values follow the same formulas as oracle.dense. The solve
is textbook preconditioned CG (Hestenes-Stiefel with M = diag(K)); the paper's
host solver is MINRES (App. B.6), which reaches the same solution K^{-1} y.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .kernel import bump_values, wendland
from .pattern import sqdist_pairs


def _values(x, radius, g, i, j, kernel):
    d2 = sqdist_pairs(x[i], x[j])
    return g[i] * g[j] * wendland(np.sqrt(d2) / float(radius), kernel), d2


def covariance_csr(x, radius, bump_width, centers, weights, noise_var, kernel="c2"):
    """Full K as scipy.sparse.csr_matrix (columns ascending within each row)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    g, _, gamma = bump_values(x, centers, bump_width, weights)
    tree = cKDTree(x)
    pairs = tree.query_pairs(float(radius), output_type="ndarray")
    if pairs.size:
        v, d2 = _values(x, radius, g, pairs[:, 0], pairs[:, 1], kernel)
        keep = (d2 < float(radius) ** 2) & gamma[pairs[:, 0]] & gamma[pairs[:, 1]]
        pairs, v = pairs[keep], v[keep]
    else:
        v = np.zeros(0)
    diag = np.arange(n)
    rows = np.concatenate([pairs[:, 0], pairs[:, 1], diag])
    cols = np.concatenate([pairs[:, 1], pairs[:, 0], diag])
    vals = np.concatenate([v, v, g * g + float(noise_var)])
    K = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    K.sort_indices()
    return K


def covariance_rows(x, radius, bump_width, centers, weights, noise_var, rows, tree=None,
                    g=None, gamma=None, kernel="c2"):
    """Rows `rows` of K (user order): list of (cols ascending, values) per row."""
    x = np.asarray(x, dtype=np.float64)
    if g is None or gamma is None:
        g, _, gamma = bump_values(x, centers, bump_width, weights)
    if tree is None:
        tree = cKDTree(x)
    out = []
    nb = tree.query_ball_point(x[rows], float(radius))
    r2 = float(radius) ** 2
    for i, cand in zip(rows, nb):
        cand = np.asarray(cand, dtype=np.int64)
        d2 = sqdist_pairs(np.broadcast_to(x[i], (len(cand), x.shape[1])), x[cand])
        keep = (d2 < r2) & gamma[cand] & bool(gamma[i])
        keep |= cand == i
        cols = np.sort(cand[keep])
        if i not in cols:
            cols = np.sort(np.append(cols, i))
        rho = np.sqrt(sqdist_pairs(np.broadcast_to(x[i], (len(cols), x.shape[1])), x[cols])) / float(radius)
        vals = g[i] * g[cols] * wendland(rho, kernel)
        vals[cols == i] = g[i] * g[i] + float(noise_var)
        out.append((cols, vals))
    return out


def residual_rel(K, a, y):
    """||y - K a||_2 / ||y||_2 in float64 (K any matrix-like with @)."""
    r = np.asarray(y, dtype=np.float64) - K @ np.asarray(a, dtype=np.float64)
    return float(np.linalg.norm(r) / np.linalg.norm(y))


def pcg_jacobi(K, b, tol=1e-8, max_iter=100000):
    """Jacobi-preconditioned CG for K x = b (K SPD). Returns x, iterations, and the
    (alpha, beta) coefficient history. Stops when ||b - K x|| <= tol ||b||, with the
    residual recurrence checked against a recomputed residual at the end."""
    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / K.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    bnorm = float(np.linalg.norm(b))
    alphas, betas = [], []
    it = 0
    while it < max_iter:
        if float(np.linalg.norm(r)) <= tol * bnorm:
            break
        q = K @ p
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
        it += 1
    return x, it, np.array(alphas), np.array(betas)
