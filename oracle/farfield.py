"""The far-field bump kernel (Sec. 4.3, Eq. bump_kernel) with the core kernel set to
one (test infrastructure).

    k(x_i, x_j) = sum_u g_u(x_i) g_u(x_j) + W(||x_i - x_j|| / r),
    g_u(x) = sum over the bumps p of group u of a_p bhat_p(x),

bhat_p the unweighted bumps of Eq. bump (shape parameter 1) and W the Wendland member
(Eq. wendland or its C^2 variation), plus sigma_n^2 on the diagonal. Unlike the product
construction, W carries no bump mask, and the bump term couples points at any
distance: K = K_loc + G G^T with K_loc = W + sigma_n^2 I sparse (radius-local) and
G = [g_1 .. g_U] of rank U. The hyperparameters keep the product kernel's order
(r, a_1..a_P, sigma_n^2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from .kernel import bump_values, wendland, wendland_dr
from .pattern import pairwise_sqdist, sqdist_pairs


def group_values(x, centers, bump_width, weights, groups):
    """(G (n, U), bhat (n, P)): G[:, u] = sum_{p in group u} a_p bhat_p(x)."""
    x = np.asarray(x, dtype=np.float64)
    groups = np.asarray(groups, dtype=np.int64).reshape(-1)
    P = groups.shape[0]
    _, bhat, _ = bump_values(x, centers, bump_width, np.ones(P))
    U = int(groups.max()) + 1
    G = np.zeros((x.shape[0], U))
    w = np.asarray(weights, dtype=np.float64).reshape(-1)
    for p in range(P):
        G[:, groups[p]] += w[p] * bhat[:, p]
    return G, bhat


def local_dense(x, radius, noise_var, kernel="c2"):
    """K_loc = W(||x_i - x_j|| / r) on ||x_i - x_j|| < r, plus sigma_n^2 on the diagonal."""
    x = np.asarray(x, dtype=np.float64)
    d2 = pairwise_sqdist(x, x)
    keep = d2 < float(radius) ** 2
    np.fill_diagonal(keep, True)
    K = np.where(keep, wendland(np.sqrt(d2) / float(radius), kernel), 0.0)
    K[np.diag_indices_from(K)] = 1.0 + float(noise_var)
    return K


def local_csr(x, radius, noise_var, kernel="c2"):
    """K_loc as scipy CSR (user order), from a k-d tree."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    pairs = cKDTree(x).query_pairs(float(radius), output_type="ndarray")
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 1.0 + float(noise_var))]
    if pairs.size:
        i, j = pairs[:, 0], pairs[:, 1]
        d2 = sqdist_pairs(x[i], x[j])
        keep = d2 < float(radius) ** 2
        i, j, d2 = i[keep], j[keep], d2[keep]
        v = wendland(np.sqrt(d2) / float(radius), kernel)
        rows += [i, j]
        cols += [j, i]
        vals += [v, v]
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    K.sort_indices()
    return K


def covariance_dense(x, radius, bump_width, centers, weights, noise_var, groups, kernel="c2"):
    """Dense K = G G^T + K_loc."""
    G, _ = group_values(x, centers, bump_width, weights, groups)
    return G @ G.T + local_dense(x, radius, noise_var, kernel)


def dcov_dense(x, radius, bump_width, centers, weights, noise_var, groups, kernel="c2"):
    """(K, [dK/dr, dK/da_1..dK/da_P, dK/dsigma2]):
    dK/dr = dW/dr on the radius pattern; dK/da_p = bhat_p g_u^T + g_u bhat_p^T (u the
    group of p); dK/dsigma2 = I."""
    x = np.asarray(x, dtype=np.float64)
    G, bhat = group_values(x, centers, bump_width, weights, groups)
    K = G @ G.T + local_dense(x, radius, noise_var, kernel)
    d2 = pairwise_sqdist(x, x)
    keep = d2 < float(radius) ** 2
    out = [np.where(keep, wendland_dr(np.sqrt(d2) / float(radius), float(radius), kernel), 0.0)]
    groups = np.asarray(groups, dtype=np.int64).reshape(-1)
    for p in range(bhat.shape[1]):
        gu = G[:, groups[p]]
        out.append(np.outer(bhat[:, p], gu) + np.outer(gu, bhat[:, p]))
    out.append(np.eye(x.shape[0]))
    return K, out


def cross_covariance(x_test, x, radius, bump_width, centers, weights, groups, kernel="c2"):
    """(k(x*_t, x_j) for every test point t and training point j, prior variance
    k(x*, x*) = sum_u g_u(x*)^2 + W(0))."""
    x_test = np.asarray(x_test, dtype=np.float64)
    Gt, _ = group_values(x_test, centers, bump_width, weights, groups)
    G, _ = group_values(x, centers, bump_width, weights, groups)
    d2 = pairwise_sqdist(x_test, np.asarray(x, dtype=np.float64))
    W = np.where(d2 < float(radius) ** 2, wendland(np.sqrt(d2) / float(radius), kernel), 0.0)
    return Gt @ G.T + W, np.sum(Gt * Gt, axis=1) + 1.0
