"""The non-stationary convolution Wendland kernel (Sec. 4.2, Eq. wendconv) with an
axis-anisotropic (ARD) length scale, times the bump mask: dense and sparse covariance,
the exact derivatives, and the cross-covariance for the posterior (test
infrastructure).

Eq. wendconv, with the Wendland member W of Eq. wendland (or its C^2 variation):

    k(x_i, x_j) = s(x_i) s(x_j) |S_i|^{1/4} |S_j|^{1/4} / |(S_i + S_j)/2|^{1/2} W(sqrt(Q_ij)),
    Q_ij = (x_i - x_j)^T ((S_i + S_j)/2)^{-1} (x_i - x_j),  S_i = S(x_i).

The paper leaves the length-scale field S(x) and the signal deviation s(x) open. The
reading taken here keeps the bump machinery of Sec. 4.3:

    S(x) = diag(r_1^2, ..., r_d^2) l(x)^2,    l(x) = exp( sum_q c_q bhat_q(x) ),
    s(x) = g(x) = sum_q a_q bhat_q(x),

with bhat_q the unweighted bumps (Eq. bump, shape parameter 1) at the same centres and
width as g. With l_i = l(x_i) and m_ij = (l_i^2 + l_j^2) / 2 this gives

    Q_ij = d_ij / m_ij,   d_ij = sum_k ((x_ik - x_jk) / r_k)^2,
    prefactor p_ij = (l_i l_j / m_ij)^{d/2}   (<= 1, = 1 when l_i = l_j),
    K_ij = g_i g_j p_ij W(sqrt(Q_ij)) + sigma_n^2 [i == j],

stored where Q_ij < 1 and both points lie inside some bump (the diagonal always).
All c_q = 0 and r_1 = ... = r_d = r is the stationary kernel of ``oracle.dense``.
Hyperparameters in gradient order: the radius (one r, or r_1..r_d), a_1..a_P,
c_1..c_P (when the length-scale field is on), sigma_n^2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

from .kernel import bump_values, wendland, wendland_dlog


def _radii(radius, dim):
    r = np.asarray(radius, dtype=np.float64).reshape(-1)
    if r.size == 1:
        return np.full(dim, float(r[0])), True
    if r.size != dim:
        raise ValueError("radius must be a scalar or one value per dimension")
    return r.copy(), False


def length_scale(x, centers, bump_width, ls_weights):
    """(l, bhat): l(x) = exp(sum_q c_q bhat_q(x)) (ones when ls_weights is None) and the
    unweighted bumps."""
    x = np.asarray(x, dtype=np.float64)
    P = np.asarray(centers).reshape(-1, x.shape[1]).shape[0]
    _, bhat, _ = bump_values(x, centers, bump_width, np.ones(P))
    if ls_weights is None:
        return np.ones(x.shape[0]), bhat
    return np.exp(bhat @ np.asarray(ls_weights, dtype=np.float64)), bhat


def ell_bound(ls_weights):
    """Upper bound of l(x) from the parameters alone: exp(sum of the positive c_q), as
    every bhat_q lies in [0, 1] (1 at its centre)."""
    if ls_weights is None:
        return 1.0
    return math.exp(float(sum(max(float(c), 0.0) for c in np.asarray(ls_weights).reshape(-1))))


def geometry(xa, xb, radii, la, lb):
    """Pairwise (d, m, Q, p) between the rows of xa and xb: d the ARD-scaled squared
    distance, m = (l_a^2 + l_b^2)/2, Q = d / m, p = (l_a l_b / m)^{dim/2}."""
    xa = np.asarray(xa, dtype=np.float64)
    xb = np.asarray(xb, dtype=np.float64)
    d = np.zeros((xa.shape[0], xb.shape[0]))
    for k in range(xa.shape[1]):
        diff = (xa[:, k][:, None] - xb[:, k][None, :]) / radii[k]
        d += diff * diff
    m = 0.5 * (la[:, None] ** 2 + lb[None, :] ** 2)
    Q = d / m
    p = (la[:, None] * lb[None, :] / m) ** (0.5 * xa.shape[1])
    return d, m, Q, p


def covariance_dense(x, radius, bump_width, centers, weights, noise_var, ls_weights=None, kernel="c2",
                     return_parts=False):
    """Dense K (n x n) of the kernel above."""
    x = np.asarray(x, dtype=np.float64)
    n, dim = x.shape
    radii, _ = _radii(radius, dim)
    g, b, gamma = bump_values(x, centers, bump_width, weights)
    ell, bhat = length_scale(x, centers, bump_width, ls_weights)
    d, m, Q, p = geometry(x, x, radii, ell, ell)
    keep = (Q < 1.0) & gamma[:, None] & gamma[None, :]
    np.fill_diagonal(keep, True)
    rho = np.sqrt(Q)
    W = np.where(keep, wendland(rho, kernel), 0.0)
    K = g[:, None] * g[None, :] * p * W
    K[np.diag_indices_from(K)] = g * g + float(noise_var)
    if return_parts:
        return K, dict(g=g, b=b, bhat=bhat, ell=ell, gamma=gamma, d=d, m=m, Q=Q, p=p, rho=rho, keep=keep, W=W,
                       radii=radii)
    return K


def dcov_dense(x, radius, bump_width, centers, weights, noise_var, ls_weights=None, kernel="c2"):
    """(K, [dK/dtheta]) in the gradient order above.

    dK/dr_k  = g_i g_j p_ij D(rho) ((x_ik - x_jk)/r_k)^2 / (r_k m_ij),  D = -W'(rho)/rho
               (one radius: the sum over k, = g_i g_j p_ij D(rho) Q_ij / r)
    dK/da_q  = (b_iq g_j + g_i b_jq) p_ij W_ij
    dK/dc_q  = g_i g_j (E_ij bhat_iq + E_ji bhat_jq),
               E_ij = d(p W)/d ln l_i = p_ij [ (dim/2)(1 - l_i^2/m_ij) W + D(rho) Q_ij l_i^2 / (2 m_ij) ]
    dK/dsigma2 = I
    """
    x = np.asarray(x, dtype=np.float64)
    n, dim = x.shape
    K, pt = covariance_dense(x, radius, bump_width, centers, weights, noise_var, ls_weights, kernel,
                             return_parts=True)
    radii, iso = _radii(radius, dim)
    g, b, bhat, ell, keep, Q, m, p, rho, W = (pt[k] for k in ("g", "b", "bhat", "ell", "keep", "Q", "m", "p",
                                                              "rho", "W"))
    off = keep.copy()
    np.fill_diagonal(off, False)
    D = np.where(off, wendland_dlog(rho, kernel), 0.0)
    gg = g[:, None] * g[None, :]
    out = []
    if iso:
        out.append(gg * p * D * Q / radii[0])
    else:
        for k in range(dim):
            diff = (x[:, k][:, None] - x[:, k][None, :]) / radii[k]
            out.append(gg * p * D * diff * diff / (radii[k] * m))
    Woff = np.where(off, W, 0.0)
    for q in range(b.shape[1]):
        bq = b[:, q]
        dq = (bq[:, None] * g[None, :] + g[:, None] * bq[None, :]) * p * Woff
        dq[np.diag_indices_from(dq)] = 2.0 * g * bq
        out.append(dq)
    if ls_weights is not None:
        li2 = ell[:, None] ** 2
        E = p * (0.5 * dim * (1.0 - li2 / m) * Woff + D * Q * li2 / (2.0 * m))
        E = np.where(off, E, 0.0)
        for q in range(bhat.shape[1]):
            bq = bhat[:, q]
            out.append(gg * (E * bq[:, None] + E.T * bq[None, :]))
    out.append(np.eye(n))
    return K, out


def covariance_csr(x, radius, bump_width, centers, weights, noise_var, ls_weights=None, kernel="c2"):
    """Sparse K (scipy CSR, user order): candidate pairs from a k-d tree on the
    ARD-scaled coordinates within the largest l, then the exact test Q < 1."""
    import scipy.sparse as sp
    x = np.asarray(x, dtype=np.float64)
    n, dim = x.shape
    radii, _ = _radii(radius, dim)
    g, _, gamma = bump_values(x, centers, bump_width, weights)
    ell, _ = length_scale(x, centers, bump_width, ls_weights)
    z = x / radii[None, :]
    pairs = cKDTree(z).query_pairs(float(ell.max()) * (1.0 + 1e-9), output_type="ndarray")
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [g * g + float(noise_var)]
    if pairs.size:
        i, j = pairs[:, 0], pairs[:, 1]
        d = np.zeros(len(i))
        for k in range(dim):
            diff = (x[i, k] - x[j, k]) / radii[k]
            d += diff * diff
        m = 0.5 * (ell[i] ** 2 + ell[j] ** 2)
        Q = d / m
        keep = (Q < 1.0) & gamma[i] & gamma[j]
        i, j, Q, m = i[keep], j[keep], Q[keep], m[keep]
        p = (ell[i] * ell[j] / m) ** (0.5 * dim)
        v = g[i] * g[j] * p * wendland(np.sqrt(Q), kernel)
        rows += [i, j]
        cols += [j, i]
        vals += [v, v]
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    K.sort_indices()
    return K


def cross_covariance(x_test, x, radius, bump_width, centers, weights, ls_weights=None, kernel="c2"):
    """(k(x*_t, x_j) for every test point t and training point j, g(x*))."""
    x_test = np.asarray(x_test, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    radii, _ = _radii(radius, x.shape[1])
    gs, _, gams = bump_values(x_test, centers, bump_width, weights)
    g, _, gam = bump_values(x, centers, bump_width, weights)
    ls, _ = length_scale(x_test, centers, bump_width, ls_weights)
    ell, _ = length_scale(x, centers, bump_width, ls_weights)
    d, m, Q, p = geometry(x_test, x, radii, ls, ell)
    keep = (Q < 1.0) & gams[:, None] & gam[None, :]
    return np.where(keep, gs[:, None] * g[None, :] * p * wendland(np.sqrt(Q), kernel), 0.0), gs
