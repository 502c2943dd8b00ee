"""Sparse float64 covariance (scipy CSR, user order) for sizes beyond the dense
oracle, a plain Jacobi-preconditioned conjugate-gradient solve, and the whole LML
and gradient on that path: Lanczos quadrature of the log-determinant from the CG
coefficients of the probe solves, and the gradient contraction with sparse dK.

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


def _pattern_pairs(x, radius, gamma):
    """Unordered pairs i < j of the structural pattern (k-d tree candidates, strict
    radius, both points inside some bump)."""
    tree = cKDTree(x)
    pairs = tree.query_pairs(float(radius), output_type="ndarray")
    if not pairs.size:
        return np.zeros((0, 2), dtype=np.int64), np.zeros(0)
    d2 = sqdist_pairs(x[pairs[:, 0]], x[pairs[:, 1]])
    keep = (d2 < float(radius) ** 2) & gamma[pairs[:, 0]] & gamma[pairs[:, 1]]
    return pairs[keep].astype(np.int64), d2[keep]


def dcov_csr(x, radius, bump_width, centers, weights, noise_var, kernel="c2"):
    """Sparse K and the list of sparse dK/dtheta in the order (r, a_1..a_P, sigma_n^2),
    on the structural pattern; the same formulas as oracle.dense.dcov_dense:

    dK/dr      = g_i g_j dW/dr
    dK/da_k    = (b_ik g_j + g_i b_jk) W_ij
    dK/dsigma2 = I
    """
    from .kernel import wendland_dr

    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    g, b, gamma = bump_values(x, centers, bump_width, weights)
    pairs, d2 = _pattern_pairs(x, radius, gamma)
    i, j = pairs[:, 0], pairs[:, 1]
    rho = np.sqrt(d2) / float(radius)
    W = wendland(rho, kernel)
    diag = np.arange(n)

    def sym(v, dv):
        m = sp.csr_matrix((np.concatenate([v, v, dv]), (np.concatenate([i, j, diag]), np.concatenate([j, i, diag]))),
                          shape=(n, n))
        m.sort_indices()
        return m

    K = sym(g[i] * g[j] * W, g * g + float(noise_var))
    out = [sym(g[i] * g[j] * wendland_dr(rho, float(radius), kernel), np.zeros(n))]
    for k in range(b.shape[1]):
        bk = b[:, k]
        out.append(sym((bk[i] * g[j] + g[i] * bk[j]) * W, 2.0 * bk * g))
    out.append(sp.identity(n, format="csr"))
    return K, out


def lml_components(K, y):
    """Exact LML of a sparse K through the connected components of its pattern: K is
    block diagonal over them (after a permutation), so ln|K| and y^T K^-1 y are sums
    of per-component dense Cholesky values. Returns an oracle.dense.LMLResult."""
    from scipy.sparse.csgraph import connected_components
    from .dense import LMLResult, lml_dense

    K = sp.csr_matrix(K)
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    ncomp, lab = connected_components(K, directed=False)
    order = np.argsort(lab, kind="stable")
    bounds = np.searchsorted(lab[order], np.arange(ncomp + 1))
    a = np.zeros(n)
    logdet = 0.0
    for c in range(ncomp):
        idx = order[bounds[c]:bounds[c + 1]]
        res = lml_dense(K[idx][:, idx].toarray(), y[idx])
        logdet += res.logdet
        a[idx] = res.a
    yTa = float(y @ a)
    return LMLResult(-0.5 * yTa - 0.5 * logdet - 0.5 * n * np.log(2.0 * np.pi), logdet, yTa, a)


def lanczos_logquad(alphas, betas):
    """e_1^T ln(T) e_1 for the Lanczos tridiagonal T that a CG run with coefficients
    (alpha_j, beta_j) builds (Golub-Welsch: T = V diag(theta) V^T, here the dense
    symmetric eigendecomposition of T; the quadrature is
    sum_k V_0k^2 ln theta_k):
      T_00 = 1/alpha_0,  T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
      T_j,j+1 = T_j+1,j = sqrt(beta_j)/alpha_j."""
    al = np.asarray(alphas, dtype=np.float64)
    be = np.asarray(betas, dtype=np.float64)
    m = al.shape[0]
    d = 1.0 / al
    d[1:] += be[:m - 1] / al[:m - 1]
    e = np.sqrt(be[:m - 1]) / al[:m - 1]
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    theta, V = np.linalg.eigh(T)
    return float(np.sum(V[0] ** 2 * np.log(theta)))


def lml_grad_sparse(x, y, radius, bump_width, centers, weights, noise_var, Z, tol=1e-8, probe_tol=1e-8,
                    max_iter=200000, kernel="c2"):
    """The whole LML and gradient on the sparse path, diagonal preconditioner M = D:

    a      = K^-1 y                         (pcg_jacobi to ||y - K a|| <= tol ||y||)
    q_s    = K^-1 D^1/2 z_s                 (pcg_jacobi per probe, probe_tol)
    Gamma  = ln|D| + (1/S) sum_s ||z_s||^2 e_1^T ln(T_s) e_1
             (T_s the Lanczos tridiagonal of the probe's CG coefficients: PCG with
             M = D on K q = D^1/2 z is CG on Khat = D^-1/2 K D^-1/2 started from z)
    LML    = -1/2 y^T a - 1/2 Gamma - N/2 ln(2 pi)
    w_s    = D^-1/2 z_s
    grad   = 1/2 a^T dK a - 1/2 (1/S) sum_s q_s^T dK w_s, per theta in (r, a_1..a_P, sigma_n^2).

    Returns (lml, grad, parts); the same-probe dense values (oracle.estimators with
    blocks=None) are its limit as both tolerances go to zero."""
    K, dKs = dcov_csr(x, radius, bump_width, centers, weights, noise_var, kernel)
    y = np.asarray(y, dtype=np.float64)
    Z = np.atleast_2d(np.asarray(Z, dtype=np.float64))
    n = y.shape[0]
    S = Z.shape[0]
    D = K.diagonal()
    a, it_y, _, _ = pcg_jacobi(K, y, tol=tol, max_iter=max_iter)
    Q = np.zeros((n, S))
    quad = np.zeros(S)
    iters = np.zeros(S, dtype=np.int64)
    for s in range(S):
        q, it, al, be = pcg_jacobi(K, np.sqrt(D) * Z[s], tol=probe_tol, max_iter=max_iter)
        Q[:, s] = q
        iters[s] = it
        quad[s] = float(Z[s] @ Z[s]) * lanczos_logquad(al, be) if it > 0 else 0.0
    gamma = float(np.sum(np.log(D)) + quad.mean())
    yTa = float(y @ a)
    lml = -0.5 * yTa - 0.5 * gamma - 0.5 * n * np.log(2.0 * np.pi)
    Wm = Z.T / np.sqrt(D)[:, None]
    fit = np.array([0.5 * float(a @ (dK @ a)) for dK in dKs])
    tau = np.array([float(np.sum(Q * (dK @ Wm))) / S for dK in dKs])
    return lml, fit - 0.5 * tau, dict(fit=fit, tau=tau, gamma=gamma, yTa=yTa, a=a, iters_y=it_y,
                                      iters_probe=iters, quad=quad, nnz=K.nnz)
