"""Same-probe stochastic estimators, evaluated exactly (dense eigen-decomposition and
dense inverse) for a given set of Rademacher probes and a given preconditioner.

The paper computes ln|K| on the host with an unnamed method (Sec. 4.6, App. B.6,
"LOGDET"). The GPU path estimates it from preconditioned conjugate gradients on
right-hand sides L z_s with Lanczos quadrature, where M = L L^T is the
preconditioner (``oracle.precond``: the diagonal of K, L = D^{1/2}, or its block
diagonal over runs of the binned point order, L the blockwise Cholesky factor). In
exact arithmetic and at full Krylov dimension that estimate equals the quantity
below, which is its plain definition:

    Khat = L^-1 K L^-T
    Gamma = ln|M| + (1/S) sum_s z_s^T ln(Khat) z_s

(ln|K| = ln|M| + ln|Khat|, ln|Khat| = tr ln Khat, and E[z z^T] = I for Rademacher
z, so Gamma is an unbiased estimate of ln|K|; preconditioned CG on K x = L z is CG
on Khat with right-hand side z.) Likewise the trace in the gradient,

    tr(K^{-1} dK) = tr(L^T K^{-1} dK L^{-T}) ~ tau = (1/S) sum_s q_s^T dK w_s,
    q_s = K^{-1} L z_s,   w_s = L^{-T} z_s,

and the same-probe gradient  Ghat = 1/2 a^T dK a - 1/2 tau. (w_s = M^-1 L z_s is
the preconditioned initial residual of the probe solve.) ``blocks=None`` means
one-point blocks (Jacobi).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .dense import dcov_dense, lml_dense
from .precond import block_factor


def _factor(K, blocks):
    """(L, Linv, ln|M|); blocks=None: the diagonal, L = D^{1/2} (built directly, as a
    matrix of one-point blocks would be)."""
    if blocks is None:
        d = np.diag(K).copy()
        if np.any(d <= 0):
            raise np.linalg.LinAlgError("diagonal not positive")
        return np.diag(np.sqrt(d)), np.diag(1.0 / np.sqrt(d)), float(np.sum(np.log(d)))
    return block_factor(K, blocks)


def _whiten(K, Linv, blocks):
    """Khat = Linv K Linv^T (a diagonal Linv is applied as a row and column scaling)."""
    if blocks is None:
        s = np.diag(Linv)
        return K * s[:, None] * s[None, :]
    Kh = Linv @ K @ Linv.T
    return 0.5 * (Kh + Kh.T)


def logdet_same_probe(K, Z, blocks=None):
    """Gamma and the per-probe terms z_s^T ln(Khat) z_s (eigh of Khat)."""
    K = np.asarray(K, dtype=np.float64)
    _, Linv, logdet_m = _factor(K, blocks)
    Khat = _whiten(K, Linv, blocks)
    lam, V = np.linalg.eigh(Khat)
    if lam.min() <= 0:
        raise np.linalg.LinAlgError("covariance not positive definite")
    proj = V.T @ np.asarray(Z, dtype=np.float64).T          # (n, S)
    terms = (proj ** 2 * np.log(lam)[:, None]).sum(axis=0)  # (S,)
    return float(logdet_m + terms.mean()), terms


def hutchinson_variance(A, n_probes):
    """Variance of the S-probe Rademacher trace estimate of tr(A) for symmetric A:
    2 (||A||_F^2 - sum_i A_ii^2) / S."""
    A = np.asarray(A, dtype=np.float64)
    return 2.0 * (np.sum(A * A) - np.sum(np.diag(A) ** 2)) / n_probes


def grad_same_probe(x, y, Z, radius, bump_width, centers, weights, noise_var, K=None, kernel="c2", blocks=None,
                    dcov=None):
    """Ghat (P+2,) in the order (r, a_1..a_P, sigma_n^2), plus its halves. dcov = (K, [dK])
    of another kernel (``oracle.wendconv.dcov_dense``) replaces the stationary one."""
    K_, dKs = dcov if dcov is not None else dcov_dense(x, radius, bump_width, centers, weights, noise_var, kernel)
    K = K_ if K is None else np.asarray(K, dtype=np.float64)
    res = lml_dense(K, y)
    L, Linv, _ = _factor(K, blocks)
    Z = np.asarray(Z, dtype=np.float64)
    c = scipy.linalg.cho_factor(K, lower=True)
    Q = scipy.linalg.cho_solve(c, L @ Z.T)                      # (n, S) = q_s columns
    Wm = Linv.T @ Z.T                                           # (n, S) = w_s columns
    S = Z.shape[0]
    fit = np.array([0.5 * res.a @ (dK @ res.a) for dK in dKs])
    tau = np.array([float(np.sum(Q * (dK @ Wm))) / S for dK in dKs])
    return fit - 0.5 * tau, dict(fit=fit, tau=tau, lml=res)


def lml_same_probe(K, y, Z, blocks=None):
    """LMLhat = -1/2 y^T a - 1/2 Gamma - N/2 ln(2 pi)."""
    res = lml_dense(K, y)
    gamma, terms = logdet_same_probe(K, Z, blocks)
    n = len(y)
    return -0.5 * res.yTa - 0.5 * gamma - 0.5 * n * np.log(2 * np.pi), dict(
        gamma=gamma, terms=terms, yTa=res.yTa, logdet=res.logdet, a=res.a)
