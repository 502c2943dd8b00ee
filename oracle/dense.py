"""Dense float64 covariance, log marginal likelihood and its exact gradient.

For N up to a few thousand points. Everything follows the plain definitions:

* K_ij = g_i g_j W(||x_i - x_j|| / r) on the stored pattern, plus the noise
  variance on the diagonal (Sec. 4.1 product construction, Sec. 4.3 bump mask,
  Sec. 3 normal likelihood with noise matrix V = sigma_n^2 I);
* LML = -1/2 y^T K^{-1} y - 1/2 ln|K| - N/2 ln(2 pi) (Sec. 3, first displayed
  equation, zero prior mean; the paper writes it up to a constant, the constant
  is kept here);
* dLML/dtheta = 1/2 a^T (dK/dtheta) a - 1/2 tr(K^{-1} dK/dtheta), a = K^{-1} y,
  for theta = (r, a_1..a_P, sigma_n^2), the standard derivative of the Gaussian
  log density.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg

from .kernel import bump_values, wendland, wendland_dr


def _pattern_mask(d2, radius, gamma):
    keep = (d2 < float(radius) ** 2) & gamma[:, None] & gamma[None, :]
    np.fill_diagonal(keep, True)
    return keep


def covariance_dense(x, radius, bump_width, centers, weights, noise_var, return_parts=False, kernel="c2"):
    """Dense K (n x n, float64) on the structural pattern of oracle.pattern; `kernel`
    selects the Wendland member (oracle.kernel.wendland)."""
    from .pattern import pairwise_sqdist

    x = np.asarray(x, dtype=np.float64)
    g, b, gamma = bump_values(x, centers, bump_width, weights)
    d2 = pairwise_sqdist(x, x)
    keep = _pattern_mask(d2, radius, gamma)
    rho = np.sqrt(d2) / float(radius)
    W = np.where(keep, wendland(rho, kernel), 0.0)
    K = g[:, None] * g[None, :] * W
    K[np.diag_indices_from(K)] += float(noise_var)
    if return_parts:
        return K, dict(g=g, b=b, gamma=gamma, rho=rho, keep=keep, W=W)
    return K


def dcov_dense(x, radius, bump_width, centers, weights, noise_var, kernel="c2"):
    """List of dense dK/dtheta in the order (r, a_1..a_P, sigma_n^2).

    dK/dr      = g_i g_j dW/dr                      (Wendland derivative)
    dK/da_k    = (b_ik g_j + g_i b_jk) W_ij          (product rule on g_i g_j)
    dK/dsigma2 = I
    """
    K, parts = covariance_dense(x, radius, bump_width, centers, weights, noise_var,
                                return_parts=True, kernel=kernel)
    g, b, keep, rho, W = parts["g"], parts["b"], parts["keep"], parts["rho"], parts["W"]
    out = [g[:, None] * g[None, :] * np.where(keep, wendland_dr(rho, float(radius), kernel), 0.0)]
    for k in range(b.shape[1]):
        bk = b[:, k]
        out.append((bk[:, None] * g[None, :] + g[:, None] * bk[None, :]) * W)
    out.append(np.eye(x.shape[0]))
    return K, out


@dataclass
class LMLResult:
    lml: float
    logdet: float
    yTa: float
    a: np.ndarray


def lml_dense(K, y):
    """Cholesky K = L L^T; a = L^-T L^-1 y; ln|K| = 2 sum ln L_ii; LML as above."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    c, low = scipy.linalg.cho_factor(K, lower=True)
    a = scipy.linalg.cho_solve((c, low), y)
    logdet = 2.0 * float(np.sum(np.log(np.diag(c))))
    yTa = float(y @ a)
    lml = -0.5 * yTa - 0.5 * logdet - 0.5 * n * np.log(2.0 * np.pi)
    return LMLResult(lml, logdet, yTa, a)


def grad_exact(x, y, radius, bump_width, centers, weights, noise_var, kernel="c2", dcov=None):
    """Exact gradient (n_bumps + 2,) in the order (r, a_1..a_P, sigma_n^2), with
    K^{-1} formed from the Cholesky factor. Also returns the two halves
    (data-fit 1/2 a^T dK a and trace 1/2 tr(K^{-1} dK)) for diagnostics. dcov = (K, [dK])
    of another kernel replaces the stationary one."""
    K, dKs = dcov if dcov is not None else dcov_dense(x, radius, bump_width, centers, weights, noise_var, kernel)
    res = lml_dense(K, y)
    c = scipy.linalg.cho_factor(K, lower=True)
    Kinv = scipy.linalg.cho_solve(c, np.eye(K.shape[0]))
    fit = np.array([0.5 * res.a @ (dK @ res.a) for dK in dKs])
    trace = np.array([0.5 * float(np.sum(Kinv * dK)) for dK in dKs])
    return fit - trace, dict(fit=fit, trace=trace, lml=res)
