"""Posterior mean and variance of the latent function at test points (dense, float64).

Sec. 3, Eq. posterior, with zero prior mean: for a test point x*,

    mean(x*) = k(X, x*)^T K^{-1} y
    var(x*)  = k(x*, x*) - k(X, x*)^T K^{-1} k(X, x*)

where K is the training covariance including the noise on its diagonal (the
normal likelihood of Sec. 3 with V = sigma_n^2 I) and k is the noise-free kernel
(Sec. 4.1 product construction, Sec. 4.3 bump mask), so k(x*, x*) = g(x*)^2 W(0)
= g(x*)^2: the posterior of the latent f*, not of a new noisy observation.
App. B.7 keeps K^{-1} y for the mean; the variance needs one solve per test point.

The cross-covariance uses the same structural pattern as the training matrix: a
pair contributes when ||x* - x_j|| < r and both points lie strictly inside some
bump. A test point that coincides with a training point gets no noise term (the
noise belongs to the observations).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .dense import covariance_dense
from .kernel import bump_values, wendland
from .pattern import pairwise_sqdist


def cross_covariance(x_test, x, radius, bump_width, centers, weights, kernel="c2"):
    """k(x*_t, x_j) for every test point t and training point j (n_test x N)."""
    x_test = np.asarray(x_test, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    gs, _, gams = bump_values(x_test, centers, bump_width, weights)
    g, _, gam = bump_values(x, centers, bump_width, weights)
    d2 = pairwise_sqdist(x_test, x)
    keep = (d2 < float(radius) ** 2) & gams[:, None] & gam[None, :]
    rho = np.sqrt(d2) / float(radius)
    return np.where(keep, gs[:, None] * g[None, :] * wendland(rho, kernel), 0.0), gs


def posterior_dense(x, y, x_test, radius, bump_width, centers, weights, noise_var, K=None, kernel="c2"):
    """(mean, var, a) at the test points, by Cholesky of the dense training K.

    K may be given (for instance the matrix a device path stored, in user order);
    otherwise it is built from the points."""
    if K is None:
        K = covariance_dense(x, radius, bump_width, centers, weights, noise_var, kernel=kernel)
    Ks, gs = cross_covariance(x_test, x, radius, bump_width, centers, weights, kernel)
    c = scipy.linalg.cho_factor(K, lower=True)
    a = scipy.linalg.cho_solve(c, np.asarray(y, dtype=np.float64))
    V = scipy.linalg.cho_solve(c, Ks.T)
    mean = Ks @ a
    var = gs ** 2 - np.einsum("tj,jt->t", Ks, V)
    return mean, var, a
