"""Pins for the dense covariance, log marginal likelihood and exact gradient."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats
from scipy.spatial.distance import cdist

import oracle
import workloads


def _small(seed=1, n=300, dim=2, r=0.15, P=3, w=0.5, noise=1e-3, points="uniform"):
    return workloads.make_random_problem(seed, n, dim, r, n_bumps=P, bump_width=w,
                                         noise_var=noise, points=points)


def _K(p):
    return oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)


def test_bitwise_symmetric_and_psd():
    """Theorem 1 (App. A): f(x)f(x')k(x,x') is a valid kernel, so K - sigma^2 I is PSD."""
    p = _small()
    K = _K(p)
    assert np.array_equal(K, K.T)
    lam = np.linalg.eigvalsh(K)
    assert lam.min() >= p.noise_var * (1 - 1e-9)


def test_rank_one_bump_mask():
    """With r far beyond the cloud, W ~ 1 and K - sigma^2 I ~ g g^T (rank 1), the
    'box' structure of the product bump kernel (Sec. 4.3, App. C.1)."""
    p = _small(n=120, r=1e7, w=0.45)
    K = _K(p)
    g, _, _ = oracle.bump_values(p.x, p.centers, p.bump_width, p.weights)
    A = K - p.noise_var * np.eye(p.n)
    np.testing.assert_allclose(A, np.outer(g, g), rtol=0, atol=1e-12 * np.max(g) ** 2)
    sv = np.linalg.svd(A, compute_uv=False)
    assert sv[1] < 1e-10 * sv[0]


def test_two_point_closed_form():
    x = np.array([[0.2, 0.3], [0.23, 0.34]])
    r, w = 0.1, 0.5
    c = np.array([[0.25, 0.25]])
    wt = np.array([1.3])
    noise = 0.01
    y = np.array([0.7, -0.2])
    K = oracle.covariance_dense(x, r, w, c, wt, noise)
    b = [math.exp(1 - 1 / (1 - ((xi[0] - 0.25) ** 2 + (xi[1] - 0.25) ** 2) / w ** 2)) for xi in x]
    g = [1.3 * bi for bi in b]
    rho = 0.05 / r
    Wv = (1 - rho) ** 4 * (4 * rho + 1)
    A, B, C = g[0] ** 2 + noise, g[0] * g[1] * Wv, g[1] ** 2 + noise
    np.testing.assert_allclose(K, [[A, B], [B, C]], rtol=1e-14)
    det = A * C - B * B
    quad = (C * y[0] ** 2 - 2 * B * y[0] * y[1] + A * y[1] ** 2) / det
    res = oracle.lml_dense(K, y)
    assert res.logdet == pytest.approx(math.log(det), rel=1e-13)
    assert res.yTa == pytest.approx(quad, rel=1e-13)
    assert res.lml == pytest.approx(-0.5 * quad - 0.5 * math.log(det) - math.log(2 * math.pi), rel=1e-13)


def test_lml_matches_library_gaussian_density():
    p = _small(seed=4, n=400)
    K = _K(p)
    res = oracle.lml_dense(K, p.y)
    ref = scipy.stats.multivariate_normal(mean=np.zeros(p.n), cov=K).logpdf(p.y)
    assert res.lml == pytest.approx(ref, rel=1e-10)
    assert oracle.residual_rel(K, res.a, p.y) < 1e-12


def test_stationary_limit_textbook():
    """One very wide bump: g ~ const and K reduces to a Wendland GP built from
    library pairwise distances."""
    p = _small(seed=7, n=300, r=0.2)
    c = np.array([[0.5, 0.5]])
    wt = np.array([1.7])
    K = oracle.covariance_dense(p.x, p.radius, 1e4, c, wt, p.noise_var)
    g = 1.7 * np.exp(1 - 1 / (1 - np.sum((p.x - 0.5) ** 2, axis=1) / 1e8))
    rho = cdist(p.x, p.x) / p.radius
    Wm = np.where(rho < 1, (1 - rho) ** 4 * (4 * rho + 1), 0.0)
    Kt = np.outer(g, g) * Wm + p.noise_var * np.eye(p.n)
    np.testing.assert_allclose(K, Kt, rtol=1e-12, atol=1e-15)


def test_diagonal_case_closed_forms():
    """r below the minimum pair distance: K is diagonal, everything is closed form."""
    p = _small(seed=8, n=200, r=1e-6, P=2, w=0.6)
    K = _K(p)
    assert np.count_nonzero(K - np.diag(np.diag(K))) == 0
    g, b, _ = oracle.bump_values(p.x, p.centers, p.bump_width, p.weights)
    d = g * g + p.noise_var
    res = oracle.lml_dense(K, p.y)
    assert res.logdet == pytest.approx(np.sum(np.log(d)), rel=1e-13)
    np.testing.assert_allclose(res.a, p.y / d, rtol=1e-13)
    grad, _ = oracle.grad_exact(p.x, p.y, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    a = p.y / d
    expect = [0.0]
    for k in range(2):
        dk = 2 * g * b[:, k]
        expect.append(0.5 * np.sum(a * a * dk) - 0.5 * np.sum(dk / d))
    expect.append(0.5 * np.sum(a * a) - 0.5 * np.sum(1 / d))
    np.testing.assert_allclose(grad, expect, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,points,kernel", [(2, "uniform", "c2"), (3, "gmm", "c2"), (2, "uniform", "c6"),
                                               (3, "gmm", "c6")])
def test_gradient_matches_central_differences(dim, points, kernel):
    p = _small(seed=12, n=250, dim=dim, r=0.15 if dim == 2 else 0.25, P=3, w=0.55, points=points)
    grad, _ = oracle.grad_exact(p.x, p.y, p.radius, p.bump_width, p.centers, p.weights, p.noise_var, kernel=kernel)

    def lml(theta):
        K = oracle.covariance_dense(p.x, theta[0], p.bump_width, p.centers, theta[1:-1], theta[-1], kernel=kernel)
        return oracle.lml_dense(K, p.y).lml

    theta = np.concatenate([[p.radius], p.weights, [p.noise_var]])
    for k in range(len(theta)):
        h = 1e-5 * abs(theta[k])
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (lml(tp) - lml(tm)) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=2e-6, abs=1e-6 * max(1.0, abs(grad).max()))


@pytest.mark.parametrize("dim", [2, 3])
def test_c6_covariance_positive_definite(dim):
    """Eq. wendland's member is positive definite in up to three dimensions, so K - sigma^2 I
    (the noise-free part) has no negative eigenvalue on distinct points."""
    p = _small(seed=21, n=300, dim=dim, r=0.3, P=3, w=0.8, points="uniform")
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, 0.0, kernel="c6")
    lam = np.linalg.eigvalsh(K)
    assert lam.min() > -1e-12 * lam.max()
