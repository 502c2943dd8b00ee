"""Pins of the posterior oracle (Sec. 3, Eq. posterior) against facts it must satisfy:

* the Gaussian conditioning identity through the inverse of the joint covariance of
  (y, f*), built by the training-matrix code on the augmented point set;
* exact identities at the training points: mean = y - sigma^2 a and
  var = sigma^2 - sigma^4 [K^{-1}]_ii (k(X, x_i) = K e_i - sigma^2 e_i);
* the one-point closed form;
* the support special cases and the prior bound 0 <= var <= g(x*)^2;
* planted mistakes that each pin catches.
"""
import numpy as np
import pytest

import oracle


def _problem(seed=3, n=60, dim=2, radius=0.3, noise=1e-3):
    rng = np.random.default_rng(seed)
    x = rng.random((n, dim))
    centers = rng.random((3, dim))
    weights = rng.uniform(0.5, 1.5, 3)
    y = np.sin(5 * x[:, 0]) + 0.1 * rng.standard_normal(n)
    return x, y, dict(radius=radius, bump_width=0.7, centers=centers, weights=weights, noise_var=noise)


def _joint_inverse(x, y, xs, p):
    """Mean and variance at one test point from the inverse of the joint covariance."""
    xa = np.vstack([x, xs[None, :]])
    Ka = oracle.covariance_dense(xa, **p)
    Ka[-1, -1] -= p["noise_var"]  # f* carries no observation noise
    M = np.linalg.inv(Ka)
    var = 1.0 / M[-1, -1]
    mean = -(M[-1, :-1] @ y) * var
    return mean, var


@pytest.mark.parametrize("dim", [2, 3])
def test_conditioning_identity(dim):
    x, y, p = _problem(dim=dim, radius=0.35 if dim == 3 else 0.3)
    xt = np.random.default_rng(9).random((12, dim))
    mean, var, _ = oracle.posterior_dense(x, y, xt, **p)
    gt, _, gam = oracle.bump_values(xt, p["centers"], p["bump_width"], p["weights"])
    assert gam.sum() >= 6
    for t in range(len(xt)):
        if not gam[t]:  # no prior variance: the joint covariance is singular
            assert mean[t] == 0.0 and var[t] == 0.0
            continue
        m2, v2 = _joint_inverse(x, y, xt[t], p)
        assert abs(mean[t] - m2) <= 1e-9 * (1 + abs(m2))
        assert abs(var[t] - v2) <= 1e-9 * (1 + abs(v2))


def test_training_point_identities():
    x, y, p = _problem()
    mean, var, a = oracle.posterior_dense(x, y, x, **p)
    K = oracle.covariance_dense(x, **p)
    Kinv = np.linalg.inv(K)
    s2 = p["noise_var"]
    np.testing.assert_allclose(mean, y - s2 * a, rtol=0, atol=1e-10 * np.abs(y).max())
    np.testing.assert_allclose(var, s2 - s2 ** 2 * np.diag(Kinv), rtol=0, atol=1e-12)


def test_one_point_closed_form():
    x = np.array([[0.40, 0.50]])
    y = np.array([0.7])
    p = dict(radius=0.5, bump_width=0.9, centers=np.array([[0.5, 0.5]]), weights=np.array([1.3]), noise_var=0.01)
    xt = np.array([[0.55, 0.42]])
    mean, var, _ = oracle.posterior_dense(x, y, xt, **p)
    g = lambda z: 1.3 * np.exp(1 - 1 / (1 - np.sum((z - 0.5) ** 2) / 0.81))
    rho = np.linalg.norm(x[0] - xt[0]) / 0.5
    k = g(xt[0]) * g(x[0]) * (1 - rho) ** 4 * (4 * rho + 1)
    d = g(x[0]) ** 2 + 0.01
    assert mean[0] == pytest.approx(k * 0.7 / d, rel=1e-13)
    assert var[0] == pytest.approx(g(xt[0]) ** 2 - k * k / d, rel=1e-13)


def test_support_special_cases_and_bounds():
    x, y, p = _problem(radius=0.1)
    p["centers"] = np.array([[0.3, 0.3]])
    p["weights"] = np.array([1.0])
    p["bump_width"] = 0.5
    far = np.array([[0.95, 0.95]])           # outside the bump: no prior variance
    inside = np.array([[0.3, 0.3]])
    gs, _, _ = oracle.bump_values(inside, p["centers"], p["bump_width"], p["weights"])
    # a training set with no point within r of `inside`
    keep = np.linalg.norm(x - inside, axis=1) >= p["radius"]
    mean, var, _ = oracle.posterior_dense(x[keep], y[keep], np.vstack([far, inside]), **p)
    assert mean[0] == 0.0 and var[0] == 0.0
    assert mean[1] == 0.0 and var[1] == pytest.approx(gs[0] ** 2, rel=1e-15)
    xt = np.random.default_rng(4).random((40, 2))
    mean, var, _ = oracle.posterior_dense(x, y, xt, **p)
    gt, _, _ = oracle.bump_values(xt, p["centers"], p["bump_width"], p["weights"])
    assert np.all(var >= -1e-12) and np.all(var <= gt ** 2 + 1e-12)


def test_planted_mistakes_fail_a_pin():
    x, y, p = _problem()
    K = oracle.covariance_dense(x, **p)
    Ks, gs = oracle.cross_covariance(x, x, p["radius"], p["bump_width"], p["centers"], p["weights"])
    s2 = p["noise_var"]
    a = np.linalg.solve(K, y)
    Kinv = np.linalg.inv(K)
    good_var = s2 - s2 ** 2 * np.diag(Kinv)
    # noise left out of the solve
    Kf = K - s2 * np.eye(len(x))
    Kf += 1e-9 * np.eye(len(x))
    bad_var = gs ** 2 - np.einsum("tj,jt->t", Ks, np.linalg.solve(Kf, Ks.T))
    assert np.abs(bad_var - good_var).max() > 1e-6
    # noise wrongly added to k(x*, x*)
    bad_var = gs ** 2 + s2 - np.einsum("tj,jt->t", Ks, Kinv @ Ks.T)
    assert np.abs(bad_var - good_var).max() > 1e-6
    # cross-covariance missing the test point's bump factor
    Ks_bad = Ks / np.where(gs[:, None] > 0, gs[:, None], 1.0)
    assert np.abs(Ks_bad @ a - (y - s2 * a)).max() > 1e-3
