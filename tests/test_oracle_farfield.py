"""Pins of the far-field bump kernel (Eq. bump_kernel, core kernel 1) in oracle.farfield.

- A worked three-point case: two points farther apart than r inside one bump
  interact only through the bump term a^2 b(x_0) b(x_1) (b = exp(1 - 1/(1 - s))); a
  point outside every bump interacts with its neighbour only through W (W(1/2) = 3/16).
- Grouping: two bumps in one group add the cross term a_1 a_2 (b_1 b_2^T + b_2 b_1^T)
  to the covariance of the same bumps in separate groups.
- K - K_loc has rank at most U; the matrix determinant lemma ln|K| = ln|K_loc| +
  ln|I + G^T K_loc^-1 G| holds (the operator the device applies is K_loc + G G^T).
- Every gradient component matches central differences of the exact LML.
- The sparse local matrix equals the dense one; the cross-covariance at training
  points is K without the noise.
Planted mistakes (a wrong group, a one-sided amplitude derivative) fail."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import farfield as FF


def test_worked_three_points():
    # one bump at (0.5, 0.5), width 0.4, amplitude 1.3; r = 0.2
    c = np.array([[0.5, 0.5]])
    b = np.exp(1.0 - 1.0 / 0.75)  # the bump at s = ||x - c||^2 / w^2 = 1/4
    # points 0 and 1 at s = 1/4, sqrt(0.08) > r apart; point 2 on the bump's boundary (outside)
    x = np.array([[0.5, 0.3], [0.7, 0.5], [0.9, 0.5]])
    K = FF.covariance_dense(x, 0.2, 0.4, c, [1.3], 1e-3, groups=[0])
    assert K[0, 1] == pytest.approx(1.3 ** 2 * b * b, rel=1e-14)
    assert K[1, 2] == 0.0 and K[0, 2] == 0.0
    assert K[0, 0] == pytest.approx(1.3 ** 2 * b * b + 1.0 + 1e-3, rel=1e-14)
    # points 1 and 2 outside the bump, 0.1 = r/2 apart: only W(1/2) = 3/16
    x3 = np.array([[0.5, 0.3], [0.95, 0.5], [1.05, 0.5]])
    K3 = FF.covariance_dense(x3, 0.2, 0.4, c, [1.3], 1e-3, groups=[0])
    assert K3[1, 2] == pytest.approx(3.0 / 16.0, rel=1e-14)
    assert K3[0, 1] == 0.0 and K3[0, 2] == 0.0


def test_grouping_adds_the_cross_term():
    p = workloads.make_random_problem(3, 90, 2, 0.1, n_bumps=2, bump_width=0.6)
    a = np.array([0.8, 1.4])
    Ks = FF.covariance_dense(p.x, 0.1, 0.6, p.centers, a, 1e-3, groups=[0, 0])
    Kd = FF.covariance_dense(p.x, 0.1, 0.6, p.centers, a, 1e-3, groups=[0, 1])
    _, bhat, _ = oracle.bump_values(p.x, p.centers, 0.6, np.ones(2))
    cross = a[0] * a[1] * (np.outer(bhat[:, 0], bhat[:, 1]) + np.outer(bhat[:, 1], bhat[:, 0]))
    np.testing.assert_allclose(Ks - Kd, cross, rtol=0, atol=1e-13)


def test_low_rank_structure_and_determinant_lemma():
    p = workloads.make_random_problem(4, 300, 2, 0.08, n_bumps=4, bump_width=0.5)
    groups = [0, 1, 0, 2]
    K = FF.covariance_dense(p.x, 0.08, 0.5, p.centers, p.weights, 1e-3, groups)
    Kl = FF.local_dense(p.x, 0.08, 1e-3)
    s = np.linalg.svd(K - Kl, compute_uv=False)
    assert np.all(s[3:] <= 1e-12 * s[0]) and s[2] > 1e-6 * s[0]
    G, _ = FF.group_values(p.x, p.centers, 0.5, p.weights, groups)
    lhs = np.linalg.slogdet(K)[1]
    rhs = np.linalg.slogdet(Kl)[1] + np.linalg.slogdet(np.eye(3) + G.T @ np.linalg.solve(Kl, G))[1]
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("kernel", ["c2", "c6"])
def test_gradient_matches_central_differences(kernel):
    p = workloads.make_random_problem(5, 150, 2, 0.15, n_bumps=3, bump_width=0.5, noise_var=1e-2)
    groups = [0, 1, 0]

    def lml(theta):
        K = FF.covariance_dense(p.x, theta[0], 0.5, p.centers, theta[1:4], theta[4], groups, kernel)
        return oracle.lml_dense(K, p.y).lml
    theta = np.concatenate([[0.15], p.weights, [1e-2]])
    dc = FF.dcov_dense(p.x, 0.15, 0.5, p.centers, p.weights, 1e-2, groups, kernel)
    g, _ = oracle.grad_exact(p.x, p.y, 0.15, 0.5, p.centers, p.weights, 1e-2, dcov=dc)
    for k in range(len(theta)):
        h = 1e-6 * abs(theta[k])
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (lml(tp) - lml(tm)) / (2 * h)
        assert fd == pytest.approx(g[k], rel=2e-6, abs=1e-6 * np.abs(g).max()), (k, fd, g[k])


def test_sparse_local_and_cross_at_training_points():
    p = workloads.make_random_problem(6, 500, 3, 0.15, n_bumps=3, bump_width=0.5)
    groups = [0, 1, 1]
    np.testing.assert_allclose(FF.local_csr(p.x, 0.15, 1e-3, "c6").toarray(), FF.local_dense(p.x, 0.15, 1e-3, "c6"),
                               rtol=0, atol=1e-15)
    K = FF.covariance_dense(p.x, 0.15, 0.5, p.centers, p.weights, 1e-3, groups)
    Kx, prior = FF.cross_covariance(p.x[:40], p.x, 0.15, 0.5, p.centers, p.weights, groups)
    ref = K[:40].copy()
    ref[np.arange(40), np.arange(40)] -= 1e-3
    np.testing.assert_allclose(Kx, ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(prior, np.diag(K)[:40] - 1e-3, rtol=1e-14)


def _fails(fn, *a):
    with pytest.raises(AssertionError):
        fn(*a)


def test_planted_mistakes_fail(monkeypatch):
    real = FF.group_values

    def merged(x, centers, bump_width, weights, groups):
        return real(x, centers, bump_width, weights, np.zeros_like(np.asarray(groups)))
    monkeypatch.setattr(FF, "group_values", merged)
    _fails(test_grouping_adds_the_cross_term)
    monkeypatch.setattr(FF, "group_values", real)

    real_outer = np.outer
    calls = {"n": 0}

    def one_sided(a, b):
        calls["n"] += 1
        return real_outer(a, b) if calls["n"] % 2 else 0.0 * real_outer(a, b)
    monkeypatch.setattr(FF.np, "outer", one_sided)
    _fails(test_gradient_matches_central_differences, "c2")
