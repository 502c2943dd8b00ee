"""Pins of the non-stationary, axis-anisotropic Wendland kernel (Eq. wendconv with the
bump-driven length-scale field) in oracle.wendconv.

- With every c_q = 0 and equal radii it is the stationary kernel of oracle.dense
  (covariance, its derivatives, the sparse matrix and the cross-covariance).
- On points along one axis only that axis's radius matters (the radii are not mixed up).
- The prefactor at coincident points is sech(ln l_i - ln l_j)^{d/2} (closed form of
  (l_i l_j / m)^{d/2}), at most 1.
- Every component of the exact gradient matches central differences of the exact LML.
- The sparse matrix equals the dense one, the cross-covariance at training points is K
  without the noise, and l(x) never exceeds its parameter bound.
- The construction is not positive semi-definite in general with a Wendland core (the
  cited argument needs a Gaussian scale mixture): a recorded C^6 case has a negative
  eigenvalue far beyond rounding.
Planted mistakes (a wrong prefactor power, a halved Wendland derivative, swapped
radii) fail one of them."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import wendconv as WC


def _prob(seed=7, n=160, dim=2, r=0.25):
    return workloads.make_random_problem(seed, n, dim, r, n_bumps=3, bump_width=0.7, noise_var=1e-2)


@pytest.mark.parametrize("kernel", ["c2", "c6"])
def test_stationary_limit(kernel):
    p = _prob()
    kw = dict(bump_width=p.bump_width, centers=p.centers, weights=p.weights, noise_var=p.noise_var, kernel=kernel)
    K0, d0 = oracle.dcov_dense(p.x, p.radius, **kw)
    K1, d1 = WC.dcov_dense(p.x, p.radius, ls_weights=None, **kw)
    K2, d2 = WC.dcov_dense(p.x, [p.radius, p.radius], ls_weights=np.zeros(3), **kw)
    scale = np.abs(K0).max()
    assert np.abs(K1 - K0).max() <= 1e-14 * scale and np.abs(K2 - K0).max() <= 1e-14 * scale
    for a, b in zip(d0, d1):
        assert np.abs(a - b).max() <= 1e-12 * max(np.abs(a).max(), 1e-300)
    # ARD radius components sum to the isotropic one; a_q and sigma^2 unchanged
    np.testing.assert_allclose(d2[0] + d2[1], d0[0], rtol=0, atol=1e-12 * np.abs(d0[0]).max())
    for q in range(3):
        np.testing.assert_allclose(d2[2 + q], d0[1 + q], rtol=0, atol=1e-13 * np.abs(d0[1 + q]).max())
    Ks = WC.covariance_csr(p.x, [p.radius] * 2, p.bump_width, p.centers, p.weights, p.noise_var, np.zeros(3),
                           kernel)
    np.testing.assert_allclose(Ks.toarray(), K0, rtol=0, atol=1e-14 * scale)


def test_axis_line_sees_only_its_radius():
    p = _prob(n=80)
    x = p.x.copy()
    x[:, 1] = 0.4  # all points on the line y = 0.4
    kw = dict(bump_width=p.bump_width, centers=p.centers, weights=p.weights, noise_var=p.noise_var)
    K_ard = WC.covariance_dense(x, [0.2, 0.05], **kw)
    K_iso = oracle.covariance_dense(x, 0.2, **kw)
    np.testing.assert_allclose(K_ard, K_iso, rtol=1e-13, atol=1e-15)
    assert np.abs(WC.covariance_dense(x, [0.05, 0.2], **kw) - K_iso).max() > 1e-3


@pytest.mark.parametrize("dim", [2, 3])
def test_prefactor_at_coincident_points(dim):
    # two copies of one point with different length scales: K_12 = g^2 sech(u_1 - u_2)^{d/2}
    x = np.full((2, dim), 0.5)
    la, lb = np.array([np.exp(0.4), np.exp(-0.3)]), np.array([np.exp(0.4), np.exp(-0.3)])
    d, m, Q, p = WC.geometry(x, x, np.full(dim, 0.2), la, lb)
    assert Q[0, 1] == 0.0
    assert p[0, 1] == pytest.approx((1.0 / np.cosh(0.7)) ** (dim / 2), rel=1e-14)
    assert p[0, 0] == 1.0 and p[0, 1] < 1.0


@pytest.mark.parametrize("kernel,dim,ard", [("c2", 2, True), ("c6", 2, False), ("c2", 3, True)])
def test_gradient_matches_central_differences(kernel, dim, ard):
    p = _prob(seed=11 + dim, n=120, dim=dim, r=0.3)
    c = np.array([0.6, -0.4, 0.3])
    radius = np.array([0.3, 0.22, 0.26][:dim]) if ard else 0.27
    kw = dict(bump_width=p.bump_width, centers=p.centers, kernel=kernel)

    def lml(theta):
        nr = dim if ard else 1
        r = theta[:nr] if ard else theta[0]
        K = WC.covariance_dense(p.x, r, weights=theta[nr:nr + 3], ls_weights=theta[nr + 3:nr + 6],
                                noise_var=theta[-1], **kw)
        return oracle.lml_dense(K, p.y).lml
    theta = np.concatenate([np.atleast_1d(radius), p.weights, c, [p.noise_var]])
    dc = WC.dcov_dense(p.x, radius, weights=p.weights, ls_weights=c, noise_var=p.noise_var, **kw)
    g, _ = oracle.grad_exact(p.x, p.y, radius, p.bump_width, p.centers, p.weights, p.noise_var, dcov=dc)
    assert len(g) == len(theta)
    for k in range(len(theta)):
        h = 1e-6 * max(abs(theta[k]), 1e-2)
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (lml(tp) - lml(tm)) / (2 * h)
        assert fd == pytest.approx(g[k], rel=2e-6, abs=1e-6 * np.abs(g).max()), (k, fd, g[k])


@pytest.mark.parametrize("dim,kernel", [(2, "c2"), (3, "c6")])
def test_sparse_equals_dense_and_cross_at_training_points(dim, kernel):
    p = _prob(seed=21, n=400, dim=dim, r=0.15)
    c = np.array([0.9, -0.7, 0.4])
    radii = np.array([0.15, 0.1, 0.12][:dim])
    args = (p.x, radii, p.bump_width, p.centers, p.weights, p.noise_var)
    Kd = WC.covariance_dense(*args, ls_weights=c, kernel=kernel)
    Ks = WC.covariance_csr(*args, ls_weights=c, kernel=kernel)
    np.testing.assert_allclose(Ks.toarray(), Kd, rtol=0, atol=1e-14 * np.abs(Kd).max())
    assert Ks.nnz > 2 * p.n
    Kx, gs = WC.cross_covariance(p.x[:50], p.x, radii, p.bump_width, p.centers, p.weights, c, kernel)
    ref = Kd[:50].copy()
    ref[np.arange(50), np.arange(50)] -= p.noise_var
    np.testing.assert_allclose(Kx, ref, rtol=0, atol=1e-14 * np.abs(Kd).max())
    ell, _ = WC.length_scale(p.x, p.centers, p.bump_width, c)
    assert ell.max() <= WC.ell_bound(c) and ell.min() >= np.exp(-0.7) * (1 - 1e-15)


def test_not_positive_semidefinite_in_general():
    # C^6 member, 2-D, ARD radii, length-scale weights of both signs
    rng = np.random.default_rng(6)
    p = workloads.make_random_problem(106, 400, 2, 0.2, n_bumps=4, bump_width=0.6)
    radii = rng.uniform(0.05, 0.3, 2)
    c = rng.uniform(-2, 2, 4)
    K = WC.covariance_dense(p.x, radii, p.bump_width, p.centers, p.weights, 0.0, ls_weights=c, kernel="c6")
    ev = np.linalg.eigvalsh(K)
    assert ev.min() < -1e-7 * ev.max()
    # the stationary kernel on the same points is positive semi-definite to rounding
    K0 = WC.covariance_dense(p.x, radii, p.bump_width, p.centers, p.weights, 0.0, kernel="c6")
    ev0 = np.linalg.eigvalsh(K0)
    assert ev0.min() > -1e-12 * ev0.max()


def _fails(fn, *a):
    with pytest.raises(AssertionError):
        fn(*a)


def test_planted_mistakes_fail(monkeypatch):
    real_geometry = WC.geometry

    def wrong_power(xa, xb, radii, la, lb):
        d, m, Q, p = real_geometry(xa, xb, radii, la, lb)
        return d, m, Q, p ** 2  # (l l / m)^d instead of ^{d/2}
    monkeypatch.setattr(WC, "geometry", wrong_power)
    _fails(test_prefactor_at_coincident_points, 2)
    monkeypatch.setattr(WC, "geometry", real_geometry)

    def swapped(xa, xb, radii, la, lb):
        return real_geometry(xa, xb, radii[::-1], la, lb)
    monkeypatch.setattr(WC, "geometry", swapped)
    _fails(test_axis_line_sees_only_its_radius)
    monkeypatch.setattr(WC, "geometry", real_geometry)

    real_dlog = WC.wendland_dlog
    monkeypatch.setattr(WC, "wendland_dlog", lambda rho, kernel="c2": 0.5 * real_dlog(rho, kernel))
    _fails(test_gradient_matches_central_differences, "c2", 2, True)
