"""Pins for the probe generator and the same-probe estimators."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")))


def test_splitmix64_published_outputs():
    z = oracle.splitmix64(GOLD["seed"], np.arange(len(GOLD["outputs_hex"])))
    assert [int(v) for v in z] == [int(h, 16) for h in GOLD["outputs_hex"]]


def test_probe_indexing_and_masks():
    Z = oracle.rademacher_probes(123, 5, 40)
    # counter k = s * 2^40 + u: probe s at point u is the sign of output k
    for s in range(5):
        for u in (0, 7, 39):
            v = int(oracle.splitmix64(123, np.array([s * (1 << 40) + u]))[0])
            assert Z[s, u] == (-1.0 if v >> 63 else 1.0)
    m = oracle.probe_sign_masks(123, 5, 40)
    for s in range(5):
        assert np.array_equal(((m >> np.uint64(s)) & np.uint64(1)).astype(bool), Z[s] < 0)
    # roughly balanced
    Zb = oracle.rademacher_probes(0, 64, 4000)
    assert abs(Zb.mean()) < 0.01


def _problem(seed=3, n=300, r=0.12):
    return workloads.make_random_problem(seed, n, 2, r, n_bumps=3, bump_width=0.5, noise_var=1e-3)


def test_diagonal_case_estimators_exact():
    """Diagonal K: Khat = I, so Gamma = ln|K| and the Hutchinson trace is exact."""
    p = _problem(n=150, r=1e-6)
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    Z = oracle.rademacher_probes(5, 3, p.n)
    gam, terms = oracle.logdet_same_probe(K, Z)
    assert gam == pytest.approx(oracle.lml_dense(K, p.y).logdet, rel=1e-13)
    gh, _ = oracle.grad_same_probe(p.x, p.y, Z, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    ge, _ = oracle.grad_exact(p.x, p.y, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    np.testing.assert_allclose(gh, ge, rtol=1e-11, atol=1e-11)


def test_logdet_estimator_unbiased():
    """Gamma over independent probe sets scatters around ln|K| with the Rademacher
    variance 2(||A||_F^2 - sum A_ii^2)/S of A = ln(Khat)."""
    p = _problem()
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    exact = oracle.lml_dense(K, p.y).logdet
    D = np.diag(K)
    Kh = K / np.sqrt(np.outer(D, D))
    lam, V = np.linalg.eigh(Kh)
    A = (V * np.log(lam)) @ V.T
    S, reps = 8, 200
    sd = np.sqrt(oracle.hutchinson_variance(A, S))
    vals = np.array([oracle.logdet_same_probe(K, oracle.rademacher_probes(seed, S, p.n))[0]
                     for seed in range(reps)])
    assert abs(vals.mean() - exact) < 4 * sd / np.sqrt(reps)
    assert 0.7 < vals.std() / sd < 1.3


def test_gradient_estimator_unbiased():
    p = _problem(n=200)
    ge, parts = oracle.grad_exact(p.x, p.y, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    reps, S = 100, 8
    vals = np.array([oracle.grad_same_probe(p.x, p.y, oracle.rademacher_probes(seed, S, p.n), p.radius,
                                            p.bump_width, p.centers, p.weights, p.noise_var)[0]
                     for seed in range(reps)])
    se = vals.std(axis=0) / np.sqrt(reps)
    assert np.all(np.abs(vals.mean(axis=0) - ge) <= 4.5 * se + 1e-9 * np.abs(ge).max())
    # the data-fit half is deterministic
    _, sp = oracle.grad_same_probe(p.x, p.y, oracle.rademacher_probes(0, S, p.n), p.radius,
                                   p.bump_width, p.centers, p.weights, p.noise_var)
    np.testing.assert_allclose(sp["fit"], parts["fit"], rtol=1e-12)


def test_lml_same_probe_diagonal_case_is_exact():
    """Diagonal K (radius far below the point spacing): Khat = I, so the probe
    log-determinant is ln|K| for any probes and the same-probe LML equals the Gaussian
    log density, here taken from scipy's multivariate normal (an independent library
    routine), for the diagonal and the block preconditioner alike."""
    from scipy.stats import multivariate_normal
    p = _problem(n=120, r=1e-6)
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    ref = multivariate_normal(mean=np.zeros(p.n), cov=K).logpdf(p.y)
    for seed, S in ((1, 1), (7, 5)):
        Z = oracle.rademacher_probes(seed, S, p.n)
        for blocks in (None, oracle.block_partition(np.arange(p.n), 16)):
            v, parts = oracle.lml_same_probe(K, p.y, Z, blocks)
            assert v == pytest.approx(ref, rel=1e-12, abs=1e-9)
            assert parts["gamma"] == pytest.approx(parts["logdet"], rel=1e-12)


def test_lml_same_probe_one_block_is_exact():
    """With one block holding every point, M = K and Khat = I: every probe set gives
    Gamma = ln|K| and the same-probe LML is the exact Gaussian log density of a
    correlated K (scipy's multivariate normal as the independent value)."""
    from scipy.stats import multivariate_normal
    p = _problem(n=90, r=0.3)
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    assert np.count_nonzero(K - np.diag(np.diag(K))) > 10 * p.n
    ref = multivariate_normal(mean=np.zeros(p.n), cov=K).logpdf(p.y)
    one = oracle.block_partition(np.arange(p.n), p.n)
    for seed in (0, 3):
        v, parts = oracle.lml_same_probe(K, p.y, oracle.rademacher_probes(seed, 4, p.n), one)
        assert v == pytest.approx(ref, rel=1e-11)


def test_lml_same_probe_unbiased():
    """Over independent probe sets, the same-probe LML (Jacobi preconditioner) scatters
    around the exact LML with standard deviation sd(Gamma)/2."""
    p = _problem(n=200)
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    exact = oracle.lml_dense(K, p.y).lml
    D = np.diag(K)
    lam, V = np.linalg.eigh(K / np.sqrt(np.outer(D, D)))
    A = (V * np.log(lam)) @ V.T
    S, reps = 8, 150
    sd = 0.5 * np.sqrt(oracle.hutchinson_variance(A, S))
    vals = np.array([oracle.lml_same_probe(K, p.y, oracle.rademacher_probes(seed, S, p.n))[0]
                     for seed in range(reps)])
    assert abs(vals.mean() - exact) < 4 * sd / np.sqrt(reps)
    assert 0.7 < vals.std() / sd < 1.3
