"""Pins for the sparse oracle: identical to the dense one; PCG against Cholesky."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("dim,points", [(2, "uniform"), (3, "gmm")])
def test_csr_equals_dense(dim, points):
    p = workloads.make_random_problem(21, 900, dim, 0.08 if dim == 2 else 0.15, n_bumps=3,
                                      bump_width=0.45, points=points)
    Kd = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    Ks = oracle.covariance_csr(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    np.testing.assert_array_equal(Ks.toarray(), Kd)
    _, _, gamma = oracle.bump_values(p.x, p.centers, p.bump_width, p.weights)
    pat = oracle.pattern_bruteforce(p.x, p.radius, gamma)
    coo = Ks.tocoo()
    got = np.stack([coo.row, coo.col], 1)
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    np.testing.assert_array_equal(got, pat)


def test_rows_equal_dense():
    p = workloads.make_random_problem(22, 700, 2, 0.09, n_bumps=2, bump_width=0.5)
    Kd = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    rows = np.array([0, 5, 99, 699])
    for i, (cols, vals) in zip(rows, oracle.covariance_rows(p.x, p.radius, p.bump_width, p.centers,
                                                           p.weights, p.noise_var, rows)):
        nz = np.nonzero(Kd[i])[0]
        assert set(nz) <= set(cols)
        np.testing.assert_array_equal(vals, Kd[i, cols])


def test_pcg_matches_cholesky():
    p = workloads.make_problem("c1")
    K = oracle.covariance_csr(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    a, it, al, be = oracle.pcg_jacobi(K, p.y, tol=1e-10)
    res = oracle.lml_dense(K.toarray(), p.y)
    assert oracle.residual_rel(K, a, p.y) <= 1e-10
    np.testing.assert_allclose(a, res.a, rtol=0, atol=1e-6 * np.abs(res.a).max())
    assert len(al) == it and it > 100


@pytest.mark.parametrize("kernel", ["c2", "c6"])
def test_sparse_derivatives_equal_dense(kernel):
    p = workloads.make_random_problem(23, 500, 2, 0.1, n_bumps=3, bump_width=0.45)
    Kd, dd = oracle.dcov_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var, kernel)
    Ks, ds = oracle.dcov_csr(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var, kernel)
    np.testing.assert_allclose(Ks.toarray(), Kd, rtol=1e-14, atol=0)
    assert len(ds) == len(dd) == p.n_bumps + 2
    for a, b in zip(ds, dd):
        np.testing.assert_allclose(a.toarray(), b, rtol=1e-13, atol=1e-13 * np.abs(b).max())


@pytest.mark.parametrize("r", [0.03, 0.12])
def test_lml_components_equals_dense(r):
    """Many small components (r = 0.03 at 400 points) and one large one (0.12)."""
    p = workloads.make_random_problem(24, 400, 2, r, n_bumps=3, bump_width=0.5)
    K = oracle.covariance_csr(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    a = oracle.lml_components(K, p.y)
    b = oracle.lml_dense(K.toarray(), p.y)
    assert a.lml == pytest.approx(b.lml, rel=1e-12)
    assert a.logdet == pytest.approx(b.logdet, rel=1e-12)
    np.testing.assert_allclose(a.a, b.a, rtol=1e-10, atol=1e-12 * np.abs(b.a).max())


def test_lanczos_quadrature_closed_forms():
    """One step on a 1 x 1 system gives ln a; run to full dimension on a matrix with unit
    diagonal (so the Jacobi preconditioner is the identity), the quadrature is
    z^T ln(A) z / ||z||^2 exactly (the Krylov space is the whole space)."""
    assert oracle.lanczos_logquad([1.0 / 3.7], [0.0]) == pytest.approx(np.log(3.7), rel=1e-15)
    rng = np.random.default_rng(0)
    n = 12
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    d = np.sqrt(np.diag(A))
    A = A / np.outer(d, d)
    z = oracle.rademacher_probes(1, 1, n)[0]
    _, it, al, be = oracle.pcg_jacobi(A, z, tol=1e-14, max_iter=n)
    assert it == n
    lam, V = np.linalg.eigh(A)
    want = float(((V.T @ z) ** 2 * np.log(lam)).sum())
    assert float(z @ z) * oracle.lanczos_logquad(al, be) == pytest.approx(want, rel=1e-10)


def test_sparse_lml_and_gradient_equal_same_probe_dense():
    """The sparse path (CG solves, Lanczos quadrature, sparse contraction) reaches the
    dense same-probe LML and gradient with the diagonal preconditioner."""
    p = workloads.make_random_problem(25, 1200, 2, 0.07, n_bumps=3, bump_width=0.45)
    Z = oracle.rademacher_probes(9, 6, p.n)
    lml, grad, parts = oracle.lml_grad_sparse(p.x, p.y, p.radius, p.bump_width, p.centers, p.weights,
                                              p.noise_var, Z, tol=1e-13, probe_tol=1e-12)
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    lref, lparts = oracle.lml_same_probe(K, p.y, Z)
    gref, gparts = oracle.grad_same_probe(p.x, p.y, Z, p.radius, p.bump_width, p.centers, p.weights,
                                          p.noise_var, K=K)
    assert parts["gamma"] == pytest.approx(lparts["gamma"], rel=1e-10)
    assert lml == pytest.approx(lref, rel=1e-10)
    np.testing.assert_allclose(parts["fit"], gparts["fit"], rtol=1e-8)
    np.testing.assert_allclose(parts["tau"], gparts["tau"], rtol=1e-7, atol=1e-9 * np.abs(gparts["tau"]).max())
    np.testing.assert_allclose(grad, gref, rtol=1e-7, atol=1e-9 * np.abs(gref).max())
