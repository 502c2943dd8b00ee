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
