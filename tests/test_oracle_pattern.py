"""Pins for the sparsity pattern: brute force vs k-d tree, strict boundary,
symmetry, expected density."""
import math

import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("points,dim,n,r", [("uniform", 2, 1500, 0.05), ("gmm", 2, 1500, 0.03),
                                            ("uniform", 3, 1200, 0.12), ("gmm", 3, 1200, 0.06)])
def test_bruteforce_equals_kdtree(points, dim, n, r):
    p = workloads.make_random_problem(11, n, dim, r, n_bumps=3, bump_width=0.45, points=points)
    _, _, gamma = oracle.bump_values(p.x, p.centers, p.bump_width, p.weights)
    assert (~gamma).sum() > 0 or points == "gmm"
    bf = oracle.pattern_bruteforce(p.x, r, gamma)
    kd = oracle.pattern_kdtree(p.x, r, gamma)
    np.testing.assert_array_equal(bf, kd)


def test_pattern_symmetric_and_has_diagonal():
    p = workloads.make_random_problem(5, 800, 2, 0.07, n_bumps=2, bump_width=0.4)
    _, _, gamma = oracle.bump_values(p.x, p.centers, p.bump_width, p.weights)
    pat = oracle.pattern_bruteforce(p.x, p.radius, gamma)
    s = set(map(tuple, pat))
    assert all((j, i) in s for i, j in s)
    assert all((i, i) in s for i in range(p.n))
    # uncovered points keep only their diagonal
    for i in np.nonzero(~gamma)[0][:20]:
        assert not any((i, j) in s for j in range(p.n) if j != i)


def test_strict_boundary_and_duplicates():
    r = 0.25  # exactly representable
    x = np.array([[0.5, 0.5], [0.75, 0.5], [0.5, 0.5], [0.5, 0.74999]])
    gamma = np.ones(4, dtype=bool)
    pat = set(map(tuple, oracle.pattern_bruteforce(x, r, gamma)))
    assert (0, 1) not in pat                 # distance exactly r is outside
    assert (0, 2) in pat and (2, 0) in pat   # duplicates are neighbours
    assert (0, 3) in pat                     # just inside
    kd = set(map(tuple, oracle.pattern_kdtree(x, r, gamma)))
    assert kd == pat


def test_expected_row_density_uniform():
    """Interior points of a uniform cloud: E[#neighbours incl. self] = 1 + (N-1) pi r^2."""
    n, r = 20000, 0.02
    x = workloads.uniform_points(np.random.default_rng(9), n, 2)
    gamma = np.ones(n, dtype=bool)
    pat = oracle.pattern_kdtree(x, r, gamma)
    counts = np.bincount(pat[:, 0], minlength=n)
    interior = np.all((x > r) & (x < 1 - r), axis=1)
    expect = 1 + (n - 1) * math.pi * r * r
    mean = counts[interior].mean()
    se = counts[interior].std() / math.sqrt(interior.sum())
    assert abs(mean - expect) < 4 * se + 0.05


def test_mean_row_count_matches_bruteforce():
    x = workloads.uniform_points(np.random.default_rng(2), 1000, 3)
    r = 0.1
    gamma = np.ones(1000, dtype=bool)
    pat = oracle.pattern_bruteforce(x, r, gamma)
    assert oracle.mean_row_count(x, r) == pytest.approx(len(pat) / 1000, rel=1e-12)


def test_boundary_exemptions():
    r = 0.5
    x = np.array([[0.0, 0.0], [0.5 * (1 + 2e-7), 0.0], [0.4, 0.0]])
    pairs = np.array([[0, 1], [0, 2]])
    ex = oracle.boundary_exempt_pairs(x, r, pairs)
    assert ex.tolist() == [True, False]
    pts = oracle.boundary_exempt_points(x, np.array([[0.0, 0.0]]), 0.4)
    assert pts.tolist() == [False, False, True]
