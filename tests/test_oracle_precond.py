"""Pins of the binned point order and of the block-preconditioned estimators.

The order: a hand-worked five-point example and hand-worked Z-order codes; on random
and clustered clouds, a permutation whose cell numbers never decrease, sub-cell codes
non-decreasing inside a cell, remaining ties in user order, cells of side at
least r, and every pair closer than r in the same or neighbouring cells; the batched
path's grid (refined cells, a smaller cap) keeps pairs within `refine` cells.

The estimators with a block preconditioner M = L L^T: a single block holding every
point makes Khat the identity, so Gamma equals ln|K| for any probes; averaged over
all 2^n sign vectors of a tiny problem, Gamma equals ln|K| and the same-probe gradient
equals the exact gradient for any partition (the Rademacher average of z^T A z is
tr A exactly); the factor is lower triangular in each block's own point order with
L L^T = M. Planted mistakes (the upper factor, L^-1 for L^-T, a dropped ln|M|) fail.
The Rademacher average holds for any invertible factor F with ln|M| = ln det(F)^2,
so the factor's orientation is pinned by the structure test, not by the average."""
import itertools

import numpy as np
import pytest

import oracle
import workloads


def test_bin_order_worked_example():
    # r = 0.5: bounding box (0.1, 0.05)-(0.9, 0.7), h = r (1 + 1e-6), 2 x 2 cells.
    # Cells (first coordinate fastest): p0 (1, 0) -> 1; p1 (0, 0) -> 0; p2: x offset 0.5 < h
    # -> (0, 1) -> 2; p3 (0, 1) -> 2; p4 (0, 0) -> 0.
    # Inside cell 0, sub-cell steps f = floor(frac * 1024): p1 (0, 102), p4 (614, 0); the
    # highest set bit of the Z-order code is p4's x bit 9 (code bit 18) against p1's y
    # bit 6 (code bit 13), so p1 comes first. Inside cell 2: p2 (1023, 307), p3 (0, 102):
    # p3 first. Order: [p1, p4, p0, p3, p2].
    x = np.array([[0.9, 0.1], [0.1, 0.1], [0.6, 0.7], [0.1, 0.6], [0.4, 0.05]])
    assert list(oracle.bin_order(x, 0.5)) == [1, 4, 0, 3, 2]
    lo, h, nb = oracle.grid(x, 0.5)
    assert nb == [2, 2] and np.all(h >= 0.5)
    assert list(oracle.sub_cell_codes(x, 0.5)[[1, 4]]) == [oracle.morton([[0, 102]])[0], oracle.morton([[614, 0]])[0]]


def test_morton_codes_worked():
    # x = 3 = 0b011, y = 5 = 0b101: x bits 0, 1 -> code bits 0, 2; y bits 0, 2 -> code bits 1, 5
    assert list(oracle.morton([[1, 0], [0, 1], [3, 5], [1023, 1023]])) == [1, 2, 39, (1 << 20) - 1]
    # 3-D: bit b of axis k goes to 3 b + k
    assert list(oracle.morton([[1, 0, 0], [0, 0, 1], [2, 0, 0], [0, 2, 1]])) == [1, 4, 8, 16 + 4]


@pytest.mark.parametrize("dim,kind,r", [(2, "uniform", 0.05), (3, "uniform", 0.15), (2, "gmm", 0.02),
                                        (1, "uniform", 0.01)])
def test_bin_order_properties(dim, kind, r):
    rng = np.random.default_rng(11 + dim)
    n = 1500
    x = workloads.uniform_points(rng, n, dim) if kind == "uniform" else workloads.gmm_points(rng, n, dim, 6,
                                                                                           (0.01, 0.05))
    order = oracle.bin_order(x, r)
    assert np.array_equal(np.sort(order), np.arange(n))
    c, nb = oracle.bin_coords(x, r)
    lo, h, _ = oracle.grid(x, r)
    assert np.all(h >= r)
    key = np.zeros(n, dtype=np.int64)
    for k in range(dim - 1, -1, -1):
        key = key * nb[k] + c[:, k]
    ks = key[order]
    assert np.all(np.diff(ks) >= 0)
    same = np.diff(ks) == 0
    code = oracle.sub_cell_codes(x, r)[order]
    assert np.all(np.diff(code)[same] >= 0)
    tie = same & (np.diff(code) == 0)
    assert np.all(np.diff(order)[tie] > 0)
    assert np.all(code < (1 << (10 * dim)))
    # unclamped coordinates already lie on the grid
    raw = np.floor((x - lo[None, :]) / h[None, :])
    assert np.all(raw >= 0) and np.all(raw <= np.array(nb) - 1)
    d2 = oracle.pairwise_sqdist(x, x)
    i, j = np.nonzero(d2 < r * r)
    assert np.all(np.abs(c[i] - c[j]) <= 1)


def test_block_partition_runs():
    order = np.array([5, 3, 9, 0, 1, 2, 4, 6, 7, 8])
    blocks = oracle.block_partition(order, 4)
    assert [list(b) for b in blocks] == [[5, 3, 9, 0], [1, 2, 4, 6], [7, 8]]
    assert len(oracle.block_partition(np.arange(128), 64)) == 2


def _dense_problem(n, seed=4):
    p = workloads.make_random_problem(seed, n, 2, 0.9, n_bumps=2, bump_width=1.2, noise_var=1e-2)
    K = oracle.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    return p, K


def test_block_factor_structure():
    p, K = _dense_problem(30)
    blocks = oracle.block_partition(np.random.default_rng(0).permutation(30), 8)
    L, Linv, logdet = oracle.block_factor(K, blocks)
    member = np.zeros((30, 30), dtype=bool)
    for b in blocks:
        member[np.ix_(b, b)] = True
    np.testing.assert_allclose(L @ L.T, np.where(member, K, 0.0), atol=1e-13)
    np.testing.assert_allclose(Linv @ L, np.eye(30), atol=1e-10)
    assert np.all(L[~member] == 0.0)
    for b in blocks:  # lower triangular in the order the block lists its points
        Lb = L[np.ix_(b, b)]
        assert np.all(np.triu(Lb, 1) == 0.0) and np.all(np.diag(Lb) > 0)
    ref = sum(np.linalg.slogdet(K[np.ix_(b, b)])[1] for b in blocks)
    assert logdet == pytest.approx(ref, rel=1e-13)
    # one-point blocks are the diagonal
    L1, _, ld1 = oracle.block_factor(K, oracle.jacobi_partition(30))
    np.testing.assert_allclose(L1, np.diag(np.sqrt(np.diag(K))), rtol=1e-15)
    assert ld1 == pytest.approx(np.sum(np.log(np.diag(K))), rel=1e-14)


def test_single_block_makes_gamma_exact():
    p, K = _dense_problem(60)
    Z = oracle.rademacher_probes(9, 4, p.n)
    gam, terms = oracle.logdet_same_probe(K, Z, blocks=[np.arange(p.n)])
    assert gam == pytest.approx(oracle.lml_dense(K, p.y).logdet, rel=1e-12)
    assert np.all(np.abs(terms) < 1e-8 * p.n)


def _all_signs(n):
    return np.array(list(itertools.product([1.0, -1.0], repeat=n)))


PARTITIONS = [[[0, 4], [1, 2, 6], [3, 5]], [[6, 0, 3], [5, 1], [4], [2]], [list(range(7))]]


@pytest.mark.parametrize("part", PARTITIONS)
def test_rademacher_average_is_exact(part):
    p, K = _dense_problem(7)
    blocks = [np.array(b) for b in part]
    Z = _all_signs(7)
    exact = oracle.lml_dense(K, p.y).logdet
    gam, _ = oracle.logdet_same_probe(K, Z, blocks)
    assert gam == pytest.approx(exact, rel=1e-12, abs=1e-12)
    gh, _ = oracle.grad_same_probe(p.x, p.y, Z, p.radius, p.bump_width, p.centers, p.weights, p.noise_var,
                                   blocks=blocks)
    ge, _ = oracle.grad_exact(p.x, p.y, p.radius, p.bump_width, p.centers, p.weights, p.noise_var)
    np.testing.assert_allclose(gh, ge, rtol=1e-10, atol=1e-12)
    # a few probes do not reproduce it (the pin is not vacuous)
    g4, _ = oracle.logdet_same_probe(K, Z[:3], blocks)
    if len(part) > 1:
        assert abs(g4 - exact) > 1e-8


def _fails(fn, *a):
    with pytest.raises(AssertionError):
        fn(*a)


def test_planted_mistakes_fail(monkeypatch):
    import oracle.estimators as E
    real = E.block_factor

    def transposed(K, blocks):
        L, Linv, ld = real(K, blocks)
        return L.T, Linv.T, ld  # the upper factor: still unbiased, but not M = L L^T
    monkeypatch.setattr(oracle, "block_factor", transposed)
    _fails(test_block_factor_structure)
    monkeypatch.setattr(oracle, "block_factor", real)

    def w_untransposed(K, blocks):
        L, Linv, ld = real(K, blocks)
        return L, Linv.T, ld  # w = L^-1 z instead of L^-T z; Khat = L^-T K L^-1
    monkeypatch.setattr(E, "block_factor", w_untransposed)
    _fails(test_rademacher_average_is_exact, PARTITIONS[0])

    def no_logdet(K, blocks):
        L, Linv, _ = real(K, blocks)
        return L, Linv, 0.0
    monkeypatch.setattr(E, "block_factor", no_logdet)
    _fails(test_single_block_makes_gamma_exact)


@pytest.mark.parametrize("refine", [1, 2])
def test_batched_grid_refinement_and_cap(refine):
    """The batched path's grid: cells of side r (1 + 1e-6) / refine unless widened past
    max(4 n, min_cells) cells; every pair closer than r then lies at most `refine` cells
    apart along each axis, and refine = 1 with the single-matrix cap is the plain order."""
    from scipy.spatial import cKDTree
    p = workloads.make_random_problem(41, 3000, 2, 0.03, points="gmm")
    x, r = p.x, 0.03
    lo, h, nb = oracle.grid(x, r, refine=refine, min_cells=4096)
    assert int(np.prod(nb)) <= max(4 * len(x), 4096)
    base = r * (1 + 1e-6) / refine
    assert np.all(h >= base * (1 - 1e-12))
    if int(np.prod([np.floor((x[:, k].max() - x[:, k].min()) / base) + 1 for k in range(2)])) <= max(4 * len(x), 4096):
        np.testing.assert_allclose(h, base, rtol=1e-15)  # no widening needed: side exactly r (1 + 1e-6) / refine
    c, _ = oracle.bin_coords(x, r, refine=refine, min_cells=4096)
    pairs = cKDTree(x).query_pairs(r, output_type="ndarray")
    assert np.all(np.abs(c[pairs[:, 0]] - c[pairs[:, 1]]) <= refine)
    order = oracle.bin_order(x, r, refine=refine, min_cells=4096)
    key = c[order, 1] * nb[0] + c[order, 0]
    assert np.all(np.diff(key) >= 0) and sorted(order.tolist()) == list(range(len(x)))
    if refine == 1:
        np.testing.assert_array_equal(oracle.bin_order(x, r, refine=1, min_cells=65536), oracle.bin_order(x, r))
