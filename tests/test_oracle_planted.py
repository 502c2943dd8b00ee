"""The pins must catch plausible mistakes: each case plants one in the oracle (CPU
only, via monkeypatch) and checks that a pin test then fails."""
import numpy as np
import pytest

import oracle
import oracle.dense
import oracle.estimators
import oracle.kernel
import oracle.probes
import test_oracle_dense as TD
import test_oracle_estimators as TE
import test_oracle_kernel as TK
import test_oracle_sparse as TS


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def _w_exp3(rho):
    rho = np.asarray(rho, dtype=np.float64)
    return np.where(rho < 1, (1 - rho) ** 3 * (4 * rho + 1), 0.0)


def _w_sign(rho):
    rho = np.asarray(rho, dtype=np.float64)
    return np.where(rho < 1, (1 - rho) ** 4 * (4 * rho - 1), 0.0)


@pytest.mark.parametrize("bad", [_w_exp3, _w_sign])
def test_wrong_wendland_caught(monkeypatch, bad):
    monkeypatch.setattr(oracle, "wendland_c2", bad)
    _fails(TK.test_wendland_c2_closed_forms)
    _fails(TK.test_wendland_integrals)


def test_wrong_radius_derivative_caught(monkeypatch):
    def bad(rho, r):  # dropped one factor of rho
        rho = np.asarray(rho, dtype=np.float64)
        return np.where(rho < 1, 20 * rho * (1 - rho) ** 3 / r, 0.0)
    monkeypatch.setattr(oracle, "wendland_c2_dr", bad)
    _fails(TK.test_wendland_radius_derivative_closed_form_and_fd)
    monkeypatch.setattr(oracle.kernel, "wendland_c2_dr", bad)  # reached through oracle.kernel.wendland_dr
    _fails(TD.test_gradient_matches_central_differences, 2, "uniform", "c2")


def test_wrong_bump_caught(monkeypatch):
    orig = oracle.kernel.bump_values

    def bad(x, centers, bump_width, weights, chunk=1 << 16):  # width instead of width^2
        return orig(x, centers, np.sqrt(bump_width), weights, chunk)
    monkeypatch.setattr(oracle, "bump_values", bad)
    _fails(TK.test_bump_closed_forms)


def test_wrong_mask_product_caught(monkeypatch):
    orig = oracle.kernel.bump_values

    def bad(x, centers, bump_width, weights, chunk=1 << 16):  # g squared by mistake
        g, b, gamma = orig(x, centers, bump_width, weights, chunk)
        return g * g, b, gamma
    monkeypatch.setattr(oracle.dense, "bump_values", bad)
    _fails(TD.test_two_point_closed_form)


def test_dropped_constant_caught(monkeypatch):
    orig = oracle.dense.lml_dense

    def bad(K, y):
        r = orig(K, y)
        return oracle.LMLResult(r.lml + 0.5 * len(y) * np.log(2 * np.pi), r.logdet, r.yTa, r.a)
    monkeypatch.setattr(oracle, "lml_dense", bad)
    _fails(TD.test_lml_matches_library_gaussian_density)


def test_wrong_trace_term_caught(monkeypatch):
    orig = oracle.dense.grad_exact

    def bad(*args):  # trace term with the wrong sign
        g, parts = orig(*args)
        return parts["fit"] + parts["trace"], parts
    monkeypatch.setattr(oracle, "grad_exact", bad)
    _fails(TD.test_diagonal_case_closed_forms)


def test_wrong_splitmix_caught(monkeypatch):
    def bad(seed, k):
        k = np.asarray(k, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(seed) + k * oracle.probes._GAMMA   # off-by-one counter
            z = (z ^ (z >> np.uint64(30))) * oracle.probes._M1
            z = (z ^ (z >> np.uint64(27))) * oracle.probes._M2
            return z ^ (z >> np.uint64(31))
    monkeypatch.setattr(oracle, "splitmix64", bad)
    _fails(TE.test_splitmix64_published_outputs)


def test_wrong_same_probe_lml_caught(monkeypatch):
    orig = oracle.estimators.lml_same_probe

    def bad_sign(K, y, Z, blocks=None):  # +1/2 Gamma instead of -1/2 Gamma
        v, parts = orig(K, y, Z, blocks)
        return v + parts["gamma"], parts

    def bad_const(K, y, Z, blocks=None):  # dropped -N/2 ln(2 pi)
        v, parts = orig(K, y, Z, blocks)
        return v + 0.5 * len(y) * np.log(2 * np.pi), parts

    def bad_fit(K, y, Z, blocks=None):  # y^T a without the factor 1/2
        v, parts = orig(K, y, Z, blocks)
        return v - 0.5 * parts["yTa"], parts

    for bad in (bad_sign, bad_const, bad_fit):
        monkeypatch.setattr(oracle, "lml_same_probe", bad)
        _fails(TE.test_lml_same_probe_diagonal_case_is_exact)
        _fails(TE.test_lml_same_probe_one_block_is_exact)


def test_wrong_lanczos_offdiagonal_caught(monkeypatch):
    import scipy.linalg

    def bad(alphas, betas):  # beta_j / alpha_j instead of sqrt(beta_j) / alpha_j
        al = np.asarray(alphas, dtype=np.float64)
        be = np.asarray(betas, dtype=np.float64)
        m = al.shape[0]
        d = 1.0 / al
        d[1:] += be[:m - 1] / al[:m - 1]
        theta, V = scipy.linalg.eigh_tridiagonal(d, be[:m - 1] / al[:m - 1])
        return float(np.sum(V[0] ** 2 * np.log(theta)))
    monkeypatch.setattr(oracle, "lanczos_logquad", bad)
    _fails(TS.test_lanczos_quadrature_closed_forms)
