"""Pins of the block Metropolis-Hastings oracle against facts any correct sampler
satisfies: it samples a known target (a product of independent normals, flat prior on
wide bounds) with the right means and variances; a constant log-likelihood accepts
every in-bounds move and no out-of-bounds one; a rejected move leaves the state
unchanged; blocks move only their own components. Planted mistakes fail one of them."""
import numpy as np
import pytest

import oracle
import workloads


def _gauss(mu, sd):
    mu, sd = np.asarray(mu), np.asarray(sd)
    return lambda th: float(-0.5 * np.sum(((th - mu) / sd) ** 2))


def test_samples_a_known_target():
    mu, sd = np.array([1.0, -2.0, 0.5]), np.array([0.5, 1.0, 0.2])
    blocks = [[0], [1, 2]]
    draws = workloads.mcmc_draws(7, 40000, [len(b) for b in blocks])
    chain, lls, acc, _ = oracle.block_mh(mu + 1.0, blocks, 1.2 * sd, mu - 50, mu + 50, draws, _gauss(mu, sd))
    c = np.array(chain[2000:])
    assert np.allclose(c.mean(0), mu, atol=0.06 * sd.max() * 3)
    assert np.allclose(c.std(0), sd, rtol=0.06)
    assert 0.2 < np.mean(acc) < 0.9


def test_constant_loglik_and_bounds():
    blocks = [[0], [1]]
    draws = workloads.mcmc_draws(3, 300, [1, 1])
    chain, _, acc, margins = oracle.block_mh([0.5, 0.5], blocks, [0.3, 0.3], [0, 0], [1, 1], draws, lambda th: 0.0)
    c = np.array(chain)
    assert np.all((c > 0) & (c < 1))
    k = 0
    for it, sweep in enumerate(draws):
        for b, (eps, u) in enumerate(sweep):
            inside = margins[k] is not None
            assert acc[k] == inside  # log u < 0 always: every in-bounds move is accepted
            k += 1


def test_rejection_keeps_state_and_blocks_are_separate():
    blocks = [[0], [1]]
    draws = workloads.mcmc_draws(5, 200, [1, 1])
    chain, _, acc, _ = oracle.block_mh([0.0, 0.0], blocks, [1.0, 1.0], [-9, -9], [9, 9], draws,
                                       _gauss([0.0, 0.0], [0.3, 0.3]))
    for it in range(len(draws)):
        a0, a1 = acc[2 * it], acc[2 * it + 1]
        prev, cur = chain[it], chain[it + 1]
        if not a0 and not a1:
            assert np.array_equal(prev, cur)
        if a0 and not a1:
            assert cur[1] == prev[1]


def _fails(fn):
    with pytest.raises(AssertionError):
        fn()


def test_planted_mistakes_fail(monkeypatch):
    import oracle.mcmc as M
    monkeypatch.setattr(M, "_margin", lambda llp, ll, u: 2 * (llp - ll) - np.log(u))  # tempered target
    _fails(test_samples_a_known_target)
    monkeypatch.setattr(M, "_margin", lambda llp, ll, u: (llp - ll) - u)  # log dropped
    _fails(test_samples_a_known_target)
    monkeypatch.setattr(M, "_margin", lambda llp, ll, u: (ll - llp) - np.log(u))  # sign flipped
    _fails(test_samples_a_known_target)
