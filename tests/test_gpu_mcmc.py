"""Block-MCMC building blocks through the C ABI: the same-pattern refill equals a fresh
assembly bit for bit; the LML without gradient equals the LML of gp2s_lml_grad bit for
bit (the probe block's coefficients never depend on the solutions it skips); and a
sampler run takes the oracle sampler's decisions on the same draws, with the oracle's
same-probe LML as the likelihood (decisions are compared wherever the oracle's margin
exceeds 1e-6 |LML|, far above the 1e-8 relative LML bar)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import exported_user_csr, oracle_blocks, params_of

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_refill_equals_fresh_assembly(gpu, precision):
    G = _G()
    prob = workloads.make_random_problem(51, 2200, 2, 0.06, n_bumps=3, bump_width=0.5)
    p0 = params_of(prob)
    m = G.gp2s_assemble(prob.x, p0, precision)
    p1 = G.HostParams(p0.dim, p0.radius, p0.bump_width, p0.noise_var * 3, p0.centers,
                      np.asarray(p0.weights) * np.array([0.7, 1.3, 1.1]), kernel="c6")
    m.refill(p1)
    fresh = G.gp2s_assemble(prob.x, p1, precision)
    _, ra = exported_user_csr(m)
    _, rb = exported_user_csr(fresh)
    for k in ("rp", "col", "val", "perm"):
        assert np.array_equal(ra[k], rb[k]), k
    opts = G.default_opts(n_probes=8, seed=4)
    for h in (m, fresh):
        h.set_block_product(8, 0)  # one summation order on both handles (the tuner times candidates)
    r1, _ = G.gp2s_lml(m, prob.y, opts)
    r2, _ = G.gp2s_lml(fresh, prob.y, opts)
    assert r1.lml == r2.lml
    bad = G.HostParams(p0.dim, p0.radius * 1.1, p0.bump_width, p0.noise_var, p0.centers, p0.weights)
    with pytest.raises(G.GP2SError) as e:
        m.refill(bad)
    assert e.value.status == 1


def test_lml_without_gradient_is_bitwise_the_same(gpu):
    G = _G()
    prob = workloads.make_random_problem(52, 3000, 3, 0.1, n_bumps=4, bump_width=0.5, points="gmm")
    m = G.gp2s_assemble(prob.x, params_of(prob), "mixed")
    opts = G.default_opts(n_probes=16, seed=9)
    r1, _ = G.gp2s_lml(m, prob.y, opts)
    r2, _, _ = G.gp2s_lml_grad(m, prob.y, opts)
    assert r1.lml == r2.lml and r1.logdet == r2.logdet and r1.probe_iters == r2.probe_iters


def test_sampler_follows_oracle_decisions(gpu):
    G = _G()
    prob = workloads.make_random_problem(53, 700, 2, 0.12, n_bumps=2, bump_width=0.6)
    p0 = params_of(prob)
    S, seed = 8, 21
    opts = G.default_opts(n_probes=S, seed=seed, tol=1e-10, probe_tol=1e-10, max_iter=50000)
    theta0 = G.mcmc.theta_of(p0)
    steps = np.array([0.1 * theta0[0], 0.15, 0.15, 0.3 * theta0[-1]])
    bounds = (theta0 / 5, theta0 * 5)
    blocks = [[0], [1, 2], [3]]
    draws = workloads.mcmc_draws(99, 5, [len(b) for b in blocks])
    Z = oracle.rademacher_probes(seed, S, prob.n)

    def loglik(th):
        K = oracle.covariance_dense(prob.x, th[0], prob.bump_width, prob.centers, th[1:3], th[3])
        return oracle.lml_same_probe(K, prob.y, Z, oracle_blocks(prob.x, th[0]))[0]
    chain_o, lls_o, acc_o, marg_o = oracle.block_mh(theta0, blocks, steps, bounds[0], bounds[1], draws, loglik)
    mh = G.BlockMH(prob.x, prob.y, p0, "fp64", opts, blocks=blocks, steps=steps, bounds=bounds)
    res = mh.run(len(draws), draws=draws)
    mh.free()
    print(f"oracle accepted {acc_o}\ndevice accepted {res['accepted']}\nLML {lls_o[-1]:.8f} vs {res['lml'][-1]:.8f} "
          f"(evals {res['evals']}, refills {res['refills']}, assemblies {res['assemblies']})", flush=True)
    tie = 1e-6 * abs(lls_o[0])
    compared = 0
    for k, (mo, ao, ad) in enumerate(zip(marg_o, acc_o, res["accepted"])):
        if mo is not None and abs(mo) < tie:
            break  # a decision within the LML bar of the threshold: the runs may part here
        assert ao == ad, (k, mo)
        compared += 1
    else:
        np.testing.assert_allclose(res["chain"], np.array(chain_o), rtol=1e-14, atol=0)
        np.testing.assert_allclose(res["lml"], np.array(lls_o), rtol=1e-8)
    assert compared >= len(acc_o) // 2
    assert res["refills"] > 0 and res["evals"] == sum(m is not None for m in marg_o)


def test_sampler_with_the_general_kernel(gpu):
    """The same decisions as the oracle sampler for Eq. wendconv with axis radii and
    length-scale weights (theta = (r_1, r_2, a, c, sigma^2)); moves of a or sigma^2 may
    refill (when the spare handle holds the current pattern), moves of the radii or c
    assemble."""
    from oracle import wendconv as WC
    G = _G()
    prob = workloads.make_random_problem(54, 600, 2, 0.12, n_bumps=2, bump_width=0.6)
    S, seed = 8, 22
    opts = G.default_opts(n_probes=S, seed=seed, tol=1e-10, probe_tol=1e-10, max_iter=50000)
    p0 = G.HostParams(2, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights, 0,
                      np.array([0.12, 0.09]), np.array([0.3, -0.2]))
    theta0 = G.mcmc.theta_of(p0)
    assert len(theta0) == 2 + 2 + 2 + 1
    steps = np.array([0.01, 0.01, 0.15, 0.15, 0.1, 0.1, 0.3 * prob.noise_var])
    blocks = [[0, 1], [2, 3], [4, 5], [6]]
    bounds = (np.array([0.02, 0.02, 0.05, 0.05, -3, -3, 1e-6]), np.array([0.5, 0.5, 5, 5, 3, 3, 1e-2]))
    draws = workloads.mcmc_draws(98, 3, [len(b) for b in blocks])
    Z = oracle.rademacher_probes(seed, S, prob.n)

    def loglik(th):
        radii, a, c, nv = th[:2], th[2:4], th[4:6], th[6]
        K = WC.covariance_dense(prob.x, radii, prob.bump_width, prob.centers, a, nv, ls_weights=c)
        blocks_ = oracle.block_partition(oracle.bin_order(prob.x, radii, WC.ell_bound(c)), oracle.BLOCK)
        return oracle.lml_same_probe(K, prob.y, Z, blocks_)[0]
    chain_o, lls_o, acc_o, marg_o = oracle.block_mh(theta0, blocks, steps, bounds[0], bounds[1], draws, loglik)
    mh = G.BlockMH(prob.x, prob.y, p0, "fp64", opts, blocks=blocks, steps=steps, bounds=bounds)
    res = mh.run(len(draws), draws=draws)
    mh.free()
    print(f"oracle accepted {acc_o}\ndevice accepted {res['accepted']} (refills {res['refills']}, "
          f"assemblies {res['assemblies']})", flush=True)
    tie = 1e-6 * abs(lls_o[0])
    compared = 0
    for k, (mo, ao, ad) in enumerate(zip(marg_o, acc_o, res["accepted"])):
        if mo is not None and abs(mo) < tie:
            break
        assert ao == ad, (k, mo)
        compared += 1
    else:
        np.testing.assert_allclose(res["chain"], np.array(chain_o), rtol=1e-14, atol=0)
        np.testing.assert_allclose(res["lml"], np.array(lls_o), rtol=1e-8)
    assert compared >= len(acc_o) // 2
    assert res["assemblies"] + res["refills"] == res["evals"] + 1  # one handle build or refill per LML
