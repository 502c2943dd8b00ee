"""The printed Wendland member of Eq. wendland (C^6, kernel "c6") through the C ABI:
stored entries, the same-probe log-determinant and gradient, and the posterior, against
the oracle with the same kernel. Same bars as the C^2 parity tests (entries 1e-5 relative
in the mixed path, 1e-9 in float64; log-det 1e-8 relative; gradient 1e-4 relative with
the usual floor; posterior as in test_gpu_posterior)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import exported_user_csr, oracle_blocks, rel_entry_errors

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


CASES = {
    "gmm3d": lambda: workloads.make_random_problem(41, 2500, 3, 0.1, n_bumps=4, bump_width=0.5, points="gmm"),
    "ragged2d": lambda: workloads.make_random_problem(42, 1500, 2, 0.08, n_bumps=3, bump_width=0.45),
}


def _params(G, prob):
    return G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights,
                        kernel="c6")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_c6_entries_lml_grad_posterior(gpu, name, precision):
    G = _G()
    prob = CASES[name]()
    kw = dict(radius=prob.radius, bump_width=prob.bump_width, centers=prob.centers, weights=prob.weights,
              noise_var=prob.noise_var)
    m = G.gp2s_assemble(prob.x, _params(G, prob), precision)
    Kg, _ = exported_user_csr(m)
    Kref = oracle.covariance_csr(prob.x, kernel="c6", **kw)
    Kc2 = oracle.covariance_csr(prob.x, **kw)
    assert (Kref != 0).nnz <= Kg.nnz  # explicit zeros aside, the same structural pattern
    err, _ = rel_entry_errors(Kg, Kref)
    err_c2, _ = rel_entry_errors(Kg, Kc2)
    print(f"[{name}/{precision}] nnz={m.nnz} max rel entry error vs c6 {err:.2e} (vs c2 {err_c2:.2e})", flush=True)
    assert err <= (1e-5 if precision == "mixed" else 1e-9)
    assert err_c2 > 1e-2  # it is really the other member
    # same-probe log-determinant and gradient
    S = 16
    opts = G.default_opts(n_probes=S, seed=11, tol=1e-10, probe_tol=1e-10, max_iter=40000)
    rep, grad, a = G.gp2s_lml_grad(m, prob.y, opts)
    Kd = Kg.toarray()
    Z = oracle.rademacher_probes(11, S, prob.n)
    blocks = oracle_blocks(prob.x, prob.radius)
    gam, _ = oracle.logdet_same_probe(Kd, Z, blocks)
    assert abs(rep.logdet - gam) <= 1e-8 * abs(gam)
    gref, parts = oracle.grad_same_probe(prob.x, prob.y, Z, K=Kd, kernel="c6", blocks=blocks, **kw)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(parts["fit"]) + 0.5 * np.abs(parts["tau"])))
    gerr = np.abs(grad - gref) / scale
    print(f"[{name}/{precision}] logdet rel {abs(rep.logdet - gam) / abs(gam):.2e} grad max rel {gerr.max():.2e}",
          flush=True)
    assert np.all(gerr <= 1e-4)
    # posterior mean and variance at a few test points
    rng = np.random.default_rng(3)
    lo, hi = prob.x.min(0), prob.x.max(0)
    xt = workloads.f32(lo + (hi - lo) * rng.random((40, prob.dim)))
    a64, _ = G.gp2s_solve(m, prob.y, G.default_opts(tol=1e-12, max_iter=100000))
    mean, var, _ = G.gp2s_predict(m, xt, a64, G.default_opts(tol=1e-10, max_iter=100000))
    mref, vref, aref = oracle.posterior_dense(prob.x, prob.y, xt, K=Kd, kernel="c6", **kw)
    Ks, gs = oracle.cross_covariance(xt, prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights, "c6")
    tol_m, tol_v = (1e-5, 2e-5) if precision == "mixed" else (1e-9, 1e-9)
    assert np.all(np.abs(mean.cpu().numpy() - mref) <= tol_m * (np.abs(Ks) @ np.abs(aref)) + 1e-14)
    assert np.all(np.abs(var.cpu().numpy() - vref) <= tol_v * gs ** 2 + 1e-14)
    m.free()


def test_c6_batch_matches_single(gpu):
    G = _G()
    probs = [CASES["ragged2d"](), workloads.make_random_problem(43, 1800, 3, 0.11, n_bumps=2, bump_width=0.6)]
    opts = G.default_opts(n_probes=8, seed=2, tol=1e-10, probe_tol=1e-9, max_iter=30000, precond="jacobi")
    b = G.Batch([p.x for p in probs], [_params(G, p) for p in probs], "fp64", opts)
    lml, grads, _ = b.run([p.y for p in probs])
    for i, p in enumerate(probs):
        m = G.gp2s_assemble(p.x, _params(G, p), "fp64")
        rep, g1, _ = G.gp2s_lml_grad(m, p.y, opts)
        assert abs(lml[i] - rep.lml) <= 1e-9 * abs(rep.lml)
        sc = np.maximum(np.abs(g1), 1e-8 * np.abs(g1).max())
        assert np.all(np.abs(grads[i] - g1) <= 1e-6 * sc)
    b.free()
