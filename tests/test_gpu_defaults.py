"""Parity at the solver settings the benchmark times, which are the library defaults:
the y solve to ||y - K a|| <= 1e-8 ||y||, probe columns to a relative CG residual of
1e-5, S = 64 Rademacher probes, block-Jacobi preconditioner. Bars: the residual 1e-8
(recomputed on the CPU from the exported CSR), the same-probe log-determinant and LML
1e-8 relative, the same-probe gradient 1e-4 relative per component (floor 1e-6 of the
magnitude of its two halves), against the oracle on the same probes, the same stored
matrix and the same preconditioner blocks (its own binned order).

Also: the gradient on a 5 000-point subsample of the clustered 3-D workload against
central differences of the exact LML, within 4 Hutchinson standard deviations of the
block-preconditioned trace estimate (the check config 3 names); support flags that
stay correct for bump amplitudes of either sign; the autograd function with
hyperparameters resident on the GPU.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from gpu_util import compare_patterns, exported_user_csr, oracle_blocks, params_of, pattern_pairs, rel_entry_errors

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


CASES = {
    "c1": lambda: workloads.make_problem("c1"),
    "c2_sub5000": lambda: workloads.make_problem("c2").subsample(5000, seed=1),
}


@pytest.mark.parametrize("precond", ["block", "block64"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_lml_grad_at_default_settings(gpu, name, precision, precond):
    """The library defaults (block preconditioner over 128-point runs), and the same with
    the 64-point blocks the 10 M-point measurement uses."""
    G = _G()
    prob = CASES[name]()
    opts = G.default_opts(seed=11)
    assert (opts.n_probes, opts.tol, opts.probe_tol, opts.precond) == (64, 1e-8, 1e-5, 1)
    if precond == "block64":
        opts = G.default_opts(seed=11, precond=precond)
    print(f"[{name}/{precision}] n={prob.n} defaults S=64 tol=1e-8 probe_tol=1e-5 {precond}", flush=True)
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    rep, grad, a = G.gp2s_lml_grad(m, prob.y, opts)  # GP2S_E_NOCONV would raise here
    Kg, _ = exported_user_csr(m)
    res = oracle.residual_rel(Kg, a.cpu().numpy(), prob.y)
    Kd = Kg.toarray()
    Z = oracle.rademacher_probes(11, 64, prob.n)
    blocks = oracle_blocks(prob.x, prob.radius, precond)
    lml_ref, parts = oracle.lml_same_probe(Kd, prob.y, Z, blocks)
    rel_ld = abs(rep.logdet - parts["gamma"]) / abs(parts["gamma"])
    rel_lml = abs(rep.lml - lml_ref) / abs(lml_ref)
    gref, gparts = oracle.grad_same_probe(prob.x, prob.y, Z, prob.radius, prob.bump_width, prob.centers,
                                          prob.weights, prob.noise_var, K=Kd, blocks=blocks)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(gparts["fit"]) + 0.5 * np.abs(gparts["tau"])))
    err = np.abs(grad - gref) / scale
    print(f"[{name}/{precision}] iters {rep.iters}/{rep.probe_iters} resid {res:.2e} logdet rel {rel_ld:.2e} "
          f"lml rel {rel_lml:.2e} grad max rel {err.max():.2e}", flush=True)
    assert res <= 1e-8
    assert rel_ld <= 1e-8
    assert rel_lml <= 1e-8
    assert np.all(err <= 1e-4)


def _components_inverse(K):
    """K^-1 of a sparse SPD K as a sparse matrix: K is block diagonal over the connected
    components of its pattern, so is its inverse."""
    from scipy.sparse.csgraph import connected_components
    K = sp.csr_matrix(K)
    ncomp, lab = connected_components(K, directed=False)
    order = np.argsort(lab, kind="stable")
    bounds = np.searchsorted(lab[order], np.arange(ncomp + 1))
    rows, cols, vals = [], [], []
    for c in range(ncomp):
        idx = order[bounds[c]:bounds[c + 1]]
        inv = np.linalg.inv(K[idx][:, idx].toarray())
        rows.append(np.repeat(idx, len(idx)))
        cols.append(np.tile(idx, len(idx)))
        vals.append(inv.reshape(-1))
    n = K.shape[0]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def test_c3_subsample_gradient_vs_finite_differences(gpu):
    """Config 3's check: 5 000 points of the clustered 3-D workload (its r, 16 bumps),
    32 probes, library defaults otherwise, mixed precision. Every gradient component is
    within 4 sigma_Hutch of the central difference of the exact LML, sigma_Hutch from the
    Rademacher variance 2(||A_s||_F^2 - sum A_ii^2)/S of A = L^T K^-1 dK L^-T with the
    block preconditioner M = L L^T (the trace half enters the gradient with weight 1/2).
    The exact LML of the oracle's sparse K is summed over the connected components of
    its pattern (each a dense Cholesky)."""
    G = _G()
    prob = workloads.make_problem("c3").subsample(5000, seed=0)
    S = 32
    opts = G.default_opts(n_probes=S, seed=5)
    print(f"[c3_sub5000] n={prob.n} r={prob.radius:.5f} P={prob.n_bumps} S={S}", flush=True)
    m = G.gp2s_assemble(prob.x, params_of(prob), "mixed")
    rep, grad, _ = G.gp2s_lml_grad(m, prob.y, opts)
    theta = np.concatenate([[prob.radius], prob.weights, [prob.noise_var]])

    def lml_at(th):
        K = oracle.covariance_csr(prob.x, th[0], prob.bump_width, prob.centers, th[1:-1], th[-1])
        return oracle.lml_components(K, prob.y)

    fd = np.zeros_like(theta)
    fd_fit = np.zeros_like(theta)
    for k in range(len(theta)):
        h = 1e-5 * abs(theta[k])
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        lp, lm = lml_at(tp), lml_at(tm)
        fd[k] = (lp.lml - lm.lml) / (2 * h)
        fd_fit[k] = -0.5 * (lp.yTa - lm.yTa) / (2 * h)
    K, dKs = oracle.dcov_csr(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights, prob.noise_var)
    Kinv = _components_inverse(K)
    L, Linv, _ = oracle.block_factor(K.toarray(), oracle_blocks(prob.x, prob.radius))
    Ls, Linvs = sp.csr_matrix(L), sp.csr_matrix(Linv)
    sd = np.zeros_like(theta)
    for k, dK in enumerate(dKs):
        A = (Ls.T @ (Kinv @ (dK @ Linvs.T))).tocsr()
        As = 0.5 * (A + A.T)
        var = 2.0 * (As.multiply(As).sum() - np.sum(As.diagonal() ** 2)) / S
        sd[k] = 0.5 * np.sqrt(var)
    dev = np.abs(grad - fd)
    print(f"[c3_sub5000] |grad - fd| / sigma: {np.round(dev / np.maximum(sd, 1e-300), 2)}", flush=True)
    assert np.all(dev <= 4 * sd + 1e-6 * np.abs(fd))
    # the data-fit half 1/2 a^T dK a (oracle, exact a) against the central difference of
    # -1/2 y^T K^-1 y: deterministic, to 1e-6
    res = oracle.lml_components(K, prob.y)
    fit = np.array([0.5 * res.a @ (dK @ res.a) for dK in dKs])
    np.testing.assert_allclose(fit, fd_fit, rtol=1e-6, atol=1e-6 * np.abs(fd_fit).max())


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_amplitudes_of_either_sign(gpu, precision):
    """A negative bump amplitude makes g negative over part of the cloud; the support
    flag is geometric, so the pattern and the values still match the oracle, and a
    refill from positive amplitudes gives bitwise the same handle."""
    G = _G()
    prob = workloads.make_random_problem(41, 1500, 2, 0.07, n_bumps=4, bump_width=0.5)
    w = np.array([1.0, -1.5, 0.7, 0.5])
    g, _, gamma = oracle.bump_values(prob.x, prob.centers, prob.bump_width, w)
    assert np.sum(gamma & (g < 0)) > 50 and np.sum(gamma & (g > 0)) > 50
    pneg = G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, w)
    Kref = oracle.covariance_csr(prob.x, prob.radius, prob.bump_width, prob.centers, w, prob.noise_var)
    ex_pts = oracle.boundary_exempt_points(prob.x, prob.centers, prob.bump_width)
    m = G.gp2s_assemble(prob.x, pneg, precision)
    Kg, raw = exported_user_csr(m)
    nmis, nex = compare_patterns(pattern_pairs(Kg), pattern_pairs(Kref), prob.x, prob, ex_pts)
    err, _ = rel_entry_errors(Kg, Kref)
    print(f"[neg/{precision}] nnz={m.nnz} mismatches={nmis} exempt={nex} max rel K error {err:.2e}", flush=True)
    assert nmis == 0
    assert err <= (1e-5 if precision == "mixed" else 1e-9)
    m2 = G.gp2s_assemble(prob.x, params_of(prob), precision)
    m2.refill(pneg)
    _, raw2 = exported_user_csr(m2)
    for k in ("rp", "col", "val", "perm"):
        assert np.array_equal(raw[k], raw2[k]), k
    rep, _, _ = G.gp2s_lml_grad(m, prob.y, G.default_opts(n_probes=8, seed=2))
    rep2, _, _ = G.gp2s_lml_grad(m2, prob.y, G.default_opts(n_probes=8, seed=2))
    assert rep.lml == pytest.approx(rep2.lml, rel=1e-12)


def test_autograd_with_hyperparameters_on_gpu(gpu):
    """radius, weights and noise variance as CUDA tensors: backward returns gradients
    on their device and dtype, equal to gp2s_lml_grad's."""
    import torch
    G = _G()
    prob = workloads.make_random_problem(9, 500, 2, 0.09, n_bumps=3, bump_width=0.5, noise_var=1e-3)
    opts = G.default_opts(n_probes=16, seed=4, tol=1e-10, probe_tol=1e-9)
    dev = torch.device("cuda:0")
    r = torch.tensor(prob.radius, dtype=torch.float64, device=dev, requires_grad=True)
    wts = torch.tensor(prob.weights, dtype=torch.float32, device=dev, requires_grad=True)
    nv = torch.tensor(prob.noise_var, dtype=torch.float64, device=dev, requires_grad=True)
    x = torch.as_tensor(prob.x, device=dev)
    y = torch.as_tensor(prob.y, device=dev)
    val = G.lml(x, y, r, wts, nv, prob.centers, prob.bump_width, "fp64", opts)
    (2.0 * val).backward()
    assert r.grad.device == dev and wts.grad.device == dev and nv.grad.device == dev
    assert wts.grad.dtype == torch.float32 and r.grad.dtype == torch.float64
    pw = G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers,
                      wts.detach().cpu().double().numpy())
    m = G.gp2s_assemble(prob.x, pw, "fp64")
    rep, g2, _ = G.gp2s_lml_grad(m, prob.y, opts)
    got = np.concatenate([[r.grad.item()], wts.grad.double().cpu().numpy(), [nv.grad.item()]])
    np.testing.assert_allclose(got, 2.0 * g2, rtol=1e-6)
