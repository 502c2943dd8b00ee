"""The block-Jacobi preconditioner through the C ABI.

The handle's internal order equals the oracle's binned order bit for bit (the blocks
of M are runs of 128 (or, optionally, 64) points of it); the same-probe log-determinant, LML and gradient
with the block preconditioner match the oracle given the same blocks (1e-8 relative
log-determinant and LML, 1e-4 relative gradient) on clouds whose size is not a
multiple of 128 and on one smaller than a block; solves reach the 1e-8 residual bar in
fewer iterations than with the diagonal; a block that is not positive definite is
reported as GP2S_E_NOT_SPD, and an unknown preconditioner as GP2S_E_INVALID."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads
from gpu_util import exported_user_csr, oracle_blocks, params_of

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


CASES = {
    "u2_ragged": lambda: workloads.make_random_problem(61, 2037, 2, 0.05, n_bumps=3, bump_width=0.5),
    "g3": lambda: workloads.make_random_problem(62, 1500, 3, 0.12, n_bumps=3, bump_width=0.6, points="gmm"),
    "tiny": lambda: workloads.make_random_problem(63, 50, 2, 0.3, n_bumps=2, bump_width=0.8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_internal_order_is_the_bin_order(gpu, name):
    G = _G()
    prob = CASES[name]()
    m = G.gp2s_assemble(prob.x, params_of(prob), "mixed")
    perm = m.export()[3].cpu().numpy().astype(np.int64)
    assert np.array_equal(perm, oracle.bin_order(prob.x, prob.radius))
    m.free()


@pytest.mark.parametrize("precond", ["block", "block64"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_block_preconditioned_lml_and_gradient(gpu, name, precision, precond):
    G = _G()
    prob = CASES[name]()
    S = 12
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    Kd = exported_user_csr(m)[0].toarray()
    opts = G.default_opts(n_probes=S, seed=17, tol=1e-10, probe_tol=1e-10, max_iter=40000, precond=precond)
    rep, grad, a = G.gp2s_lml_grad(m, prob.y, opts)
    Z = oracle.rademacher_probes(17, S, prob.n)
    blocks = oracle_blocks(prob.x, prob.radius, precond)
    gam, terms = oracle.logdet_same_probe(Kd, Z, blocks)
    lml_ref, _ = oracle.lml_same_probe(Kd, prob.y, Z, blocks)
    gref, parts = oracle.grad_same_probe(prob.x, prob.y, Z, prob.radius, prob.bump_width, prob.centers,
                                         prob.weights, prob.noise_var, K=Kd, blocks=blocks)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(parts["fit"]) + 0.5 * np.abs(parts["tau"])))
    gerr = np.abs(grad - gref) / scale
    print(f"[{name}/{precision}] n={prob.n} logdet {rep.logdet:.10f} oracle {gam:.10f} "
          f"rel {abs(rep.logdet - gam) / abs(gam):.2e}; grad max rel {gerr.max():.2e}; "
          f"iters {rep.iters}/{rep.probe_iters}", flush=True)
    assert abs(rep.logdet - gam) <= 1e-8 * abs(gam)
    assert abs(rep.lml - lml_ref) <= 1e-8 * abs(lml_ref)
    assert np.all(gerr <= 1e-4)
    np.testing.assert_allclose(a.cpu().numpy(), np.linalg.solve(Kd, prob.y), rtol=0,
                               atol=1e-6 * np.abs(np.linalg.solve(Kd, prob.y)).max())
    # without the gradient: the same LML bit for bit
    rep2, _ = G.gp2s_lml(m, prob.y, opts)
    assert rep2.lml == rep.lml and rep2.probe_iters == rep.probe_iters
    m.free()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_block_solve_reaches_the_bar_in_fewer_iterations(gpu, precision):
    G = _G()
    prob = workloads.make_random_problem(64, 20000, 2, 0.02, n_bumps=4, bump_width=0.6)
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    K, _ = exported_user_csr(m)
    a_b, rep_b = G.gp2s_solve(m, prob.y, G.default_opts(tol=1e-8, precond="block"))
    a_j, rep_j = G.gp2s_solve(m, prob.y, G.default_opts(tol=1e-8, precond="jacobi"))
    rb = oracle.residual_rel(K, a_b.cpu().numpy(), prob.y)
    rj = oracle.residual_rel(K, a_j.cpu().numpy(), prob.y)
    print(f"[{precision}] block: {rep_b.iters} iterations, resid {rb:.2e}; jacobi: {rep_j.iters}, resid {rj:.2e}",
          flush=True)
    assert rb <= 1e-8 and rj <= 1e-8
    assert rep_b.iters < rep_j.iters
    m.free()


@pytest.mark.parametrize("precond", ["block", "jacobi"])
def test_indefinite_block_is_reported(gpu, precond):
    G = _G()
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    m = G.gp2s_matrix_import(A.indptr, A.indices, A.data)
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_solve(m, np.array([1.0, -1.0, 0.5]), G.default_opts(precond=precond))
    assert e.value.status == 5
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_lml(m, np.array([1.0, -1.0, 0.5]), G.default_opts(n_probes=2, precond=precond))
    assert e.value.status == 5


def test_unknown_preconditioner_is_rejected(gpu):
    G = _G()
    prob = CASES["tiny"]()
    m = G.gp2s_assemble(prob.x, params_of(prob), "fp64")
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_solve(m, prob.y, G.default_opts(precond=7))
    assert e.value.status == 1
    m.free()
