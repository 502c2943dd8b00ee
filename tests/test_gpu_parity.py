"""HIP path vs the float64 oracle, element by element, through the C ABI.

Tolerances (float32-assembled path unless stated): sparsity pattern exact except
pairs within 1e-6 of the support boundary; K entries 1e-5 relative (float64 path
1e-9); ||y - K a|| / ||y|| <= 1e-8 recomputed on the CPU from the exported CSR;
the same-probe log-determinant within 1e-8 relative; the same-probe gradient within
1e-4 relative per component (floor 1e-6 of the magnitude of its two halves). The
same-probe values depend on the preconditioner, so the oracle is given the same one
(the diagonal, or blocks of 64 points of its own binned order).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import (compare_patterns, exported_user_csr, oracle_blocks, params_of, pattern_pairs,
                      rel_entry_errors)

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


CASES = {
    "c1": lambda: workloads.make_problem("c1"),
    "gmm3d": lambda: workloads.make_random_problem(31, 3001, 3, 0.09, n_bumps=5, bump_width=0.45, points="gmm"),
    "ragged2d": lambda: workloads.make_random_problem(32, 1237, 2, 0.07, n_bumps=3, bump_width=0.35),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, gpu):
    prob = CASES[request.param]()
    K = oracle.covariance_csr(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights, prob.noise_var)
    _, _, gamma = oracle.bump_values(prob.x, prob.centers, prob.bump_width, prob.weights)
    ex_pts = oracle.boundary_exempt_points(prob.x, prob.centers, prob.bump_width)
    return request.param, prob, K, gamma, ex_pts


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_assembly_pattern_and_values(case, precision):
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    Kg, raw = exported_user_csr(m)
    # columns ascending within each internal row, diagonal present
    rp, col = raw["rp"], raw["col"]
    for i in range(0, m.n, max(1, m.n // 500)):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    nmis, nex = compare_patterns(pattern_pairs(Kg), pattern_pairs(Kref), prob.x, prob, ex_pts)
    print(f"[{name}/{precision}] n={m.n} nnz={m.nnz} pattern mismatches={nmis} exempt={nex}", flush=True)
    assert nmis == 0
    err, nsmall = rel_entry_errors(Kg, Kref)
    tol = 1e-5 if precision == "mixed" else 1e-9
    print(f"[{name}/{precision}] max rel K error {err:.3e} (tiny entries skipped: {nsmall})", flush=True)
    assert err <= tol
    # bitwise symmetry
    D = (Kg - Kg.T).tocoo()
    assert np.count_nonzero(D.data) == 0
    # determinism: a second assembly is bitwise identical
    m2 = G.gp2s_assemble(prob.x, params_of(prob), precision)
    K2, raw2 = exported_user_csr(m2)
    assert np.array_equal(raw["rp"], raw2["rp"]) and np.array_equal(raw["col"], raw2["col"])
    assert np.array_equal(raw["val"], raw2["val"]) and np.array_equal(raw["perm"], raw2["perm"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs", [1, 7, 8, 16, 32, 64])
def test_spmv_matches_exported_matrix(case, precision, nrhs):
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    Kg, _ = exported_user_csr(m)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((prob.n, nrhs)) if nrhs > 1 else rng.standard_normal(prob.n)
    Y = G.gp2s_spmv(m, X).cpu().numpy()
    ref = Kg @ X
    np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # and against the oracle's K (float32 storage effect bounded by 1e-5 relative per entry)
    ref2 = Kref @ X
    tol = 1e-5 if precision == "mixed" else 1e-10
    assert np.abs(Y - ref2).max() <= tol * (abs(Kref) @ np.abs(X)).max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_residual_and_solution(case, precision):
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    Kg, _ = exported_user_csr(m)
    a, rep = G.gp2s_solve(m, prob.y, G.default_opts(tol=1e-8))
    a = a.cpu().numpy()
    res_cpu = oracle.residual_rel(Kg, a, prob.y)
    res_true = oracle.residual_rel(Kref, a, prob.y)
    print(f"[{name}/{precision}] CG iters={rep.iters} ir={rep.ir_steps} resid(stored K)={res_cpu:.3e} "
          f"reported={rep.resid:.3e} resid(float64 K)={res_true:.3e}", flush=True)
    assert res_cpu <= 1e-8
    assert rep.resid == pytest.approx(res_cpu, rel=1e-3, abs=1e-12)
    ref = oracle.lml_dense(Kg.toarray(), prob.y)
    np.testing.assert_allclose(a, ref.a, rtol=0, atol=1e-5 * np.abs(ref.a).max())


@pytest.mark.parametrize("precond", ["jacobi", "block"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_lml_and_gradient_same_probe(case, precision, precond):
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    S = 16
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    Kg, _ = exported_user_csr(m)
    opts = G.default_opts(n_probes=S, seed=7, tol=1e-10, probe_tol=1e-10, max_iter=40000, precond=precond)
    rep, grad, a = G.gp2s_lml_grad(m, prob.y, opts)
    Z = oracle.rademacher_probes(7, S, prob.n)
    Kd = Kg.toarray()
    blocks = oracle_blocks(prob.x, prob.radius, precond)
    gam_ref, terms = oracle.logdet_same_probe(Kd, Z, blocks)
    rel = abs(rep.logdet - gam_ref) / abs(gam_ref)
    lml_ref, parts = oracle.lml_same_probe(Kd, prob.y, Z, blocks)
    exact = oracle.lml_dense(Kref.toarray(), prob.y)
    print(f"[{name}/{precision}/{precond}] logdet gpu={rep.logdet:.10f} oracle(same probes)={gam_ref:.10f} rel={rel:.2e} "
          f"exact={exact.logdet:.6f} stderr={rep.logdet_stderr:.3f} iters={rep.iters}/{rep.probe_iters}",
          flush=True)
    assert rel <= 1e-8
    assert abs(rep.lml - lml_ref) <= 1e-8 * abs(lml_ref)
    assert abs(rep.logdet - exact.logdet) <= 5 * rep.logdet_stderr + 1e-6 * abs(exact.logdet)
    gref, gparts = oracle.grad_same_probe(prob.x, prob.y, Z, prob.radius, prob.bump_width, prob.centers,
                                          prob.weights, prob.noise_var, K=Kd, blocks=blocks)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(gparts["fit"]) + 0.5 * np.abs(gparts["tau"])))
    err = np.abs(grad - gref) / scale
    print(f"[{name}/{precision}/{precond}] grad max rel err {err.max():.2e}\n gpu={grad}\n ref={gref}", flush=True)
    assert np.all(err <= 1e-4)
    for k in range(len(gref)):
        if gref[k] == 0.0:
            assert grad[k] == 0.0


# lane per column, column slices, LDS tiles, row groups, block split, two-pass column slices,
# 4/8/16 lanes per row
BLOCK_VARIANTS = [0, 1, 2, 3, 5, 6, 4, 8, 16]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs", [8, 16, 32, 64])
def test_block_product_variants(case, precision, nrhs):
    """Every block-product kernel gives the stored matrix's product."""
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    Kg, _ = exported_user_csr(m)
    X = np.random.default_rng(11).standard_normal((prob.n, nrhs))
    ref = Kg @ X
    for v in BLOCK_VARIANTS:
        if v > nrhs or (v == 3 and nrhs not in (32, 64)):  # row groups: 32 or 64 columns
            with pytest.raises(G.GP2SError):
                m.set_block_product(nrhs, v)
            continue
        m.set_block_product(nrhs, v)
        assert m.block_product(nrhs) == v
        Y = G.gp2s_spmv(m, X).cpu().numpy()
        np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max(), err_msg=f"variant {v}")
    with pytest.raises(G.GP2SError):
        m.set_block_product(7, 1)


@pytest.mark.parametrize("S", [16, 64])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_probe_block_variants_same_probe(case, precision, S):
    """The CG probe block (products plus per-column p^T q partials) with every kernel
    that applies to S columns reaches the same-probe log-determinant and gradient of
    the oracle."""
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    Kd = exported_user_csr(m)[0].toarray()
    opts = G.default_opts(n_probes=S, seed=3, tol=1e-10, probe_tol=1e-10, max_iter=40000)
    Z = oracle.rademacher_probes(3, S, prob.n)
    blocks = oracle_blocks(prob.x, prob.radius)  # the default preconditioner
    gam_ref, _ = oracle.logdet_same_probe(Kd, Z, blocks)
    gref, gparts = oracle.grad_same_probe(prob.x, prob.y, Z, prob.radius, prob.bump_width, prob.centers,
                                          prob.weights, prob.noise_var, K=Kd, blocks=blocks)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(gparts["fit"]) + 0.5 * np.abs(gparts["tau"])))
    for v in BLOCK_VARIANTS:
        if v == 3 and S not in (32, 64):
            continue
        m.set_block_product(S, v)
        rep, grad, _ = G.gp2s_lml_grad(m, prob.y, opts)
        rel = abs(rep.logdet - gam_ref) / abs(gam_ref)
        print(f"[{name}/{precision}] variant {v}: logdet rel {rel:.2e} probe iters {rep.probe_iters}", flush=True)
        assert rel <= 1e-8
        assert np.all(np.abs(grad - gref) <= 1e-4 * scale)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_block_split_after_refill(case, precision):
    """The block split's dense blocks follow a refill: the product after new amplitudes
    and noise equals the refilled matrix's (exported) product."""
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    m.set_block_product(64, 5)
    X = np.random.default_rng(12).standard_normal((prob.n, 64))
    Y0 = G.gp2s_spmv(m, X).cpu().numpy()
    ref0 = exported_user_csr(m)[0] @ X
    np.testing.assert_allclose(Y0, ref0, rtol=1e-12, atol=1e-12 * np.abs(ref0).max())
    p2 = G.HostParams(prob.dim, prob.radius, prob.bump_width, 2.5 * prob.noise_var, prob.centers,
                      prob.weights * np.linspace(0.7, 1.3, prob.n_bumps))
    m.refill(p2)
    Y1 = G.gp2s_spmv(m, X).cpu().numpy()
    ref1 = exported_user_csr(m)[0] @ X
    assert np.abs(ref1 - ref0).max() > 1e-3 * np.abs(ref0).max()
    np.testing.assert_allclose(Y1, ref1, rtol=1e-12, atol=1e-12 * np.abs(ref1).max())


def test_block_product_choice_remembered_per_shape(case):
    """A second handle of the same shape in the context takes the tuned block product of
    the first without timing the candidates; -1 set on a handle times them afresh."""
    G = _G()
    name, prob, Kref, gamma, ex_pts = case
    opts = G.default_opts(n_probes=16, max_iter=64, check_every=32)
    m1 = G.gp2s_assemble(prob.x, params_of(prob), "mixed")
    m2 = G.gp2s_assemble(prob.x, params_of(prob), "mixed")
    G.gp2s_lml_grad(m1, prob.y, opts, want_a=False, allow_noconv=True)
    v1 = m1.block_product(16)
    assert v1 >= 0
    assert m2.block_product(16) == -1
    G.gp2s_lml_grad(m2, prob.y, opts, want_a=False, allow_noconv=True)
    assert m2.block_product(16) == v1
    m2.set_block_product(16, -1)
    assert m2.block_product(16) == -1
    G.gp2s_lml_grad(m2, prob.y, opts, want_a=False, allow_noconv=True)
    assert m2.block_product(16) >= 0
    m1.free()
    m2.free()
