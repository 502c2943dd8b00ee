"""The far-field bump kernel (Eq. bump_kernel, core kernel 1) through the C ABI, against
oracle.farfield.

The handle stores K_loc = W + sigma_n^2 I (checked like the stationary K: pattern exact
except pairs within 1e-6 of the support boundary, entries 1e-5 relative in float32,
1e-9 in float64); the rank-U bump term is applied as G (G^T v). Products with the full
K (gp2s_spmv) match the dense oracle to 1e-12 relative in float64 (1e-6 in float32,
relative to the row sums of |K| |X|); the same-probe log-determinant matches to 1e-8
relative, the LML to 1e-8 of the magnitude of its three terms (they can cancel), and
the gradient to 1e-4 (floor 1e-6 of its two halves), with the oracle
given the stored K_loc plus its own G G^T and the same preconditioner; the posterior
matches with the stationary posterior test's tolerances; refill equals a fresh
assembly."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import exported_user_csr, pattern_pairs
from oracle import farfield as FF

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


def _case(name):
    if name == "u2":
        p = workloads.make_random_problem(81, 1700, 2, 0.05, n_bumps=4, bump_width=0.35)
        return p, np.array([0, 1, 0, 2], dtype=np.int32), "c2"
    if name == "g3_c6":
        p = workloads.make_random_problem(82, 1400, 3, 0.12, n_bumps=3, bump_width=0.5, points="gmm")
        return p, np.array([0, 0, 1], dtype=np.int32), "c6"
    raise KeyError(name)


CASES = ["u2", "g3_c6"]


def _params(G, p, groups, kern, **kw):
    d = dict(dim=p.dim, radius=p.radius, bump_width=p.bump_width, noise_var=p.noise_var, centers=p.centers,
             weights=p.weights, kernel=kern, ff_groups=groups)
    d.update(kw)
    return G.HostParams(**d)


def _full_K(m, p, groups):
    Kl = exported_user_csr(m)[0]
    Gm, _ = FF.group_values(p.x, p.centers, p.bump_width, p.weights, groups)
    return Kl, Kl.toarray() + Gm @ Gm.T


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_local_matrix_and_full_products(gpu, name, precision):
    G = _G()
    p, groups, kern = _case(name)
    m = G.gp2s_assemble(p.x, _params(G, p, groups, kern), precision)
    Kl, Kd = _full_K(m, p, groups)
    ref = FF.local_csr(p.x, p.radius, p.noise_var, kern)
    diff = set(map(tuple, pattern_pairs(Kl))) ^ set(map(tuple, pattern_pairs(ref)))
    bad = [ij for ij in diff
           if abs(np.sum((p.x[ij[0]] - p.x[ij[1]]) ** 2) / p.radius ** 2 - 1.0) > 1e-6]
    assert not bad
    A = Kl.tocoo()
    want = np.asarray(ref.tocsr()[A.row, A.col]).ravel()
    mask = np.abs(want) > 1e-30
    err = np.max(np.abs(A.data[mask] - want[mask]) / np.abs(want[mask]))
    assert err <= (1e-5 if precision == "mixed" else 1e-9)
    X = np.random.default_rng(2).standard_normal((p.n, 5))
    Y = G.gp2s_spmv(m, X).cpu().numpy()
    Kfull = FF.covariance_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var, groups, kern)
    scale = np.abs(Kfull) @ np.abs(X)
    tol = 1e-6 if precision == "mixed" else 1e-12
    print(f"[{name}/{precision}] local nnz {m.nnz}, entry err {err:.2e}, product err "
          f"{np.max(np.abs(Y - Kfull @ X) / scale):.2e}", flush=True)
    assert np.all(np.abs(Y - Kfull @ X) <= tol * scale)
    m.free()


@pytest.mark.parametrize("precond", ["block", "jacobi"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_same_probe_lml_and_gradient(gpu, name, precision, precond):
    G = _G()
    p, groups, kern = _case(name)
    m = G.gp2s_assemble(p.x, _params(G, p, groups, kern), precision)
    _, Kd = _full_K(m, p, groups)
    S = 12
    opts = G.default_opts(n_probes=S, seed=31, tol=1e-10, probe_tol=1e-10, max_iter=40000, precond=precond)
    rep, grad, a = G.gp2s_lml_grad(m, p.y, opts)
    Z = oracle.rademacher_probes(31, S, p.n)
    blocks = None if precond == "jacobi" else oracle.block_partition(oracle.bin_order(p.x, p.radius), oracle.BLOCK)
    gam, _ = oracle.logdet_same_probe(Kd, Z, blocks)
    lml_ref, _ = oracle.lml_same_probe(Kd, p.y, Z, blocks)
    dc = FF.dcov_dense(p.x, p.radius, p.bump_width, p.centers, p.weights, p.noise_var, groups, kern)
    gref, parts = oracle.grad_same_probe(p.x, p.y, Z, p.radius, p.bump_width, p.centers, p.weights, p.noise_var,
                                         K=Kd, blocks=blocks, dcov=dc)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(parts["fit"]) + 0.5 * np.abs(parts["tau"])))
    # (an amplitude whose bump covers no point has gradient exactly 0 on both sides)
    gerr = np.where(scale > 0, np.abs(grad - gref) / np.where(scale > 0, scale, 1.0), np.abs(grad - gref))
    resid = np.linalg.norm(p.y - Kd @ a.cpu().numpy()) / np.linalg.norm(p.y)
    print(f"[{name}/{precision}/{precond}] logdet rel {abs(rep.logdet - gam) / abs(gam):.2e}, grad max rel "
          f"{gerr.max():.2e}, resid {resid:.1e}, iters {rep.iters}/{rep.probe_iters}", flush=True)
    assert abs(rep.logdet - gam) <= 1e-8 * abs(gam)
    # LML = -1/2 y^T a - 1/2 ln|K| - n/2 ln 2 pi can cancel to a small number: its bar is 1e-8 of
    # the magnitude of its terms
    assert abs(rep.lml - lml_ref) <= 1e-8 * 0.5 * (abs(rep.yTa) + abs(gam) + p.n * np.log(2 * np.pi))
    assert np.all(gerr <= 1e-4), (grad, gref)
    assert resid <= 1e-8
    m.free()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_posterior(gpu, precision):
    G = _G()
    p, groups, kern = _case("u2")
    m = G.gp2s_assemble(p.x, _params(G, p, groups, kern), precision)
    _, Kd = _full_K(m, p, groups)
    a, _ = G.gp2s_solve(m, p.y, G.default_opts(tol=1e-12, max_iter=100000))
    rng = np.random.default_rng(5)
    lo, hi = p.x.min(0), p.x.max(0)
    xt = workloads.f32(np.vstack([lo + (hi - lo) * rng.random((100, 2)), p.x[:10], hi + 0.5]))
    mean, var, _ = G.gp2s_predict(m, xt, a, G.default_opts(tol=1e-10, max_iter=100000))
    Ks, prior = FF.cross_covariance(xt, p.x, p.radius, p.bump_width, p.centers, p.weights, groups, kern)
    aref = np.linalg.solve(Kd, p.y)
    mref = Ks @ aref
    vref = prior - np.einsum("tj,tj->t", Ks, np.linalg.solve(Kd, Ks.T).T)
    tol_m, tol_v = (1e-5, 2e-5) if precision == "mixed" else (1e-9, 1e-9)
    em = np.abs(mean.cpu().numpy() - mref) / ((np.abs(Ks) @ np.abs(aref)) + 1e-300)
    ev = np.abs(var.cpu().numpy() - vref) / prior
    print(f"[{precision}] posterior mean err {em.max():.2e}, var err {ev.max():.2e}", flush=True)
    assert np.all(em <= tol_m) and np.all(ev <= tol_v)
    m.free()


def test_refill_equals_fresh_assembly(gpu):
    G = _G()
    p, groups, kern = _case("u2")
    m = G.gp2s_assemble(p.x, _params(G, p, groups, kern), "mixed")
    hp2 = _params(G, p, groups, kern, weights=np.asarray(p.weights) * 0.7, noise_var=p.noise_var * 3)
    m.refill(hp2)
    fresh = G.gp2s_assemble(p.x, hp2, "mixed")
    opts = G.default_opts(n_probes=8, seed=3)
    for h in (m, fresh):
        h.set_block_product(8, 0)
    r1, g1, _ = G.gp2s_lml_grad(m, p.y, opts)
    r2, g2, _ = G.gp2s_lml_grad(fresh, p.y, opts)
    assert r1.lml == r2.lml and np.array_equal(g1, g2)
    with pytest.raises(G.GP2SError) as e:
        m.refill(_params(G, p, np.array([0, 0, 0, 0], dtype=np.int32), kern))
    assert e.value.status == 1
    m.free()
    fresh.free()
