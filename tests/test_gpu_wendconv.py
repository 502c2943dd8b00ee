"""The non-stationary, axis-anisotropic Wendland kernel (Eq. wendconv with the
bump-driven length-scale field) through the C ABI, against oracle.wendconv.

Bars as for the stationary kernel: pattern exact except pairs with |Q - 1| <= 1e-6 or
a point within 1e-6 of a bump boundary; K entries 1e-5 relative (float32 path) or
1e-9 (float64); the handle's internal order equals the oracle's bin order on the
per-axis grid bit for bit; same-probe log-determinant and LML 1e-8 relative, gradient
1e-4 relative per component (floor 1e-6 of its two halves), with the oracle given the
same preconditioner blocks; posterior mean and variance with the tolerances of the
stationary posterior test. With equal radii and zero weights the device reproduces
its stationary path; refill equals a fresh assembly; the batched path rejects these
parameters."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import exported_user_csr, params_of, pattern_pairs
from oracle import wendconv as WC

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


def _case(name):
    if name == "ard2":
        p = workloads.make_random_problem(71, 1900, 2, 0.05, n_bumps=3, bump_width=0.6)
        return p, np.array([0.06, 0.035]), None, "c2"
    if name == "ns2":
        p = workloads.make_random_problem(72, 2300, 2, 0.05, n_bumps=4, bump_width=0.5)
        return p, np.array([0.045, 0.06]), np.array([0.8, -0.6, 0.4, -0.3]), "c2"
    if name == "ns3_iso_c6":
        p = workloads.make_random_problem(73, 1700, 3, 0.12, n_bumps=3, bump_width=0.6, points="gmm")
        return p, None, np.array([0.5, -0.7, 0.6]), "c6"
    raise KeyError(name)


CASES = ["ard2", "ns2", "ns3_iso_c6"]


def _params(G, p, radii, ls, kern):
    return G.HostParams(p.dim, p.radius, p.bump_width, p.noise_var, p.centers, p.weights, kern, radii, ls)


def _radius(p, radii):
    return p.radius if radii is None else radii


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_pattern_entries_and_order(gpu, name, precision):
    G = _G()
    p, radii, ls, kern = _case(name)
    m = G.gp2s_assemble(p.x, _params(G, p, radii, ls, kern), precision)
    Kg, raw = exported_user_csr(m)
    R = _radius(p, radii)
    Kref = WC.covariance_csr(p.x, R, p.bump_width, p.centers, p.weights, p.noise_var, ls, kern)
    # internal order = the oracle's bin order on the per-axis grid
    assert np.array_equal(raw["perm"].astype(np.int64),
                          oracle.bin_order(p.x, R, WC.ell_bound(ls)))
    # pattern: exact except pairs at the support boundary or touching a bump boundary
    got = set(map(tuple, pattern_pairs(Kg)))  # stored entries, explicit zeros included
    want = set(map(tuple, pattern_pairs(Kref)))
    diff = np.array(sorted(got ^ want), dtype=np.int64).reshape(-1, 2)
    n_bad = 0
    if diff.size:
        ell, _ = WC.length_scale(p.x, p.centers, p.bump_width, ls)
        radii_v = np.full(p.dim, p.radius) if radii is None else radii
        d = np.sum(((p.x[diff[:, 0]] - p.x[diff[:, 1]]) / radii_v) ** 2, axis=1)
        Q = d / (0.5 * (ell[diff[:, 0]] ** 2 + ell[diff[:, 1]] ** 2))
        gex = oracle.boundary_exempt_points(p.x, p.centers, p.bump_width)
        ok = (np.abs(Q - 1.0) <= 1e-6) | gex[diff[:, 0]] | gex[diff[:, 1]]
        n_bad = int((~ok).sum())
    A = Kg.tocoo()
    want_v = np.asarray(Kref.tocsr()[A.row, A.col]).ravel()
    mask = np.abs(want_v) > 1e-30
    err = np.max(np.abs(A.data[mask] - want_v[mask]) / np.abs(want_v[mask]))
    print(f"[{name}/{precision}] nnz {m.nnz} (oracle {Kref.nnz}), {len(diff)} pattern differences, "
          f"max rel entry error {err:.2e}", flush=True)
    assert n_bad == 0
    assert err <= (1e-5 if precision == "mixed" else 1e-9)
    m.free()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_same_probe_lml_and_gradient(gpu, name, precision):
    G = _G()
    p, radii, ls, kern = _case(name)
    hp = _params(G, p, radii, ls, kern)
    m = G.gp2s_assemble(p.x, hp, precision)
    Kd = exported_user_csr(m)[0].toarray()
    S = 12
    opts = G.default_opts(n_probes=S, seed=23, tol=1e-10, probe_tol=1e-10, max_iter=40000)
    rep, grad, a = G.gp2s_lml_grad(m, p.y, opts)
    assert len(grad) == hp.n_grad()
    R = _radius(p, radii)
    Z = oracle.rademacher_probes(23, S, p.n)
    blocks = oracle.block_partition(oracle.bin_order(p.x, R, WC.ell_bound(ls)), oracle.BLOCK)
    gam, _ = oracle.logdet_same_probe(Kd, Z, blocks)
    lml_ref, _ = oracle.lml_same_probe(Kd, p.y, Z, blocks)
    dc = WC.dcov_dense(p.x, R, p.bump_width, p.centers, p.weights, p.noise_var, ls, kern)
    gref, parts = oracle.grad_same_probe(p.x, p.y, Z, R, p.bump_width, p.centers, p.weights, p.noise_var,
                                         K=Kd, blocks=blocks, dcov=dc)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(parts["fit"]) + 0.5 * np.abs(parts["tau"])))
    gerr = np.abs(grad - gref) / scale
    print(f"[{name}/{precision}] logdet rel {abs(rep.logdet - gam) / abs(gam):.2e}, grad max rel {gerr.max():.2e}, "
          f"iters {rep.iters}/{rep.probe_iters}", flush=True)
    assert abs(rep.logdet - gam) <= 1e-8 * abs(gam)
    assert abs(rep.lml - lml_ref) <= 1e-8 * abs(lml_ref)
    assert np.all(gerr <= 1e-4), (grad, gref)
    m.free()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_posterior(gpu, precision):
    G = _G()
    p, radii, ls, kern = _case("ns2")
    m = G.gp2s_assemble(p.x, _params(G, p, radii, ls, kern), precision)
    Kd = exported_user_csr(m)[0].toarray()
    a, _ = G.gp2s_solve(m, p.y, G.default_opts(tol=1e-12, max_iter=100000))
    rng = np.random.default_rng(4)
    lo, hi = p.x.min(0), p.x.max(0)
    xt = workloads.f32(np.vstack([lo + (hi - lo) * rng.random((90, 2)), p.x[:10]]))
    mean, var, _ = G.gp2s_predict(m, xt, a, G.default_opts(tol=1e-10, max_iter=100000))
    Ks, gs = WC.cross_covariance(xt, p.x, radii, p.bump_width, p.centers, p.weights, ls, kern)
    aref = np.linalg.solve(Kd, p.y)
    mref = Ks @ aref
    vref = gs ** 2 - np.einsum("tj,tj->t", Ks, np.linalg.solve(Kd, Ks.T).T)
    tol_m, tol_v = (1e-5, 2e-5) if precision == "mixed" else (1e-9, 1e-9)
    assert np.all(np.abs(mean.cpu().numpy() - mref) <= tol_m * (np.abs(Ks) @ np.abs(aref)) + 1e-14)
    assert np.all(np.abs(var.cpu().numpy() - vref) <= tol_v * gs ** 2 + 1e-14)
    m.free()


def test_stationary_limit_matches_the_stationary_path(gpu):
    G = _G()
    p = workloads.make_random_problem(74, 1500, 2, 0.06, n_bumps=3, bump_width=0.5)
    opts = G.default_opts(n_probes=8, seed=5, tol=1e-11, probe_tol=1e-10)
    m0 = G.gp2s_assemble(p.x, params_of(p), "fp64")
    m1 = G.gp2s_assemble(p.x, G.HostParams(p.dim, p.radius, p.bump_width, p.noise_var, p.centers, p.weights, 0,
                                           np.array([p.radius, p.radius]), np.zeros(3)), "fp64")
    assert m0.nnz == m1.nnz
    K0, K1 = exported_user_csr(m0)[0], exported_user_csr(m1)[0]
    assert abs(K0 - K1).max() <= 1e-14 * abs(K0).max()
    r0, g0, _ = G.gp2s_lml_grad(m0, p.y, opts)
    r1, g1, _ = G.gp2s_lml_grad(m1, p.y, opts)
    assert abs(r1.lml - r0.lml) <= 1e-10 * abs(r0.lml)
    # (r_1, r_2, a, c, sigma^2): the axis radii sum to the isotropic radius component
    assert len(g1) == 2 + 3 + 3 + 1
    np.testing.assert_allclose(g1[0] + g1[1], g0[0], rtol=1e-7)
    np.testing.assert_allclose(g1[2:5], g0[1:4], rtol=1e-7)
    np.testing.assert_allclose(g1[-1], g0[-1], rtol=1e-7)
    m0.free()
    m1.free()


def test_refill_and_batch_rejection(gpu):
    G = _G()
    p, radii, ls, kern = _case("ns2")
    hp = _params(G, p, radii, ls, kern)
    m = G.gp2s_assemble(p.x, hp, "mixed")
    hp2 = _params(G, p, radii, ls, kern)
    hp2.weights = np.asarray(p.weights) * 1.2
    hp2.noise_var = p.noise_var * 2
    m.refill(hp2)
    fresh = G.gp2s_assemble(p.x, hp2, "mixed")
    ra, rb = exported_user_csr(m)[1], exported_user_csr(fresh)[1]
    for k in ("rp", "col", "val", "perm"):
        assert np.array_equal(ra[k], rb[k]), k
    bad = _params(G, p, radii, ls * 1.5, kern)
    with pytest.raises(G.GP2SError) as e:
        m.refill(bad)
    assert e.value.status == 1
    with pytest.raises(G.GP2SError) as e:
        G.Batch([p.x], [hp], "fp64", G.default_opts(n_probes=4))
    assert e.value.status == 1
    m.free()
    fresh.free()
