"""Edge cases and error paths of the HIP path, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import (compare_patterns, exported_user_csr, imported_blocks, params_of, pattern_pairs,
                      rel_entry_errors)

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_point(gpu, precision):
    """n = 1: K = g^2 + sigma^2; everything in closed form."""
    G = _G()
    x = np.array([[0.3, 0.4]])
    c = np.array([[0.35, 0.45]])
    w = np.array([1.3])
    p = G.HostParams(2, 0.1, 0.5, 1e-3, c, w)
    g, b, _ = oracle.bump_values(x, c, 0.5, w)
    k = g[0] ** 2 + 1e-3
    m = G.gp2s_assemble(x, p, precision)
    assert (m.n, m.nnz) == (1, 1)
    y = np.array([0.7])
    rep, grad, a = G.gp2s_lml_grad(m, y, G.default_opts(n_probes=4))
    tol = 1e-6 if precision == "mixed" else 1e-12
    assert a.cpu().numpy()[0] == pytest.approx(0.7 / k, rel=tol)
    assert rep.logdet == pytest.approx(math.log(k), rel=tol)
    assert rep.lml == pytest.approx(-0.5 * 0.49 / k - 0.5 * math.log(k) - 0.5 * math.log(2 * math.pi), rel=tol)
    av = 0.7 / k
    dk = 2 * g[0] * b[0, 0]
    np.testing.assert_allclose(grad, [0.0, 0.5 * av * av * dk - 0.5 * dk / k, 0.5 * av * av - 0.5 / k],
                               rtol=1e-5 if precision == "mixed" else 1e-10, atol=1e-12)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_points_outside_every_bump(gpu, precision):
    """No point inside a bump: K = sigma^2 I, only diagonals are stored."""
    G = _G()
    prob = workloads.make_random_problem(3, 500, 2, 0.1, n_bumps=2, bump_width=0.6)
    p = G.HostParams(2, 0.1, 0.6, 2e-3, np.array([[5.0, 5.0], [-4.0, 3.0]]), np.array([1.0, 2.0]))
    m = G.gp2s_assemble(prob.x, p, precision)
    assert m.nnz == prob.n
    rep, grad, a = G.gp2s_lml_grad(m, prob.y, G.default_opts(n_probes=8))
    # the stored diagonal is sigma^2 rounded to the path's precision
    d = float(np.float32(2e-3)) if precision == "mixed" else 2e-3
    np.testing.assert_allclose(a.cpu().numpy(), prob.y / d, rtol=1e-12)
    # the mixed path's float32 probe directions perturb the CG steps at ~1e-8
    tol = 1e-8 if precision == "mixed" else 1e-12
    assert rep.logdet == pytest.approx(prob.n * math.log(d), rel=tol)
    assert grad[0] == 0.0 and grad[1] == 0.0 and grad[2] == 0.0
    assert grad[3] == pytest.approx(0.5 * np.sum(prob.y ** 2) / d ** 2 - 0.5 * prob.n / d, rel=100 * tol)


def test_duplicates_and_clamped_points(gpu):
    """Exact duplicates (clamped to the cube faces) stay legal: pattern, values, SPD."""
    G = _G()
    rng = np.random.default_rng(4)
    x = np.clip(rng.normal(0.5, 0.4, size=(1500, 2)), 0, 1)
    x = workloads.f32(np.concatenate([x, x[:100]]))
    prob = workloads.Problem("dup", x, np.sin(x[:, 0]), 0.06, 0.7, np.array([[0.5, 0.5]]), np.array([1.1]),
                             1e-3)
    for precision in ("fp64", "mixed"):
        m = G.gp2s_assemble(prob.x, params_of(prob), precision)
        Kg, _ = exported_user_csr(m)
        Kref = oracle.covariance_csr(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights,
                                     prob.noise_var)
        ex_pts = oracle.boundary_exempt_points(prob.x, prob.centers, prob.bump_width)
        nmis, _ = compare_patterns(pattern_pairs(Kg), pattern_pairs(Kref), prob.x, prob, ex_pts)
        assert nmis == 0
        d = abs(Kg - Kref)
        assert d.max() <= (1e-5 if precision == "mixed" else 1e-12) * abs(Kref).max()
        a, rep = G.gp2s_solve(m, prob.y)
        assert oracle.residual_rel(Kg, a.cpu().numpy(), prob.y) <= 1e-8


def test_nonfinite_inputs_rejected(gpu):
    G = _G()
    prob = workloads.make_random_problem(5, 200, 2, 0.1)
    x = prob.x.copy()
    x[17, 1] = np.nan
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_assemble(x, params_of(prob), "mixed")
    assert e.value.status == 7
    m = G.gp2s_assemble(prob.x, params_of(prob), "mixed")
    y = prob.y.copy()
    y[3] = np.inf
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_solve(m, y)
    assert e.value.status == 7


def test_max_iter_reports_noconv(gpu):
    G = _G()
    prob = workloads.make_problem("c1")
    m = G.gp2s_assemble(prob.x, params_of(prob), "fp64")
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_solve(m, prob.y, G.default_opts(max_iter=3, max_ir=0))
    assert e.value.status == 6
    a, rep = G.gp2s_solve(m, prob.y, G.default_opts(max_iter=3, max_ir=0), allow_noconv=True)
    assert rep.status == 6 and rep.iters == 3 and 0 < rep.resid < 1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_imported_oracle_matrix(gpu, precision):
    """The solver and the log-determinant on the oracle's own CSR (user order)."""
    G = _G()
    prob = workloads.make_random_problem(6, 1800, 2, 0.06, n_bumps=3, bump_width=0.5)
    K = oracle.covariance_csr(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights, prob.noise_var)
    Kt = K.astype(np.float32).astype(np.float64) if precision == "mixed" else K
    m = G.gp2s_matrix_import(K.indptr, K.indices, K.data, precision)
    X = np.random.default_rng(1).standard_normal((prob.n, 5))
    np.testing.assert_allclose(G.gp2s_spmv(m, X).cpu().numpy(), Kt @ X, rtol=1e-12, atol=1e-12)
    rep, a = G.gp2s_lml(m, prob.y, G.default_opts(n_probes=8, seed=2, tol=1e-10, probe_tol=1e-9))
    Z = oracle.rademacher_probes(2, 8, prob.n)
    gam, _ = oracle.logdet_same_probe(Kt.toarray(), Z, imported_blocks(prob.n))
    assert abs(rep.logdet - gam) <= 1e-8 * abs(gam)
    assert oracle.residual_rel(Kt, a.cpu().numpy(), prob.y) <= 1e-10
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_lml_grad(m, prob.y)
    assert e.value.status == 1


def test_import_rejects_bad_csr(gpu):
    G = _G()
    rp = np.array([0, 1, 2, 3])
    with pytest.raises(G.GP2SError) as e:  # row 1 lacks its diagonal
        G.gp2s_matrix_import(rp, np.array([0, 0, 2]), np.array([1.0, 0.5, 1.0]))
    assert e.value.status == 1
    with pytest.raises(G.GP2SError) as e:  # column out of range
        G.gp2s_matrix_import(rp, np.array([0, 1, 7]), np.array([1.0, 1.0, 1.0]))
    assert e.value.status == 1


def test_indefinite_matrix_reports_not_spd(gpu):
    """A symmetric indefinite matrix: CG meets p^T K p <= 0 (or a non-positive diagonal)."""
    G = _G()
    import scipy.sparse as sp
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]]))
    m = G.gp2s_matrix_import(A.indptr, A.indices, A.data)
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_solve(m, np.array([1.0, -1.0, 0.5]))
    assert e.value.status == 5
    B = sp.csr_matrix(np.array([[-1.0, 0.0], [0.0, 1.0]]))
    m = G.gp2s_matrix_import(B.indptr, B.indices, B.data)
    with pytest.raises(G.GP2SError) as e:
        G.gp2s_solve(m, np.array([1.0, 1.0]))
    assert e.value.status == 5


def test_autograd_function(gpu):
    """GP2SLML: forward value and backward gradients equal gp2s_lml_grad's up to rounding
    order (each handle tunes its own block-product variant by timing, and the variants
    sum a row in different orders); the gradient agrees with the exact dense LML's
    within the Hutchinson standard deviation."""
    import torch
    G = _G()
    prob = workloads.make_random_problem(8, 600, 2, 0.09, n_bumps=3, bump_width=0.5, noise_var=1e-3)
    S = 64
    opts = G.default_opts(n_probes=S, seed=11, tol=1e-10, probe_tol=1e-9)
    r = torch.tensor(prob.radius, dtype=torch.float64, requires_grad=True)
    wts = torch.tensor(prob.weights, dtype=torch.float64, requires_grad=True)
    nv = torch.tensor(prob.noise_var, dtype=torch.float64, requires_grad=True)
    x = torch.as_tensor(prob.x).cuda()
    y = torch.as_tensor(prob.y).cuda()
    val = G.lml(x, y, r, wts, nv, prob.centers, prob.bump_width, "fp64", opts)
    val.backward()
    grad = np.concatenate([[r.grad.item()], wts.grad.numpy(), [nv.grad.item()]])
    m = G.gp2s_assemble(prob.x, params_of(prob), "fp64")
    rep, g2, _ = G.gp2s_lml_grad(m, prob.y, opts)
    np.testing.assert_allclose(val.item(), rep.lml, rtol=1e-8)
    np.testing.assert_allclose(grad, g2, rtol=1e-8)
    # exact gradient and its Hutchinson spread
    ge, parts = oracle.grad_exact(prob.x, prob.y, prob.radius, prob.bump_width, prob.centers, prob.weights,
                                  prob.noise_var)
    K, dKs = oracle.dcov_dense(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights, prob.noise_var)
    D = np.diag(K)
    Kinv = np.linalg.inv(K)
    for k, dK in enumerate(dKs):
        A = np.sqrt(D)[:, None] * (Kinv @ dK) / np.sqrt(D)[None, :]
        A = 0.5 * (A + A.T)
        sd = 0.5 * math.sqrt(oracle.hutchinson_variance(A, S))
        assert abs(grad[k] - ge[k]) <= 4 * sd + 1e-7 * abs(ge[k]), (k, grad[k], ge[k], sd)


def _irregular_spd(seed, n, hubs, hub_len):
    """Symmetric, strictly diagonally dominant CSR with heavy-tailed row lengths: most
    rows hold a handful of entries, `hubs` rows about `hub_len` (rows far longer than
    one 2048-entry pass of the streaming product), and blocks of one-entry rows."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    lens = np.minimum((rng.pareto(1.3, n) * 6).astype(int), 400)
    lens[rng.choice(n, n // 5, replace=False)] = 0  # diagonal-only rows
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(0, n, rows.size)
    for h in rng.choice(n, hubs, replace=False):
        c = rng.choice(n, hub_len, replace=False)
        rows = np.concatenate([rows, np.full(hub_len, h)])
        cols = np.concatenate([cols, c])
    A = sp.csr_matrix((rng.uniform(-1, 1, rows.size), (rows, cols)), shape=(n, n))
    A = (A + A.T).tocsr()
    A.setdiag(0.0)
    A.eliminate_zeros()
    d = np.asarray(abs(A).sum(axis=1)).ravel() + 1.0
    A = (A + sp.diags(d)).tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", ["heavy_tail", "diagonal"])
def test_product_and_solve_irregular_rows(gpu, precision, shape):
    """The single-RHS product balances work by entries (blocks of rows by entry span, a
    last row running over several passes): rows of 1 to several thousand entries, and
    more rows per block than threads, against the float64 product of the stored values
    (float32-rounded in the mixed path), and a CG solve through the same product."""
    G = _G()
    import scipy.sparse as sp
    if shape == "heavy_tail":
        A = _irregular_spd(11, 9000, hubs=4, hub_len=6000)
        assert np.diff(A.indptr).max() > 2 * 2048
    else:
        A = sp.identity(5003, format="csr") * 2.0
    At = A.astype(np.float32).astype(np.float64) if precision == "mixed" else A
    m = G.gp2s_matrix_import(A.indptr, A.indices, A.data, precision)
    x = np.random.default_rng(2).standard_normal(A.shape[0])
    y = G.gp2s_spmv(m, x).cpu().numpy()
    ref = At @ x
    scale = abs(At) @ np.abs(x)
    print(f"[{shape}/{precision}] n={A.shape[0]} nnz={A.nnz} max row {np.diff(A.indptr).max()} "
          f"product err {np.max(np.abs(y - ref) / scale):.2e}", flush=True)
    assert np.all(np.abs(y - ref) <= 1e-13 * scale)
    a, rep = G.gp2s_solve(m, x, G.default_opts(tol=1e-12, max_iter=20000))
    assert oracle.residual_rel(At, a.cpu().numpy(), x) <= 1e-11
    m.free()


def test_timing_mask_records_only_selected_categories(gpu):
    """Per-kernel event timing honours the category mask: with one category selected the
    others run without event records (zero counts), and turning timing on for all
    categories records the standalone product again."""
    G = _G()
    A = _irregular_spd(5, 3000, hubs=2, hub_len=800)
    m = G.gp2s_matrix_import(A.indptr, A.indices, A.data, "fp64")
    ctx = m.ctx
    x = np.random.default_rng(4).standard_normal(A.shape[0])
    try:
        ctx.set_timing(True, only=["cg_matvec1"])
        G.gp2s_spmv(m, x)
        a, rep = G.gp2s_solve(m, x, G.default_opts(tol=1e-10))
        st = ctx.stats()
        print("[timing mask] " + " ".join(f"{k}={v[1]}" for k, v in st.items() if v[1]), flush=True)
        assert st["cg_matvec1"][1] > 0 and st["cg_matvec1"][0] > 0.0
        assert all(cnt == 0 for k, (_, cnt) in st.items() if k != "cg_matvec1")
        ctx.set_timing(True)
        G.gp2s_spmv(m, x)
        st = ctx.stats()
        assert st["spmv"][1] == 1 and st["cg_matvec1"][1] == 0
    finally:
        ctx.set_timing(False)
    assert all(cnt == 0 for _, cnt in ctx.stats().values())
    m.free()


def test_allocator_failure_reports_oom_without_leak(gpu):
    """A device allocator that fails on its k-th call: assembly or the LML+gradient
    returns GP2S_E_OOM (never a crash or another status), and once the handles and the
    context are released every allocation has been freed."""
    import torch
    G = _G()
    prob = workloads.make_random_problem(17, 900, 2, 0.08, n_bumps=3, bump_width=0.5)
    opts = G.default_opts(n_probes=8, seed=1)
    live = {}
    calls = [0, -1]  # calls so far, the call that fails

    def alloc(nbytes):
        calls[0] += 1
        if calls[0] == calls[1]:
            return None
        p = torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.current_stream())
        live[p] = nbytes
        return p

    def free(p):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    def run():
        ctx = G.Context(alloc=alloc, free=free)
        try:
            m = G.gp2s_assemble(prob.x, params_of(prob), "mixed", ctx)
            try:
                G.gp2s_lml_grad(m, prob.y, opts)
            finally:
                m.free()
        finally:
            ctx.close()

    run()
    total = calls[0]
    assert total > 5 and not live
    for k in sorted(set(np.linspace(1, total, 15).astype(int))):
        calls[0], calls[1] = 0, int(k)
        with pytest.raises(G.GP2SError) as e:
            run()
        print(f"[oom] failing allocation {k} of {total}: status {e.value.status}", flush=True)
        assert e.value.status == 3
        assert not live, f"{len(live)} allocations leaked after failing call {k}"


def _grouping_case(shape):
    """Clouds that stress the 16-row groups of the assembly: all rows in one cell with
    fewer or more candidates than a wave's 64 lanes, every row in a cell of its own, and
    groups mixing rows inside and outside the bumps (sizes not multiples of 16)."""
    rng = np.random.default_rng(17)
    if shape == "one_cell_small":
        x = 0.5 + 0.01 * rng.standard_normal((50, 2))
        return x, 0.5, np.array([[0.5, 0.5]]), np.array([1.2]), 0.8
    if shape == "one_cell_big":
        x = 0.5 + 0.01 * rng.standard_normal((301, 2))
        return x, 0.5, np.array([[0.5, 0.5]]), np.array([1.2]), 0.8
    if shape == "cell_per_row":
        x = rng.uniform(0.0, 1.0, (37, 2))
        return x, 0.004, np.array([[0.5, 0.5]]), np.array([1.0]), 2.0
    x = rng.uniform(0.0, 1.0, (203, 2))  # mixed support: the bump covers about half the points
    return x, 0.15, np.array([[0.0, 0.5]]), np.array([0.9]), 0.7


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", ["one_cell_small", "one_cell_big", "cell_per_row", "mixed_support"])
def test_assembly_row_groups(gpu, precision, shape):
    """Pattern and values against the oracle on clouds whose binned rows fill the
    assembly's 16-row groups in unusual ways."""
    G = _G()
    x, r, c, w, bw = _grouping_case(shape)
    x = workloads.f32(x)  # float32-representable, as the workloads' coordinates are
    noise = 1e-3
    p = G.HostParams(2, r, bw, noise, c, w)
    Kref = oracle.covariance_csr(x, r, bw, c, w, noise)
    m = G.gp2s_assemble(x, p, precision)
    Kg, raw = exported_user_csr(m)
    rp, col = raw["rp"], raw["col"]
    for i in range(m.n):
        cc = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cc) > 0) and i in cc
    ex_pts = oracle.boundary_exempt_points(x, c, bw)

    class _P:  # the fields compare_patterns reads
        radius = r
    nmis, nex = compare_patterns(pattern_pairs(Kg), pattern_pairs(Kref), x, _P, ex_pts)
    err, _ = rel_entry_errors(Kg, Kref)
    print(f"[{shape}/{precision}] n={m.n} nnz={m.nnz} (oracle {Kref.nnz}) mismatches={nmis} exempt={nex} "
          f"max rel entry err {err:.2e}", flush=True)
    assert nmis == 0
    assert err <= (1e-5 if precision == "mixed" else 1e-9)
    m.free()
