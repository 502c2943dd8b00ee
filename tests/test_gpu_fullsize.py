"""Full-size workloads (the sizes the benchmark runs): sampled rows against the
oracle evaluated row by row, and size-independent properties."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import params_of

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


def _sampled_rows_check(prob, precision, n_rows=400, seed=0):
    G = _G()
    m = G.gp2s_assemble(prob.x, params_of(prob), precision)
    rp, col, val, perm = (t.cpu().numpy() for t in m.export())
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm), dtype=perm.dtype)
    rng = np.random.default_rng(seed)
    users = np.sort(rng.choice(prob.n, n_rows, replace=False))
    ref = oracle.covariance_rows(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights,
                                 prob.noise_var, users)
    ex_pts = oracle.boundary_exempt_points(prob.x, prob.centers, prob.bump_width)
    tol = 1e-5 if precision == "mixed" else 1e-9
    worst = 0.0
    mism = 0
    for u, (rcols, rvals) in zip(users, ref):
        p = inv[u]
        gcols_int = col[rp[p]:rp[p + 1]]
        gvals = val[rp[p]:rp[p + 1]].astype(np.float64)
        gcols = perm[gcols_int]
        got = dict(zip(gcols.tolist(), gvals.tolist()))
        want = dict(zip(rcols.tolist(), rvals.tolist()))
        for j in set(got) ^ set(want):
            pair = np.array([[u, j]])
            if not (oracle.boundary_exempt_pairs(prob.x, prob.radius, pair)[0] or ex_pts[u] or ex_pts[j]):
                mism += 1
        scale = 1e-30 * max(want[u], 1e-300)
        for j in set(got) & set(want):
            if abs(want[j]) >= scale:
                worst = max(worst, abs(got[j] - want[j]) / abs(want[j]))
    print(f"[{prob.name}/{precision}] n={m.n} nnz={m.nnz} ({m.nnz / m.n:.1f}/row) sampled rows={n_rows} "
          f"pattern mismatches={mism} max rel err={worst:.2e}", flush=True)
    assert mism == 0
    assert worst <= tol
    return m


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_full_assembly_rows_and_residual(precision):
    G = _G()
    prob = workloads.make_problem("c2")
    m = _sampled_rows_check(prob, precision)
    assert abs(m.nnz / m.n - 63.3) < 0.5
    a, rep = G.gp2s_solve(m, prob.y, G.default_opts(tol=1e-8))
    # residual recomputed on the CPU from the exported matrix
    import scipy.sparse as sp
    rp, col, val, perm = (t.cpu().numpy() for t in m.export())
    rows = perm[np.repeat(np.arange(m.n), np.diff(rp))]
    K = sp.csr_matrix((val.astype(np.float64), (rows, perm[col])), shape=(m.n, m.n))
    res = oracle.residual_rel(K, a.cpu().numpy(), prob.y)
    print(f"[c2/{precision}] iters={rep.iters} resid={res:.3e}", flush=True)
    assert res <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c3_full_assembly_rows(precision):
    prob = workloads.make_problem("c3")
    m = _sampled_rows_check(prob, precision, n_rows=300)
    assert abs(m.nnz / m.n - 100.0) < 3.0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c4_full_assembly_rows(precision):
    prob = workloads.make_problem("c4")
    m = _sampled_rows_check(prob, precision, n_rows=300)
    assert abs(m.nnz / m.n - 50.0) < 1.5
