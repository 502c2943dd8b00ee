"""Batched instances: each instance of a batch equals its own single-instance run
(same probes), and the oracle on the same probes; hyperparameter changes and the
capacity limit behave as documented."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import exported_user_csr, params_of

pytestmark = pytest.mark.gpu


def _G():
    import paper_2512_06143_amd as G
    return G


def _instances():
    specs = [(900, 2, 0.07, "uniform"), (2500, 3, 0.12, "gmm"), (1300, 2, 0.05, "gmm"), (3100, 3, 0.09, "uniform"),
             (700, 2, 0.11, "uniform"), (2049, 2, 0.04, "uniform")]
    out = []
    for k, (n, d, r, pts) in enumerate(specs):
        p = workloads.make_random_problem(70 + k, n, d, r, n_bumps=2 + k % 3, bump_width=0.55, points=pts,
                                          noise_var=[1e-4, 1e-3, 3e-4][k % 3])
        out.append(p)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_single_runs_and_oracle(gpu, precision):
    G = _G()
    probs = _instances()
    S = 16
    opts = G.default_opts(n_probes=S, seed=5, tol=1e-10, probe_tol=1e-9, max_iter=30000, precond="jacobi")
    b = G.Batch([p.x for p in probs], [params_of(p) for p in probs], precision, opts)
    info = b.info()
    print(f"[batch/{precision}] {info}", flush=True)
    lml, grads, reps = b.run([p.y for p in probs])
    for i, p in enumerate(probs):
        m = G.gp2s_assemble(p.x, params_of(p), precision)
        rep, g1, _ = G.gp2s_lml_grad(m, p.y, opts)
        assert abs(lml[i] - rep.lml) <= 1e-9 * abs(rep.lml), (i, lml[i], rep.lml)
        assert abs(reps[i]["logdet"] - rep.logdet) <= 1e-9 * abs(rep.logdet)
        scale = np.maximum(np.abs(g1), 1e-8 * np.abs(g1).max())
        assert np.all(np.abs(grads[i] - g1) <= 1e-6 * scale), (i, grads[i], g1)
        assert reps[i]["resid"] <= 1e-10
        if i in (1, 4):
            Kd = exported_user_csr(m)[0].toarray()
            Z = oracle.rademacher_probes(5, S, p.n)
            gam, _ = oracle.logdet_same_probe(Kd, Z)
            assert abs(reps[i]["logdet"] - gam) <= 1e-8 * abs(gam)
            gref, parts = oracle.grad_same_probe(p.x, p.y, Z, p.radius, p.bump_width, p.centers, p.weights,
                                                 p.noise_var, K=Kd)
            sc = np.maximum(np.abs(gref), 1e-6 * (np.abs(parts["fit"]) + 0.5 * np.abs(parts["tau"])))
            assert np.all(np.abs(grads[i] - gref) <= 1e-4 * sc)
    b.free()


def test_batch_new_hyperparameters_and_capacity(gpu):
    G = _G()
    probs = _instances()[:3]
    opts = G.default_opts(n_probes=8, seed=1, tol=1e-9, probe_tol=1e-7, precond="jacobi")
    b = G.Batch([p.x for p in probs], [params_of(p) for p in probs], "fp64", opts)
    # smaller radius and new weights / noise: equals a fresh single-instance evaluation
    new = []
    for p in probs:
        q = params_of(p)
        q.radius = p.radius * 0.9
        q.weights = np.asarray(p.weights) * 1.1
        q.noise_var = p.noise_var * 2
        new.append(q)
    lml, grads, reps = b.run([p.y for p in probs], params=new)
    for i, p in enumerate(probs):
        m = G.gp2s_assemble(p.x, new[i], "fp64")
        rep, g1, _ = G.gp2s_lml_grad(m, p.y, opts)
        assert abs(lml[i] - rep.lml) <= 1e-8 * abs(rep.lml)
    # a much larger radius needs more entries than reserved
    big = [params_of(p) for p in probs]
    big[0].radius = probs[0].radius * 12  # every pair of the first instance
    with pytest.raises(G.GP2SError) as e:
        b.run([p.y for p in probs], params=big)
    assert e.value.status == 4
    # geometry changes are rejected
    bad = [params_of(p) for p in probs]
    bad[1].bump_width = 0.3
    with pytest.raises(G.GP2SError) as e:
        b.run([p.y for p in probs], params=bad)
    assert e.value.status == 1
    b.free()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_block_preconditioner_against_oracle(gpu, precision):
    """The block preconditioner in the batch: each instance's blocks are 64-point runs of
    its own bin order (the batch's grid: the tuned bin refinement, at most max(4 n, 4096)
    cells), so the same-probe log-determinant and gradient equal the oracle's with those
    blocks (1e-8 and 1e-4), the y residual meets the tolerance, and the LML matches the
    Jacobi-preconditioned batch to the probe noise of both estimates."""
    G = _G()
    probs = _instances()
    S = 16
    opts = G.default_opts(n_probes=S, seed=5, tol=1e-10, probe_tol=1e-10, max_iter=30000, precond="block")
    b = G.Batch([p.x for p in probs], [params_of(p) for p in probs], precision, opts)
    info = b.info()
    lml, grads, reps = b.run([p.y for p in probs])
    bj = G.Batch([p.x for p in probs], [params_of(p) for p in probs], precision,
                 G.default_opts(n_probes=S, seed=5, tol=1e-10, probe_tol=1e-10, max_iter=30000, precond="jacobi"))
    lml_j, _, reps_j = bj.run([p.y for p in probs])
    for i, p in enumerate(probs):
        m = G.gp2s_assemble(p.x, params_of(p), precision)
        Kd = exported_user_csr(m)[0].toarray()
        m.free()
        Z = oracle.rademacher_probes(5, S, p.n)
        order = oracle.bin_order(p.x, p.radius, refine=info["bin_refinement"], min_cells=4096)
        blocks = oracle.block_partition(order, oracle.BATCH_BLOCK)
        gam, _ = oracle.logdet_same_probe(Kd, Z, blocks)
        gref, parts = oracle.grad_same_probe(p.x, p.y, Z, p.radius, p.bump_width, p.centers, p.weights,
                                             p.noise_var, K=Kd, blocks=blocks)
        sc = np.maximum(np.abs(gref), 1e-6 * (np.abs(parts["fit"]) + 0.5 * np.abs(parts["tau"])))
        gerr = np.max(np.abs(grads[i] - gref) / sc)
        print(f"[batch-block/{precision}] instance {i}: logdet rel {abs(reps[i]['logdet'] - gam) / abs(gam):.2e}, "
              f"grad {gerr:.2e}, iters {reps[i]['iters']}/{reps[i]['probe_iters']} vs jacobi "
              f"{reps_j[i]['iters']}/{reps_j[i]['probe_iters']}, stderr {reps[i]['logdet_stderr']:.3g} vs "
              f"{reps_j[i]['logdet_stderr']:.3g}", flush=True)
        assert abs(reps[i]["logdet"] - gam) <= 1e-8 * abs(gam)
        assert gerr <= 1e-4
        assert reps[i]["resid"] <= 1e-10
        noise = 4 * np.hypot(reps[i]["logdet_stderr"], reps_j[i]["logdet_stderr"])
        assert abs(lml[i] - lml_j[i]) <= 0.5 * noise + 1e-8 * abs(lml[i])
    b.free()
    bj.free()


def test_batch_with_a_large_instance(gpu):
    """A 60 000-point instance beside two small ones (2-D and 3-D): each instance equals
    its own single-instance run on the same probes (diagonal preconditioner, so both
    define the same estimator), and every residual meets the tolerance."""
    G = _G()
    probs = [workloads.make_random_problem(90, 60_000, 2, 0.0146, n_bumps=4, bump_width=0.55),
             workloads.make_random_problem(91, 1800, 3, 0.1, n_bumps=3, bump_width=0.5, points="gmm"),
             workloads.make_random_problem(92, 900, 2, 0.06, n_bumps=2, bump_width=0.55)]
    S = 16
    opts = G.default_opts(n_probes=S, seed=8, tol=1e-10, probe_tol=1e-9, max_iter=40000, precond="jacobi")
    b = G.Batch([p.x for p in probs], [params_of(p) for p in probs], "mixed", opts)
    print(f"[batch/large] {b.info()}", flush=True)
    lml, grads, reps = b.run([p.y for p in probs])
    for i, p in enumerate(probs):
        m = G.gp2s_assemble(p.x, params_of(p), "mixed")
        rep, g1, _ = G.gp2s_lml_grad(m, p.y, opts)
        print(f"[batch/large] instance {i}: n={p.n} lml {lml[i]:.8f} single {rep.lml:.8f} iters "
              f"{reps[i]['iters']}/{reps[i]['probe_iters']}", flush=True)
        assert abs(lml[i] - rep.lml) <= 1e-9 * abs(rep.lml)
        scale = np.maximum(np.abs(g1), 1e-8 * np.abs(g1).max())
        assert np.all(np.abs(grads[i] - g1) <= 1e-6 * scale), (i, grads[i], g1)
        assert reps[i]["resid"] <= 1e-10
        m.free()
    b.free()
