"""Benchmark: seconds per LML + gradient on one MI355X, plus assembly nnz/s, CG
product bandwidth and the roofline of the dominant kernel.

A step is one pass of the whole hot path over one synthetic instance whose inputs
are already in HBM: bin + cull + assemble K, solve K a = y (block-Jacobi PCG with
refinement), probe solves + log-determinant, LML, and the gradient kernel.
Default workload: 200 000 uniform 2-D points, r = 0.01 (63 stored entries per row),
8 bumps, 64 probes; float32 K with float64 CG, timed against the float64-plain path
on the same inputs. Beside the timed steps (not in `value`):

* `parity`: every parity error against the oracle at the solver settings the steps
  use (the 4 000-point workload and a 5 000-point subsample of the timed one, dense
  same-probe oracle; sampled rows and the CPU-recomputed residual of the timed
  matrix itself);
* `large`: the 10 000 000-point clustered workload (the size the metric names):
  assembly nnz/s, the single-RHS product, per-kernel times and rooflines of the
  64-column probe block at that size from LML+gradient runs capped at two iteration
  counts (their difference gives the time per iteration), the y solve to convergence,
  and the projected seconds per LML+gradient;
* `batch`: the 64-instance batched workload, instances per second;
* `posterior`, `mcmc`, `variants`: the posterior at 100 000 test points, one block
  Metropolis-Hastings sweep, and one LML+gradient with each other kernel (the C^6
  member, Eq. wendconv with axis radii, the far-field bump kernel) on the timed cloud;
* `cpu_baseline`: the oracle's sparse LML+gradient timed on a bounded window.

The timed steps bracket only the dominant kernel with HIP events (for its roofline);
the per-kernel breakdown comes from one extra, untimed, fully instrumented step.

Prints one JSON line (last line of stdout).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_VALU_LANE = 256 * 64 * 2.4e9   # lane-instructions/s: 256 CUs x 64 lanes x 2.4 GHz


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(cat, n, nnz, S, prec, precond="block"):
    """Algorithmic HBM bytes of one launch of a timed kernel category: the CSR once,
    each vector stream once, at the types the path stores them in (the probe block
    of the mixed path keeps its search directions P and, with the block
    preconditioner, z = M^-1 r in float32; products Q, x and r are float64; the y
    solve applies a float32 copy of M^-1)."""
    mrow = 64 if precond in ("block64", 2) else 128                # M^-1 values per row
    vb = 4 if prec == "mixed" else 8                        # stored K value
    block = "block" in cat
    pb = 4 if (prec == "mixed" and block) else 8            # P element
    K = nnz * (4 + vb) + (n + 1) * 8
    if cat in ("cg_matvec_block", "cg_matvec1", "spmv"):
        return K + n * S * (pb + 8)                 # read P once, write Q
    if precond in ("block", "block64", 1, 2):
        zb = 4 if (prec == "mixed" and block) else 8        # stored z
        mb = 8 if block else 4                              # M^-1 element (mrow per row)
        if cat in ("cg_update_block", "cg_update1"):
            return n * S * (8 * 4 + pb + 8 + zb) + n * mrow * mb  # X, R read+write; P, Q read; z written; M^-1
        if cat in ("cg_pupdate_block", "cg_pupdate1"):
            return n * S * (zb + pb * 2)            # z read; P read+write
    if cat in ("cg_update_block", "cg_update1"):
        return n * S * (8 * 4 + pb + 8) + n * 8     # X, R read+write; P, Q read; 1/diag
    if cat in ("cg_pupdate_block", "cg_pupdate1"):
        return n * S * (8 + pb * 2) + n * 8         # R read; P read+write; 1/diag
    if cat == "asm_fill":
        return nnz * (4 + vb)                       # CSR written
    return None


# CG convergence poll interval of the single-matrix solves: the host learns of convergence
# at most two polls late (the polls are lagged so the queue never drains), and the
# iterations in between are full-cost no-ops; 4 measured 4.7% faster per step than 32 at
# 200 000 points. The batched leg keeps 32 (there it is also the captured chunk length).
POLL = 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c2_mixed.md")
TRAFFIC_KERNEL = {"cg_update_block": "k_bj_update<128, 4, float, true, false, double, float>",
                  "cg_pupdate_block": "k_cg_pupdate_z32<float>", "cg_matvec1": "k_spmv_a<float, true>"}
# sources of the CG kernels whose counters the summary holds (hashed in this order)
TRAFFIC_SOURCES = ("spmv.hip", "spmm_rows.h", "grouped.hip", "pcg.hip", "blockjac.hip", "bj_apply.h", "gp2s_internal.h")


def block_kernel_name(variant, S):
    """Kernel name (as rocprofv3 prints it) of the mixed path's probe-block product, or
    None for the split product (variant 5, two different kernels). Variant 6 launches
    k_spmm_s twice per product."""
    if variant == 5:
        return None
    if variant == 6:
        return f"k_spmm_s<{S}, float, float, true>"
    if variant == 0:
        return "k_spmm<float, float, double, true>"
    if variant == 1:
        return f"k_spmm_s<{S}, float, float, true>"
    if variant == 2:
        return f"k_spmm_t<{S}, float, float, true>"
    if variant == 3:
        return f"k_spmm_g<{S}, float, float, true>"
    return f"k_spmm_e<{variant}, {S}, float, float, true>"


def measured_traffic(cat, config, precision, kernel_name=None, launches=1):
    """Scaled FETCH_SIZE + WRITE_SIZE bytes per dispatch from the committed rocprofv3
    summary, times the dispatches per timed launch, or None when it does not cover
    this kernel/workload or the kernel sources changed since the counters were taken."""
    import hashlib
    name = kernel_name or TRAFFIC_KERNEL.get(cat)
    if config != "c2" or precision != "mixed" or name is None or not os.path.exists(TRAFFIC_FILE):
        return None
    h = hashlib.sha256()
    for fn in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_06143_amd", "csrc", fn), "rb") as fh:
            h.update(fh.read())
    text = open(TRAFFIC_FILE).read()
    if f"kernel-source-sha256: {h.hexdigest()}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"| `{name}` |"):
            cells = [c.strip() for c in line.strip("|").split("|")]
            return (float(cells[2]) + float(cells[5])) * 1e6 * launches
    return None


def make_inputs(args):
    import numpy as np
    import workloads
    t0 = time.perf_counter()
    prob = workloads.make_problem(args.config, n=args.n)
    log(f"[bench] generated {args.config}: n={prob.n} d={prob.dim} r={prob.radius:.6g} P={prob.n_bumps} "
        f"({time.perf_counter() - t0:.1f}s)")
    return prob


BLOCK_PRODUCT = {}  # variant of the probe-block product chosen in the last step
NOCONV = {"steps": 0, "noconv": 0}  # steps run / steps whose CG stopped at max_iter


def run_step(G, x, y, params, precision, opts, block_product=None, keep=False):
    m = G.gp2s_assemble(x, params, precision)
    S = opts.n_probes
    if block_product is not None and S > 1:
        m.set_block_product(S, block_product)
    rep, grad, a = G.gp2s_lml_grad(m, y, opts, want_a=keep, allow_noconv=True)
    NOCONV["steps"] += 1
    if rep.status:
        NOCONV["noconv"] += 1
        log(f"[bench] WARNING: CG stopped at max_iter ({precision}): y iters={rep.iters} probe iters={rep.probe_iters}")
    if S > 1:
        BLOCK_PRODUCT[precision] = m.block_product(S)
    n, nnz = m.n, m.nnz
    if keep:
        return rep, grad, n, nnz, m, a
    m.free()
    return rep, grad, n, nnz


def cpu_baseline(prob, opts, side=0.06):
    """The oracle as it stands, timed on a bounded sample: a complete LML + gradient of
    its sparse float64 path (oracle.lml_grad_sparse: k-d tree assembly, Jacobi-PCG y
    solve, one Jacobi-PCG solve per probe with Lanczos quadrature from its coefficients,
    sparse dK contraction) on the points of the same cloud inside a square window of
    side `side` centred at (0.5, 0.5), with the step's probe count and tolerances, on one
    thread (BLAS limited to one thread). Measured, not projected."""
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_limits
    c = np.full(prob.dim, 0.5)
    sel = np.all(np.abs(prob.x - c) <= side / 2, axis=1)
    xs, ys = prob.x[sel], prob.y[sel]
    S = int(opts.n_probes)
    Z = oracle.rademacher_probes(int(opts.seed), S, xs.shape[0])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        lml, grad, parts = oracle.lml_grad_sparse(xs, ys, prob.radius, prob.bump_width, prob.centers, prob.weights,
                                                  prob.noise_var, Z, tol=float(opts.tol),
                                                  probe_tol=float(opts.probe_tol))
        dt = time.perf_counter() - t0
    its = int(parts["iters_y"]) + int(np.sum(parts["iters_probe"]))
    log(f"[bench] cpu oracle: {xs.shape[0]} points, {parts['nnz']} nnz, {S} probes: {dt:.1f}s "
        f"(y {parts['iters_y']} iterations, probes {int(np.max(parts['iters_probe']))} max)")
    return {
        "value": dt, "unit": "s per LML+grad (measured, on the sample)", "cores": 1, "kind": "oracle",
        "sample": (f"{xs.shape[0]} points of the timed cloud in the square of side {side} centred at (0.5, 0.5) "
                   f"({parts['nnz']} stored entries), {S} probes, tol {opts.tol:g}, probe tol {opts.probe_tol:g}, "
                   f"Jacobi preconditioner; oracle.lml_grad_sparse complete: assembly, y solve "
                   f"({parts['iters_y']} CG iterations), {S} probe solves ({its - int(parts['iters_y'])} CG "
                   f"iterations in all) with Lanczos quadrature, gradient contraction"),
        "n": int(xs.shape[0]), "nnz": int(parts["nnz"]), "cg_iterations": its,
        "nnz_iterations_per_s": parts["nnz"] * its / dt,
    }


def _export_user(m):
    """The handle's CSR in user order (scipy, float64 values) and the raw arrays."""
    import numpy as np
    import scipy.sparse as sp
    rp, col, val, perm = m.export()
    rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy().astype(np.float64)
    perm = perm.cpu().numpy().astype(np.int64)
    rows = perm[np.repeat(np.arange(m.n), np.diff(rp))]
    K = sp.csr_matrix((val, (rows, perm[col])), shape=(m.n, m.n))
    K.sort_indices()
    return K


def _pattern_errors(Kg, Kref, prob):
    """(mismatches, exempt): pairs in one stored pattern and not the other, except pairs
    with |rho^2 - 1| <= 1e-6 or touching a point within 1e-6 (in s) of a bump boundary."""
    import numpy as np
    import oracle
    a, b = Kg.tocoo(), Kref.tocoo()
    ka = a.row.astype(np.int64) * prob.n + a.col
    kb = b.row.astype(np.int64) * prob.n + b.col
    diff = np.setxor1d(ka, kb)
    if diff.size == 0:
        return 0, 0
    pairs = np.stack([diff // prob.n, diff % prob.n], 1)
    ex = oracle.boundary_exempt_pairs(prob.x, prob.radius, pairs)
    pts = oracle.boundary_exempt_points(prob.x, prob.centers, prob.bump_width)
    ex |= pts[pairs[:, 0]] | pts[pairs[:, 1]]
    return int((~ex).sum()), int(ex.sum())


def _max_rel_entry_err(Kg, Kref):
    import numpy as np
    A = Kg.tocoo()
    want = np.asarray(Kref.tocsr()[A.row, A.col]).ravel()
    mask = np.abs(want) >= 1e-30 * np.abs(Kref.diagonal()).max()
    return float(np.max(np.abs(A.data[mask] - want[mask]) / np.abs(want[mask]))) if mask.any() else 0.0


def parity_case(G, prob, precision, opts):
    """One LML + gradient through the C ABI at the given solver settings, against the
    oracle on the same probes, the same stored matrix and the same preconditioner
    blocks: the bars of the hot path (pattern exact but for the support boundary, K
    entries 1e-5 relative in float32 storage, residual 1e-8, same-probe ln|K| and LML
    1e-8, same-probe gradient 1e-4 per component)."""
    import numpy as np
    import oracle
    params = G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights)
    m = G.gp2s_assemble(prob.x, params, precision)
    rep, grad, a = G.gp2s_lml_grad(m, prob.y, opts, allow_noconv=True)
    a = a.cpu().numpy()
    Kg = _export_user(m)
    m.free()
    Kref = oracle.covariance_csr(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights, prob.noise_var)
    nmis, nex = _pattern_errors(Kg, Kref, prob)
    S = int(opts.n_probes)
    Z = oracle.rademacher_probes(int(opts.seed), S, prob.n)
    blocks = (oracle.block_partition(oracle.bin_order(prob.x, prob.radius), oracle.BLOCK)
              if int(opts.precond) == 1 else None)
    Kd = Kg.toarray()
    lml_ref, parts = oracle.lml_same_probe(Kd, prob.y, Z, blocks)
    gref, gparts = oracle.grad_same_probe(prob.x, prob.y, Z, prob.radius, prob.bump_width, prob.centers,
                                          prob.weights, prob.noise_var, K=Kd, blocks=blocks)
    scale = np.maximum(np.abs(gref), 1e-6 * (np.abs(gparts["fit"]) + 0.5 * np.abs(gparts["tau"])))
    exact = oracle.lml_dense(Kref.toarray(), prob.y)
    out = {
        "n": prob.n, "nnz": int(Kg.nnz), "converged": rep.status == 0, "iters": [rep.iters, rep.probe_iters],
        "pattern_mismatch": nmis, "pattern_exempt": nex, "max_rel_K_err": _max_rel_entry_err(Kg, Kref),
        "resid_stored_K": oracle.residual_rel(Kg, a, prob.y), "resid_fp64_K": oracle.residual_rel(Kref, a, prob.y),
        "logdet_rel_err_same_probe": abs(rep.logdet - parts["gamma"]) / abs(parts["gamma"]),
        "lml_rel_err_same_probe": abs(rep.lml - lml_ref) / abs(lml_ref),
        "grad_max_rel_err_same_probe": float(np.max(np.abs(grad - gref) / scale)),
        "logdet_z_vs_exact": (rep.logdet - exact.logdet) / rep.logdet_stderr,
        "logdet_storage_rel": abs(parts["logdet"] - exact.logdet) / abs(exact.logdet),
    }
    log(f"[bench] parity {prob.name}/{precision}: " + ", ".join(
        f"{k}={v:.2e}" if isinstance(v, float) else f"{k}={v}" for k, v in out.items()))
    return out


def parity_rows(m, a, prob, n_rows=2000):
    """The timed matrix itself: sampled rows against the oracle's rows (pattern and
    values) and the residual of the step's solution recomputed on the CPU from the
    exported CSR."""
    import numpy as np
    import oracle
    Kg = _export_user(m)
    rows = np.random.default_rng(1).choice(prob.n, size=min(n_rows, prob.n), replace=False)
    ref = oracle.covariance_rows(prob.x, prob.radius, prob.bump_width, prob.centers, prob.weights, prob.noise_var,
                                 rows)
    pts = oracle.boundary_exempt_points(prob.x, prob.centers, prob.bump_width)
    nmis = nex = 0
    err = 0.0
    dmax = np.abs(Kg.diagonal()).max()
    for i, (cols, vals) in zip(rows, ref):
        got = Kg.getrow(i)
        gc, gv = got.indices, got.data
        diff = np.setxor1d(gc, cols)
        if diff.size:
            pairs = np.stack([np.full(diff.size, i), diff], 1)
            ex = oracle.boundary_exempt_pairs(prob.x, prob.radius, pairs) | pts[diff] | pts[i]
            nmis += int((~ex).sum())
            nex += int(ex.sum())
        common, ia, ib = np.intersect1d(gc, cols, return_indices=True)
        keep = np.abs(vals[ib]) >= 1e-30 * dmax
        if keep.any():
            err = max(err, float(np.max(np.abs(gv[ia][keep] - vals[ib][keep]) / np.abs(vals[ib][keep]))))
    out = {"rows": int(rows.size), "pattern_mismatch": nmis, "pattern_exempt": nex, "max_rel_K_err": err,
           "resid_stored_K": oracle.residual_rel(Kg, a, prob.y)}
    log(f"[bench] parity on the timed matrix: {out}")
    return out


def bench_posterior(G, x, y, params, precision, prob, n_mean=100_000, n_var=64):
    """Posterior at test points (outside the timed step): the mean at n_mean uniform
    points over the data's box (cross-covariance assembly + one SpMV) and the variance
    at n_var of them (one 64-column block solve)."""
    import numpy as np
    import torch
    import workloads
    m = G.gp2s_assemble(x, params, precision)
    a, _ = G.gp2s_solve(m, y)
    rng = np.random.default_rng(77)
    lo, hi = prob.x.min(0), prob.x.max(0)
    xt = torch.as_tensor(workloads.f32(lo + (hi - lo) * rng.random((n_mean, prob.dim)))).cuda()
    G.gp2s_predict(m, xt[:1000], a, want_var=False)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mean, _, rep = G.gp2s_predict(m, xt, a, want_var=False)
    torch.cuda.synchronize()
    t_mean = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, var, rep_v = G.gp2s_predict(m, xt[:n_var], a, allow_noconv=True)
    torch.cuda.synchronize()
    t_var = time.perf_counter() - t0
    m.free()
    res = {"test_points": n_mean, "cross_nnz": int(rep.nnz_cross), "mean_s": t_mean,
           "mean_points_per_s": n_mean / t_mean, "var_points": n_var, "var_s": t_var,
           "var_iters": int(rep_v.var_iters), "var_blocks": int(rep_v.var_blocks)}
    log(f"[bench] posterior: mean at {n_mean} points {t_mean * 1e3:.2f} ms ({rep.nnz_cross} cross entries); "
        f"variance at {n_var} points {t_var:.2f} s ({rep_v.var_iters} CG iterations)")
    return res


def bench_mcmc(G, x, y, params, precision, opts, n_sweeps=1):
    """Block Metropolis-Hastings sweeps over (r, bump amplitudes, noise variance) on the
    timed workload (outside the timed step): one LML without gradient per block move,
    a pattern refill for moves that keep r, a fresh assembly for moves of r."""
    import numpy as np
    import torch
    import workloads
    P = len(np.asarray(params.weights))
    blocks = [[0], list(range(1, P + 1)), [P + 1]]
    theta = G.mcmc.theta_of(params)
    steps = np.concatenate([[0.01 * theta[0]], 0.05 * np.ones(P), [0.05 * theta[-1]]])
    draws = workloads.mcmc_draws(2024, n_sweeps, [len(b) for b in blocks])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mh = G.BlockMH(x, y, params, precision, opts, blocks=blocks, steps=steps)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    res = mh.run(n_sweeps, draws=draws)
    mh.free()
    out = {"sweeps": n_sweeps, "blocks": len(blocks), "s_per_sweep": res["seconds"] / n_sweeps,
           "s_per_lml": res["seconds"] / max(res["evals"], 1), "init_s": t_init,
           "evals": res["evals"], "refills": res["refills"], "assemblies": res["assemblies"],
           "accepted": res["accepted"], "lml": [float(v) for v in res["lml"]]}
    log(f"[bench] mcmc: {n_sweeps} sweep(s) of {len(blocks)} blocks in {res['seconds']:.2f}s "
        f"({out['s_per_lml']:.2f}s per LML; {res['refills']} refills, {res['assemblies']} assemblies; "
        f"accepted {res['accepted']})")
    return out


def bench_variants(G, x, y, params, precision, opts, steps=1):
    """One assemble + LML + gradient per kernel variant on the timed workload (outside
    the timed step): the C^6 member, the non-stationary convolution form (Eq. wendconv)
    with axis radii and a length-scale field, and the far-field bump kernel
    (Eq. bump_kernel) with the bumps in 4 groups."""
    import dataclasses
    import numpy as np
    import torch
    P = len(np.asarray(params.weights))
    r = params.radius
    variants = {
        "wendland_c6": dataclasses.replace(params, kernel=1),
        "wendconv_ard": dataclasses.replace(params, radii=np.array([r, 0.8 * r] + [r] * (params.dim - 2)),
                                            ls_weights=np.array([0.15 if q % 2 else -0.15 for q in range(P)])),
        "far_field_u4": dataclasses.replace(params, ff_groups=np.arange(P, dtype=np.int32) % 4),
    }
    out = {}
    for name, hp in variants.items():
        run_step(G, x, y, hp, precision, opts)  # warm (tuning of the new matrix's products)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rep, grad, n, nnz = run_step(G, x, y, hp, precision, opts)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        out[name] = {"s_per_lml_grad": t, "nnz": nnz, "iters": [rep.iters, rep.probe_iters], "lml": rep.lml,
                     "n_grad": len(grad)}
        log(f"[bench] variant {name}: {t:.3f}s per LML+grad, nnz={nnz}, iters y={rep.iters} probes={rep.probe_iters}")
    return out


def bench_large(G, opts, config="c4", reps=3, spmv_reps=20, caps=(20, 100, 300), converge_y=True,
                precond="block64"):
    """The 10 000 000-point clustered workload, float32 and float64 storage (outside the
    timed steps: a converged LML+gradient at this size takes minutes).

    * assembly: K nnz/s from the library's HIP events (mean of `reps`);
    * the standalone single-RHS product: algorithmic HBM rate;
    * LML + gradient with 64 probes capped at caps[0] (fresh handle: includes the
      block factorisation and the product's tuning), caps[1] and caps[2] iterations on
      the same handle: their wall-time difference gives the time per iteration of the
      two concurrent chains (y solve + probe block) at full size, the rest the fixed
      cost (right-hand sides, quadrature, gradient kernel); one more capped run with
      every kernel bracketed by events gives per-kernel times and the rooflines of the
      probe-block product and update at this size;
    * the float32-stored y solve to convergence (its iteration count);
    * projected s per LML+gradient = assembly + first-call extra + fixed + per-iteration
      x the y solve's iteration count to convergence. This is an estimate, not a bound:
      the two chains run side by side until the longer one ends, and the probe block,
      despite its looser tolerance, can need a few percent more iterations than the y
      solve (31 800 against 30 897 in a full float32-stored run at this size).
    The solves use the block preconditioner over 64-point runs: on this clustered cloud
    the y solve takes ~30 900 iterations with them and ~31 100 with 128-point runs,
    which cost more per iteration."""
    import numpy as np
    import torch
    import workloads
    t0 = time.perf_counter()
    prob = workloads.make_problem(config)
    log(f"[bench] large: generated {config}: n={prob.n} r={prob.radius:.6g} ({time.perf_counter() - t0:.1f}s)")
    x = torch.as_tensor(prob.x).cuda()
    y = torch.as_tensor(prob.y).cuda()
    params = G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights)
    v = torch.as_tensor(np.random.default_rng(0).standard_normal(prob.n)).cuda()
    ctx = G.default_context()
    S = prob.n_probes
    out = {"workload": (f"{config}: {prob.n} clustered {prob.dim}-D points (200-component mixture), "
                        f"r={prob.radius:.6g}, {prob.n_bumps} bumps, {S} probes"), "n": prob.n, "probes": S}

    def capped(cap):
        return G.default_opts(n_probes=S, max_iter=cap, tol=float(opts.tol), probe_tol=float(opts.probe_tol),
                              check_every=POLL, precond=precond)
    out["precond"] = precond

    for prec in ("mixed", "fp64"):
        G.gp2s_assemble(x, params, prec).free()  # warm
        ctx.set_timing(True)
        for k in range(reps):
            m = G.gp2s_assemble(x, params, prec)
            if k < reps - 1:
                m.free()
        st = ctx.stats()
        asm_ms = sum(st[k][0] for k in ("asm_prep", "asm_count", "asm_fill")) / reps
        n, nnz = m.n, m.nnz
        G.gp2s_spmv(m, v)  # warm
        ctx.set_timing(True)
        for _ in range(spmv_reps):
            G.gp2s_spmv(m, v)
        ms, cnt = ctx.stats()["spmv"]
        ctx.set_timing(False)
        b = kernel_bytes("spmv", n, nnz, 1, prec)
        gbs = b / (ms / cnt / 1e3) / 1e9
        r = {"nnz": nnz, "assembly_ms": asm_ms, "assembly_nnz_per_s": nnz / (asm_ms / 1e3),
             "assembly_count_ms": st["asm_count"][0] / reps, "assembly_fill_ms": st["asm_fill"][0] / reps,
             "spmv_ms": ms / cnt, "spmv_bytes": b, "spmv_GBps": gbs, "spmv_frac_hbm": gbs * 1e9 / PEAK_HBM}
        log(f"[bench] large {prec}: nnz={nnz} ({nnz / n:.1f}/row), assembly {asm_ms:.2f} ms "
            f"({nnz / (asm_ms / 1e3):.3g} nnz/s), spmv {ms / cnt:.3f} ms = {gbs:.0f} GB/s "
            f"({100 * gbs * 1e9 / PEAK_HBM:.1f}% of HBM)")
        walls = []
        for cap in caps:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep, grad, _ = G.gp2s_lml_grad(m, y, capped(cap), want_a=False, allow_noconv=True)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            log(f"[bench] large {prec}: LML+grad capped at {cap} iterations: {walls[-1]:.2f}s "
                f"(y {rep.iters}, probes {rep.probe_iters})")
        slope = (walls[2] - walls[1]) / (caps[2] - caps[1])
        fixed = walls[1] - caps[1] * slope
        first = walls[0] - (fixed + caps[0] * slope)
        ctx.set_timing(True)
        G.gp2s_lml_grad(m, y, capped(caps[1]), want_a=False, allow_noconv=True)
        st = ctx.stats()
        ctx.set_timing(False)
        kern = {k: {"ms_avg": v[0] / v[1], "launches": v[1]} for k, v in st.items() if v[1]}
        roof = {}
        for cat in ("cg_matvec_block", "cg_update_block", "cg_pupdate_block", "cg_matvec1", "cg_update1"):
            if cat in kern:
                bb = kernel_bytes(cat, n, nnz, S if "block" in cat else 1, prec, precond)
                avg = kern[cat]["ms_avg"] / 1e3
                roof[cat] = {"bound": "hbm", "achieved": bb / avg / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                             "frac": bb / avg / PEAK_HBM, "bytes_per_launch": bb, "avg_ms": avg * 1e3}
        r.update({"capped_runs": {str(c): w for c, w in zip(caps, walls)}, "s_per_iteration": slope,
                  "fixed_s": fixed, "first_call_extra_s": first, "kernels": kern, "rooflines": roof})
        log(f"[bench] large {prec}: {slope * 1e3:.2f} ms per iteration (both chains), fixed {fixed:.2f}s, "
            f"first-call extra {first:.2f}s; probe block product "
            f"{roof.get('cg_matvec_block', {}).get('frac', float('nan')):.3f} of HBM")
        if converge_y and prec == "mixed":
            last = [time.perf_counter()]

            def prog(label, it, open_cols, res):
                if time.perf_counter() - last[0] > 10.0:
                    last[0] = time.perf_counter()
                    log(f"[bench]   ... large y solve: {it} iterations, max rel resid {res:.2e}")
            ctx.set_progress(prog)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a, rep = G.gp2s_solve(m, y, G.default_opts(max_iter=200000, tol=float(opts.tol), precond=precond,
                                                       check_every=POLL), allow_noconv=True)
            torch.cuda.synchronize()
            ty = time.perf_counter() - t0
            ctx.set_progress(None)
            out["y_solve_mixed"] = {"iters": rep.iters, "ir_steps": rep.ir_steps, "resid": rep.resid, "s": ty,
                                    "converged": rep.status == 0}
            log(f"[bench] large mixed y solve: {rep.iters} iterations, resid {rep.resid:.2e}, {ty:.1f}s")
        out[prec] = r
        m.free()
        torch.cuda.empty_cache()
    if "y_solve_mixed" in out:
        iters = out["y_solve_mixed"]["iters"]
        for prec in ("mixed", "fp64"):
            r = out[prec]
            r["projected_s_per_lml_grad"] = (r["assembly_ms"] / 1e3 + r["first_call_extra_s"] + r["fixed_s"]
                                             + r["s_per_iteration"] * iters)
        out["projected_speedup_mixed_vs_fp64"] = (out["fp64"]["projected_s_per_lml_grad"]
                                                  / out["mixed"]["projected_s_per_lml_grad"])
        log(f"[bench] large projected s per LML+grad at {iters} iterations: mixed "
            f"{out['mixed']['projected_s_per_lml_grad']:.1f}s, fp64 {out['fp64']['projected_s_per_lml_grad']:.1f}s")
    del x, y, v
    torch.cuda.empty_cache()
    return out


def batch_leg(G, precision="mixed", precond="block", steps=2, warmup=1, S=16, max_iter=40000, tol=1e-8,
              probe_tol=1e-5):
    """64 independent instances (c5) planned once, then evaluated together per step:
    reassembly with the step's hyperparameters, y solves, probe solves, log-dets, LMLs
    and gradients of all instances. Instances per second."""
    import numpy as np
    import torch
    import workloads
    t0 = time.perf_counter()
    probs = workloads.make_c5()
    xs = [torch.as_tensor(p.x).cuda() for p in probs]
    ys = [torch.as_tensor(p.y).cuda() for p in probs]
    params = [G.HostParams(p.dim, p.radius, p.bump_width, p.noise_var, p.centers, p.weights) for p in probs]
    opts = G.default_opts(n_probes=S, max_iter=max_iter, tol=tol, probe_tol=probe_tol, check_every=32,
                          precond=precond)
    ctx = G.default_context()
    b = G.Batch(xs, params, precision, opts, ctx)
    info = b.info()
    log(f"[bench] batch: planned {len(probs)} instances, {info} ({time.perf_counter() - t0:.1f}s)")
    for w in range(warmup):
        lml, grads, reps = b.run(ys, params=params, allow_noconv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    noconv = 0
    for k in range(steps):
        lml, grads, reps = b.run(ys, params=params, allow_noconv=True)
        noconv += sum(1 for r in reps if r["iters"] >= max_iter or r["probe_iters"] >= max_iter)
        log(f"[bench] batch step {k}: iters y max {max(r['iters'] for r in reps)} median "
            f"{int(np.median([r['iters'] for r in reps]))}, probes max {max(r['probe_iters'] for r in reps)}, "
            f"max resid {max(r['resid'] for r in reps):.2e}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    M = len(probs)
    b.free()
    return {
        "value": M / dt, "unit": "instances/s", "s_per_batch": dt, "steps": steps, "warmup": warmup,
        "workload": (f"c5: {M} instances, N {min(p.n for p in probs)}-{max(p.n for p in probs)} "
                     f"(total {info['n_total']}), d in {{2,3}}, {S} probes each"),
        "n_total": info["n_total"], "nnz": info["nnz"], "precision": precision, "precond": precond,
        "autotuned": {k: info[k] for k in ("bin_refinement", "spmv_lanes", "spmm_lanes")},
        "max_iters_y": max(r["iters"] for r in reps), "max_iters_probe": max(r["probe_iters"] for r in reps),
        "median_iters_y": int(np.median([r["iters"] for r in reps])),
        "all_converged": noconv == 0 and max(r["resid"] for r in reps) <= tol,
    }


def bench_batch(args):
    """`--config c5`: the batched workload as the timed metric."""
    import paper_2512_06143_amd as G
    S = args.probes if args.probes is not None else 16
    r = batch_leg(G, args.precision, args.precond, args.steps, args.warmup, S, args.max_iter, args.tol,
                  args.probe_tol)
    out = {
        "metric": "instances/s, batched LML+grad (64 uneven instances)",
        "value": r["value"], "unit": "instances/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["s_per_batch"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 K / f64 CG" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": r["workload"], "n_total": r["n_total"], "nnz": r["nnz"],
                   "precision": args.precision, "precond": args.precond, "autotuned": r["autotuned"],
                   "parallelism": "single GPU"},
        "max_iters_y": r["max_iters_y"], "max_iters_probe": r["max_iters_probe"], "roofline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--n", type=int, default=None, help="override the point count (same recipe)")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--probes", type=int, default=None)
    ap.add_argument("--max-iter", type=int, default=40000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--probe-tol", type=float, default=1e-5)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64-plain comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-predict", action="store_true", help="skip the posterior (test-point) measurement")
    ap.add_argument("--no-mcmc", action="store_true", help="skip the block Metropolis-Hastings sweep")
    ap.add_argument("--no-variants", action="store_true", help="skip the kernel-variant measurements")
    ap.add_argument("--no-large", action="store_true", help="skip the 10 M-point measurements")
    ap.add_argument("--only-large", action="store_true", help="run only the 10 M-point measurements")
    ap.add_argument("--no-parity", action="store_true", help="skip the in-run parity comparison with the oracle")
    ap.add_argument("--only-assembly", action="store_true",
                    help="only assemble the --config workload (float32 and float64 storage, --steps times each) and "
                         "print the library's per-stage times: the driver for profiling the assembly kernels")
    ap.add_argument("--only-product", action="store_true",
                    help="only assemble the --config workload (float32 and float64 storage) and time the single-RHS "
                         "product gp2s_spmv (--steps launches each): the driver for profiling that kernel")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (64-instance) measurement")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="skip the extra, fully instrumented step (the per-kernel breakdown); the timed steps then "
                         "bracket the probe-block product for the roofline")
    ap.add_argument("--no-jacobi", action="store_true",
                    help="skip the same step with the diagonal preconditioner (comparison and CPU projection)")
    ap.add_argument("--precond", default="block", choices=["block", "block64", "jacobi"],
                    help="preconditioner of the timed step (the other one is timed once beside it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs on one "
              "GPU; how the path would shard over several is described in the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2512_06143_amd as G

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.config == "c5":
        return bench_batch(args)
    if args.only_assembly:
        import workloads
        prob = workloads.make_problem(args.config, n=args.n)
        x = torch.as_tensor(prob.x).cuda()
        params = G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights)
        ctx = G.default_context()
        res = {"workload": f"{args.config}: n={prob.n} r={prob.radius:.6g}"}
        for prec in ("mixed", "fp64"):
            G.gp2s_assemble(x, params, prec).free()
            ctx.set_timing(True)
            for _ in range(args.steps):
                m = G.gp2s_assemble(x, params, prec)
                nnz = m.nnz
                m.free()
            st = ctx.stats()
            ctx.set_timing(False)
            ms = {k: st[k][0] / args.steps for k in ("asm_prep", "asm_count", "asm_fill")}
            tot = sum(ms.values())
            res[prec] = {"nnz": nnz, "ms": ms, "nnz_per_s": nnz / (tot / 1e3)}
            log(f"[bench] assembly {prec}: nnz={nnz} {ms} -> {nnz / (tot / 1e3):.3g} nnz/s")
        print(json.dumps(res), flush=True)
        return
    if args.only_product:
        import workloads
        prob = workloads.make_problem(args.config, n=args.n)
        x = torch.as_tensor(prob.x).cuda()
        v = torch.as_tensor(np.random.default_rng(0).standard_normal(prob.n)).cuda()
        params = G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights)
        ctx = G.default_context()
        res = {"workload": f"{args.config}: n={prob.n} r={prob.radius:.6g}"}
        for prec in ("mixed", "fp64"):
            m = G.gp2s_assemble(x, params, prec)
            G.gp2s_spmv(m, v)  # warm
            ctx.set_timing(True)
            for _ in range(args.steps):
                G.gp2s_spmv(m, v)
            ms, cnt = ctx.stats()["spmv"]
            ctx.set_timing(False)
            b = kernel_bytes("spmv", m.n, m.nnz, 1, prec)
            gbs = b / (ms / cnt / 1e3) / 1e9
            res[prec] = {"nnz": m.nnz, "spmv_ms": ms / cnt, "spmv_bytes": b, "spmv_GBps": gbs,
                         "spmv_frac_hbm": gbs * 1e9 / PEAK_HBM}
            log(f"[bench] product {prec}: nnz={m.nnz} {ms / cnt:.3f} ms = {gbs:.0f} GB/s "
                f"({100 * gbs * 1e9 / PEAK_HBM:.1f}% of HBM)")
            m.free()
        print(json.dumps(res), flush=True)
        return
    if args.only_large:
        opts = G.default_opts(max_iter=args.max_iter, tol=args.tol, probe_tol=args.probe_tol, check_every=POLL,
                              precond=args.precond)
        print(json.dumps({"large": bench_large(G, opts)}), flush=True)
        return
    prob = make_inputs(args)
    S = args.probes if args.probes is not None else prob.n_probes
    x = torch.as_tensor(prob.x).cuda()
    y = torch.as_tensor(prob.y).cuda()
    params = G.HostParams(prob.dim, prob.radius, prob.bump_width, prob.noise_var, prob.centers, prob.weights)
    opts = G.default_opts(n_probes=S, max_iter=args.max_iter, tol=args.tol, probe_tol=args.probe_tol,
                          check_every=POLL, precond=args.precond)
    ctx = G.default_context()
    last = [0.0]

    def progress(label, it, open_cols, res):
        now = time.perf_counter()
        if now - last[0] > 10.0:
            last[0] = now
            log(f"[bench]   ... {label}: {it} iterations, {open_cols} open, max rel resid {res:.2e}")
    ctx.set_progress(progress)

    for w in range(args.warmup):
        t0 = time.perf_counter()
        rep, grad, n, nnz = run_step(G, x, y, params, args.precision, opts)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w}: {time.perf_counter() - t0:.2f}s iters y={rep.iters} probes={rep.probe_iters} "
            f"lml={rep.lml:.6f}")

    # One more untimed step with every kernel category bracketed by HIP events: the
    # per-kernel breakdown, and the dominant kernel. The timed steps then record events
    # for that kernel only (its roofline), so the host work of ~10^4 event pairs per step
    # does not enter the step time.
    if args.no_breakdown:
        stats, per, dom = None, {}, "cg_matvec_block"
    else:
        ctx.set_timing(True)
        rep, grad, n, nnz = run_step(G, x, y, params, args.precision, opts)
        stats = ctx.stats()
        ctx.set_timing(False)
        for name, (ms, cnt) in stats.items():
            if cnt:
                log(f"[bench]   {name:18s} {ms:10.2f} ms  {cnt:7d} launches  {ms / cnt:9.4f} ms avg (instrumented step)")
        per = {k: v for k, v in stats.items() if v[1] > 0}
        dom = max(per, key=lambda k: per[k][0])
    ctx.set_timing(True, only=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rep, grad, n, nnz = run_step(G, x, y, params, args.precision, opts)
        log(f"[bench] step {k}: iters y={rep.iters} probes={rep.probe_iters} resid={rep.resid:.2e} "
            f"lml={rep.lml:.6f}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    dstats = ctx.stats()
    ctx.set_timing(False)
    ms_per_step = 1e3 * t_total / args.steps
    log(f"[bench] {args.steps} step(s): {ms_per_step:.1f} ms/step; nnz={nnz} ({nnz / n:.2f}/row)")

    # dominant kernel and its roofline (its events over the timed steps)
    ms_tot, cnt = dstats[dom]
    log(f"[bench]   {dom:18s} {ms_tot:10.2f} ms total  {cnt:7d} launches  {ms_tot / cnt:9.4f} ms avg (timed steps)")
    avg_s = ms_tot / cnt / 1e3
    b = kernel_bytes(dom, n, nnz, S if "block" in dom else 1, args.precision, args.precond)
    roof = None
    if b is not None:
        roof = {"kernel": dom, "bound": "hbm", "achieved": b / avg_s / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": b / avg_s / PEAK_HBM,
                "traffic": measured_traffic(dom, args.config, args.precision,
                                            block_kernel_name(BLOCK_PRODUCT.get(args.precision), S)
                                            if dom == "cg_matvec_block" and args.precision == "mixed" else None,
                                            2 if dom == "cg_matvec_block" and BLOCK_PRODUCT.get(args.precision) == 6
                                            else 1),
                "bytes_per_launch": b, "avg_ms": avg_s * 1e3, "launches": cnt}
    if stats is None:  # no instrumented step: the timed steps' dominant-kernel events only
        stats = {k: (0.0, 0) for k in ("asm_prep", "asm_count", "asm_fill", "cg_matvec1")}
    asm_ms = sum(stats[k][0] for k in ("asm_prep", "asm_count", "asm_fill"))  # the instrumented step
    mv1 = stats["cg_matvec1"]
    spmv_gbs = (kernel_bytes("cg_matvec1", n, nnz, 1, args.precision) / (mv1[0] / mv1[1] / 1e3) / 1e9
                if mv1[1] else None)
    out = {
        "metric": "s per LML+grad, FP32-mixed vs FP64 plain (K nnz/s assembled alongside)",
        "value": ms_per_step / 1e3,
        "unit": "s/(LML+grad)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 K / f64 CG" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{args.config}: {n} {prob.meta.get('points', 'uniform')} {prob.dim}-D points, "
                                f"r={prob.radius:.6g} "
                                f"({nnz / n:.1f} stored/row), {prob.n_bumps} bumps, {S} probes"),
                   "n": n, "nnz": nnz, "probes": S, "precision": args.precision, "precond": args.precond,
                   "parallelism": "single GPU"},
        "assembly_ms": asm_ms, "assembly_nnz_per_s": nnz / (asm_ms / 1e3) if asm_ms else None,
        "cg_spmv_GBps": spmv_gbs,
        "iters_y": rep.iters, "iters_probe": rep.probe_iters, "ir_steps": rep.ir_steps,
        "block_product": ((block_kernel_name(BLOCK_PRODUCT[args.precision], S) or "split: k_spmm_sr + k_spmm_bb")
                          if BLOCK_PRODUCT.get(args.precision) is not None else None),
        "resid": rep.resid, "lml": rep.lml, "logdet": rep.logdet, "logdet_stderr": rep.logdet_stderr,
        "grad_r": float(grad[0]),
        "kernels_ms": {k: round(v[0], 3) for k, v in per.items()},  # per step, from the instrumented step
        "roofline": roof,
    }
    # the same step with the diagonal preconditioner (the comparison of preconditioners, and
    # the iteration counts of the oracle's own Jacobi PCG for the CPU projection)
    jac_iters = (rep.iters, rep.probe_iters)
    if args.precond != "jacobi" and not args.no_jacobi:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep_j, _, _, _ = run_step(G, x, y, params, args.precision, G.default_opts(
            n_probes=S, max_iter=args.max_iter, tol=args.tol, probe_tol=args.probe_tol, check_every=POLL,
            precond="jacobi"))
        torch.cuda.synchronize()
        tj = time.perf_counter() - t0
        jac_iters = (rep_j.iters, rep_j.probe_iters)
        out["jacobi_s_per_lml_grad"] = tj
        out["jacobi_iters"] = list(jac_iters)
        out["jacobi_lml"] = rep_j.lml
        out["jacobi_logdet_stderr"] = rep_j.logdet_stderr
        log(f"[bench] jacobi preconditioner: {tj:.2f}s iters y={rep_j.iters} probes={rep_j.probe_iters} "
            f"lml={rep_j.lml:.6f} (stderr of ln|K| {rep_j.logdet_stderr:.1f} vs {rep.logdet_stderr:.1f})")
    if not args.no_fp64 and args.precision == "mixed":
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep64, grad64, _, _ = run_step(G, x, y, params, "fp64", opts)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        out["fp64_plain_s_per_lml_grad"] = t64
        out["speedup_mixed_vs_fp64"] = t64 / (ms_per_step / 1e3)
        out["fp64_iters"] = [rep64.iters, rep64.probe_iters]
        out["fp64_lml"] = rep64.lml
        log(f"[bench] fp64 plain: {t64:.2f}s iters y={rep64.iters} probes={rep64.probe_iters} lml={rep64.lml:.6f}")
    out["all_converged"] = NOCONV["noconv"] == 0
    out["noconv_steps"] = NOCONV["noconv"]
    out["steps_run"] = NOCONV["steps"]
    if not args.no_parity:
        # the timed matrix itself (one more, untimed, step that keeps its handle), then the
        # dense same-probe oracle at the same solver settings
        rep_k, _, _, _, m_k, a_k = run_step(G, x, y, params, args.precision, opts, keep=True)
        par = {"settings": {"tol": args.tol, "probe_tol": args.probe_tol, "probes": S, "precond": args.precond,
                            "max_iter": args.max_iter, "seed": int(opts.seed)},
               "timed_matrix": parity_rows(m_k, a_k.cpu().numpy(), prob)}
        m_k.free()
        import workloads
        c1 = workloads.make_problem("c1")
        o1 = G.default_opts(n_probes=S, max_iter=args.max_iter, tol=args.tol, probe_tol=args.probe_tol,
                            check_every=POLL, precond=args.precond)
        par["c1_mixed"] = parity_case(G, c1, "mixed", o1)
        par["c1_fp64"] = parity_case(G, c1, "fp64", o1)
        if args.config == "c2":
            par["c2_sub5000_mixed"] = parity_case(G, prob.subsample(5000, seed=1), args.precision, o1)
        bars = {"pattern_mismatch": 0, "resid_stored_K": 1e-8, "logdet_rel_err_same_probe": 1e-8,
                "lml_rel_err_same_probe": 1e-8, "grad_max_rel_err_same_probe": 1e-4}
        ok = True
        for k, v in par.items():
            if not k.startswith("c"):
                continue
            ok &= bool(v["converged"]) and v["max_rel_K_err"] <= (1e-5 if "mixed" in k else 1e-9)
            ok &= all(v[b] <= lim for b, lim in bars.items())
        tm = par["timed_matrix"]
        ok &= tm["pattern_mismatch"] == 0 and tm["resid_stored_K"] <= 1e-8 and tm["max_rel_K_err"] <= 1e-5
        par["all_within_bars"] = bool(ok)
        out["parity"] = par
    if not args.no_predict:
        out["posterior"] = bench_posterior(G, x, y, params, args.precision, prob)
    if not args.no_mcmc:
        out["mcmc"] = bench_mcmc(G, x, y, params, args.precision, opts)
    if not args.no_variants:
        out["variants"] = bench_variants(G, x, y, params, args.precision, opts)
    if not args.no_batch:
        out["batch"] = batch_leg(G, args.precision, args.precond)
    if not args.no_large and args.config != "c4":
        del x, y
        torch.cuda.empty_cache()
        out["large"] = bench_large(G, opts)
    if not args.no_cpu:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(prob, opts)
        log(f"[bench] cpu baseline took {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
