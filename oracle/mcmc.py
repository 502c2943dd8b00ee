"""Block Metropolis-Hastings over the kernel hyperparameters (Sec. 4.6; App. D).

The hyperparameters theta = (r, a_1..a_P, sigma_n^2) are sampled in blocks (by
default the Wendland radius, the bump amplitudes and the noise variance, each a
block, as App. D separates the core-kernel block from the bump blocks). One sweep
visits every block once: a normal random-walk proposal moves that block's
components (App. D keeps proposals normal), a flat prior restricts theta to
bounds (App. D: a flat prior within well-chosen bounds), and the move is accepted
when log u < loglik(theta') - loglik(theta). Each block costs one likelihood
evaluation (Sec. 4.6). Random draws are inputs (workloads.mcmc_draws), so a
device run and this oracle take the same decisions.
"""
from __future__ import annotations

import numpy as np


def _margin(llp, ll, u):
    """Metropolis-Hastings margin for a symmetric proposal and a flat prior: the move is
    accepted when log u < loglik' - loglik, i.e. when this is positive."""
    return llp - ll - np.log(u)


def block_mh(theta0, blocks, steps, lo, hi, draws, loglik):
    """Run len(draws) sweeps. Returns (chain of theta after every sweep including the
    start, log-likelihoods alongside, per-block acceptance flags, per-block margins
    loglik' - loglik - log u (None for out-of-bounds proposals))."""
    theta = np.array(theta0, dtype=np.float64)
    steps = np.asarray(steps, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ll = float(loglik(theta))
    chain, lls, accepted, margins = [theta.copy()], [ll], [], []
    for sweep in draws:
        for idx, (eps, u) in zip(blocks, sweep):
            idx = np.asarray(idx)
            prop = theta.copy()
            prop[idx] = theta[idx] + steps[idx] * np.asarray(eps, dtype=np.float64)
            if np.any(prop[idx] <= lo[idx]) or np.any(prop[idx] >= hi[idx]):
                accepted.append(False)  # outside the flat prior's support
                margins.append(None)
                continue
            llp = float(loglik(prop))
            margin = _margin(llp, ll, u)
            ok = margin > 0.0
            accepted.append(bool(ok))
            margins.append(margin)
            if ok:
                theta, ll = prop, llp
        chain.append(theta.copy())
        lls.append(ll)
    return chain, lls, accepted, margins
