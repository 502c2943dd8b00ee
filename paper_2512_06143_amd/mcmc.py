"""Block Metropolis-Hastings training of the kernel hyperparameters (Sec. 4.6; App. D)
on the library's LML.

theta = (r | r_1..r_d, a_1..a_P, [c_1..c_P], sigma_n^2) in the gradient order of the
kernel (stationary, Eq. wendconv with axis radii and length-scale weights, or the
far-field kernel). Every sweep visits the blocks in order (by default the radius
components, the bump amplitudes, the length-scale weights and the noise variance, each
its own block, as App. D separates the core-kernel block from the bump blocks); a
block move draws a normal random-walk proposal for its components (App. D keeps
proposals normal), a flat prior restricts theta to bounds (App. D), and the move is
accepted when log u < LML(theta') - LML(theta). Each block costs one LML evaluation
(Sec. 4.6).

The LML is the library's estimate with a fixed probe seed, so every evaluation uses
the same probes (common random numbers across proposals). Moves that keep the
pattern (radii and length-scale weights unchanged) refill the stored pattern
(gp2s_matrix_refill: no count pass, no CSR allocation); other moves assemble a new
handle. Only argument marshalling happens here; every evaluation runs in the HIP
kernels.
"""
from __future__ import annotations

import time
from dataclasses import replace

import numpy as np

from .gp2s import HostParams, Matrix, _as_dev64, default_context, default_opts, gp2s_assemble, gp2s_lml


def _layout(p: HostParams):
    """(number of radius components, P, number of length-scale weights)."""
    P = len(np.asarray(p.weights).reshape(-1))
    nr = len(np.asarray(p.radii).reshape(-1)) if p.radii is not None else 1
    nc = P if p.ls_weights is not None else 0
    return nr, P, nc


def theta_of(p: HostParams) -> np.ndarray:
    """theta in the gradient order: (r | r_1..r_d, a_1..a_P, [c_1..c_P], sigma_n^2)."""
    parts = [np.atleast_1d(np.asarray(p.radii if p.radii is not None else p.radius, dtype=np.float64)).reshape(-1),
             np.asarray(p.weights, dtype=np.float64).reshape(-1)]
    if p.ls_weights is not None:
        parts.append(np.asarray(p.ls_weights, dtype=np.float64).reshape(-1))
    parts.append([p.noise_var])
    return np.concatenate(parts)


def params_of(base: HostParams, theta: np.ndarray) -> HostParams:
    nr, P, nc = _layout(base)
    theta = np.asarray(theta, dtype=np.float64)
    kw = dict(weights=np.array(theta[nr:nr + P]), noise_var=float(theta[nr + P + nc]))
    if base.radii is not None:
        kw["radii"] = np.array(theta[:nr])
    else:
        kw["radius"] = float(theta[0])
    if nc:
        kw["ls_weights"] = np.array(theta[nr + P:nr + P + nc])
    return replace(base, **kw)


def pattern_indices(base: HostParams) -> np.ndarray:
    """Components of theta that change the stored pattern (radii, length-scale weights)."""
    nr, P, nc = _layout(base)
    return np.concatenate([np.arange(nr), np.arange(nr + P, nr + P + nc)]).astype(np.int64)


class BlockMH:
    """Sampler state: the data, the current theta and its LML, and two matrix handles
    (the current state's and a proposal's)."""

    def __init__(self, x, y, params: HostParams, precision="mixed", opts=None, blocks=None, steps=None,
                 bounds=None, ctx=None):
        self.ctx = ctx or default_context()
        self.x, self.y = _as_dev64(x, self.ctx), _as_dev64(y, self.ctx)  # device-resident once
        self.base, self.precision = params, precision
        self.opts = opts or default_opts()
        nr, P, nc = _layout(params)
        default = [list(range(nr)), list(range(nr, nr + P))]
        if nc:
            default.append(list(range(nr + P, nr + P + nc)))
        default.append([nr + P + nc])
        self.blocks = blocks or default
        self._pat = pattern_indices(params)
        self.theta = theta_of(params)
        t = self.theta
        self.steps = np.asarray(steps if steps is not None else np.where(t != 0, 0.05 * np.abs(t), 0.05),
                                dtype=np.float64)
        if bounds is None:  # positive components within a factor 10, others within 1 + 10 |theta|
            span = 1.0 + 10.0 * np.abs(t)
            bounds = (np.where(t > 0, t / 10.0, t - span), np.where(t > 0, t * 10.0, t + span))
        lo, hi = bounds
        self.lo, self.hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
        self.cur = gp2s_assemble(self.x, params, precision, self.ctx)
        self.prop = None
        self.lml = self._lml(self.cur)
        self.evals = 0
        self.refills = 0
        self.assemblies = 1

    def _lml(self, m: Matrix) -> float:
        rep, _ = gp2s_lml(m, self.y, self.opts, want_a=False)
        return float(rep.lml)

    def _same_pattern(self, a: HostParams, theta: np.ndarray) -> bool:
        return a is not None and np.array_equal(theta_of(a)[self._pat], theta[self._pat])

    def _proposal_handle(self, theta: np.ndarray) -> Matrix:
        p = params_of(self.base, theta)
        if np.array_equal(theta[self._pat], self.theta[self._pat]):
            # same radii, length-scale field and geometry: refill a handle that holds the current pattern
            if self.prop is None or not self._same_pattern(self.prop.params, self.theta):
                if self.prop is not None:
                    self.prop.free()
                self.prop = gp2s_assemble(self.x, p, self.precision, self.ctx)
                self.assemblies += 1
            else:
                self.prop.refill(p)
                self.refills += 1
        else:
            if self.prop is not None:
                self.prop.free()
            self.prop = gp2s_assemble(self.x, p, self.precision, self.ctx)
            self.assemblies += 1
        return self.prop

    def run(self, n_sweeps: int, draws=None, seed: int = 0, callback=None) -> dict:
        """n_sweeps sweeps over the blocks. draws: per sweep, per block (normal offsets,
        uniform) as from workloads.mcmc_draws; drawn from numpy's PCG64(seed) in that
        layout when not given."""
        if draws is None:
            rng = np.random.default_rng(seed)
            draws = [[(rng.standard_normal(len(b)), float(rng.random())) for b in self.blocks]
                     for _ in range(n_sweeps)]
        chain, lmls, accepted, margins = [self.theta.copy()], [self.lml], [], []
        t0 = time.perf_counter()
        for k in range(n_sweeps):
            for idx, (eps, u) in zip(self.blocks, draws[k]):
                idx = np.asarray(idx)
                prop = self.theta.copy()
                prop[idx] = self.theta[idx] + self.steps[idx] * np.asarray(eps, dtype=np.float64)
                if np.any(prop[idx] <= self.lo[idx]) or np.any(prop[idx] >= self.hi[idx]):
                    accepted.append(False)
                    margins.append(None)
                    continue
                h = self._proposal_handle(prop)
                llp = self._lml(h)
                self.evals += 1
                margin = llp - self.lml - np.log(u)
                ok = margin > 0.0
                accepted.append(bool(ok))
                margins.append(margin)
                if ok:
                    self.theta, self.lml = prop, llp
                    self.cur, self.prop = self.prop, self.cur
            chain.append(self.theta.copy())
            lmls.append(self.lml)
            if callback:
                callback(k, self.theta, self.lml)
        return dict(chain=np.array(chain), lml=np.array(lmls), accepted=accepted, margins=margins,
                    seconds=time.perf_counter() - t0, evals=self.evals, refills=self.refills,
                    assemblies=self.assemblies)

    def free(self):
        for h in (self.cur, self.prop):
            if h is not None:
                h.free()
        self.cur = self.prop = None
