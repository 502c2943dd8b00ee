"""Block Metropolis-Hastings training of the kernel hyperparameters (Sec. 3.5; App. D)
on the library's LML.

theta = (r, a_1..a_P, sigma_n^2). Every sweep visits the blocks in order (by default
the Wendland radius, the bump amplitudes and the noise variance, each its own block,
as App. D separates the core-kernel block from the bump blocks); a block move draws a
normal random-walk proposal for its components (App. D keeps proposals normal), a flat
prior restricts theta to bounds (App. D), and the move is accepted when
log u < LML(theta') - LML(theta). Each block costs one LML evaluation (Sec. 3.5).

The LML is the library's estimate with a fixed probe seed, so every evaluation uses
the same probes (common random numbers across proposals). Moves that keep r reuse the
stored pattern (gp2s_matrix_refill: no count pass, no CSR allocation); moves of r
assemble a new handle. Only argument marshalling happens here; every evaluation runs
in the HIP kernels.
"""
from __future__ import annotations

import time
from dataclasses import replace

import numpy as np

from .gp2s import HostParams, Matrix, _as_dev64, default_context, default_opts, gp2s_assemble, gp2s_lml


def theta_of(p: HostParams) -> np.ndarray:
    return np.concatenate([[p.radius], np.asarray(p.weights, dtype=np.float64), [p.noise_var]])


def params_of(base: HostParams, theta: np.ndarray) -> HostParams:
    P = len(np.asarray(base.weights))
    return replace(base, radius=float(theta[0]), weights=np.array(theta[1:P + 1], dtype=np.float64),
                   noise_var=float(theta[P + 1]))


class BlockMH:
    """Sampler state: the data, the current theta and its LML, and two matrix handles
    (the current state's and a proposal's)."""

    def __init__(self, x, y, params: HostParams, precision="mixed", opts=None, blocks=None, steps=None,
                 bounds=None, ctx=None):
        self.ctx = ctx or default_context()
        self.x, self.y = _as_dev64(x, self.ctx), _as_dev64(y, self.ctx)  # device-resident once
        self.base, self.precision = params, precision
        self.opts = opts or default_opts()
        P = len(np.asarray(params.weights))
        self.blocks = blocks or [[0], list(range(1, P + 1)), [P + 1]]
        self.theta = theta_of(params)
        self.steps = np.asarray(steps if steps is not None else 0.05 * self.theta, dtype=np.float64)
        lo, hi = bounds if bounds is not None else (self.theta / 10.0, self.theta * 10.0)
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

    def _proposal_handle(self, theta: np.ndarray) -> Matrix:
        p = params_of(self.base, theta)
        if theta[0] == self.theta[0]:
            # same radius and geometry: refill a handle that holds the current pattern
            if self.prop is None or self.prop.params.radius != self.theta[0]:
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
