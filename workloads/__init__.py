"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no kernel values, no pair tests, no solves). Support radii
that must be tuned to a target row density are not computed here: they are read
from ``radii.json``, written by ``calibrate_radius.py`` (which calls the oracle).

Workload recipe (all coordinates are rounded to float32 and stored as float64,
so a float32 copy on the device is exact):

* ``c1``: N=4 000 points uniform in [0,1]^2, r=0.05, 4 bumps.
* ``c2``: N=200 000 points uniform in [0,1]^2, r=0.01, 8 bumps.
* ``c3``: N=2 000 000 points in [0,1]^3 from a 50-component Gaussian mixture
  (equal weights, means uniform, isotropic sd ~ U(0.02, 0.1), clamped to the
  cube), r calibrated for a mean of 100 stored entries per row, 16 bumps.
* ``c4``: N=10 000 000 points in [0,1]^2 from a 200-component mixture
  (sd ~ U(0.005, 0.05), clamped), r calibrated for 50 entries per row, 16 bumps.
* ``c5``: 64 independent instances, N ~ log-uniform on [5e3, 1e5], d in {2,3},
  uniform points, per-instance r calibrated to a target drawn from U(20,120).

Bump centres are uniform in the unit cube, bump weights U(0.5, 1.5), bump width
0.6; targets are y = f(x) + N(0, sd^2) with f(x) = sin(6 x1) cos(4 x2) in 2-D and
sin(6 x1) cos(4 x2) cos(3 x3) in 3-D; the noise variance on the diagonal is 1e-4
(c5: log-uniform on [1e-5, 1e-3], and the target noise sd is its square root).
The generator for config c and instance i is numpy's PCG64 seeded with 1000*c+i.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
RADII_FILE = os.path.join(_HERE, "radii.json")


@dataclass
class Problem:
    """One GP instance: points, targets and kernel hyperparameters (user order)."""

    name: str
    x: np.ndarray            # (n, dim) float64, float32-representable
    y: np.ndarray            # (n,) float64
    radius: float            # Wendland support radius r
    bump_width: float        # bump radius w
    centers: np.ndarray      # (P, dim) float64
    weights: np.ndarray      # (P,) float64
    noise_var: float         # diagonal noise variance
    n_probes: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def dim(self) -> int:
        return int(self.x.shape[1])

    @property
    def n_bumps(self) -> int:
        return int(self.weights.shape[0])

    def subsample(self, m: int, seed: int = 0) -> "Problem":
        """First m points of a seeded permutation (same hyperparameters)."""
        rng = np.random.default_rng(seed)
        idx = np.sort(rng.permutation(self.n)[:m])
        return Problem(self.name + f"_sub{m}", self.x[idx].copy(), self.y[idx].copy(),
                       self.radius, self.bump_width, self.centers.copy(),
                       self.weights.copy(), self.noise_var, self.n_probes,
                       dict(self.meta, subsample_of=self.name, subsample_seed=seed))


CONFIGS = {
    "c1": dict(cid=1, n=4000, dim=2, points="uniform", radius=0.05, n_bumps=4, n_probes=64),
    "c2": dict(cid=2, n=200_000, dim=2, points="uniform", radius=0.01, n_bumps=8, n_probes=64),
    "c3": dict(cid=3, n=2_000_000, dim=3, points="gmm", n_comp=50, sd=(0.02, 0.1),
               target_row=100.0, n_bumps=16, n_probes=32),
    "c4": dict(cid=4, n=10_000_000, dim=2, points="gmm", n_comp=200, sd=(0.005, 0.05),
               target_row=50.0, n_bumps=16, n_probes=64),
}
BUMP_WIDTH = 0.6
NOISE_VAR = 1e-4
NOISE_SD = 0.01


def f32(a: np.ndarray) -> np.ndarray:
    """Round to float32 and store as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def target_function(x: np.ndarray) -> np.ndarray:
    f = np.sin(6.0 * x[:, 0]) * np.cos(4.0 * x[:, 1])
    if x.shape[1] == 3:
        f = f * np.cos(3.0 * x[:, 2])
    return f


def uniform_points(rng: np.random.Generator, n: int, dim: int) -> np.ndarray:
    return f32(rng.random((n, dim)))


def gmm_points(rng: np.random.Generator, n: int, dim: int, n_comp: int, sd_range) -> np.ndarray:
    means = rng.random((n_comp, dim))
    sds = rng.uniform(sd_range[0], sd_range[1], size=n_comp)
    comp = rng.integers(0, n_comp, size=n)
    x = means[comp] + sds[comp, None] * rng.standard_normal((n, dim))
    np.clip(x, 0.0, 1.0, out=x)
    return f32(x)


def load_radii() -> dict:
    if not os.path.exists(RADII_FILE):
        return {}
    with open(RADII_FILE) as fh:
        return json.load(fh)


def make_points(name: str, n: int | None = None) -> np.ndarray:
    """Points only (used by the radius calibration)."""
    cfg = CONFIGS[name]
    rng = np.random.default_rng(1000 * cfg["cid"])
    n = cfg["n"] if n is None else n
    if cfg["points"] == "uniform":
        return uniform_points(rng, n, cfg["dim"])
    return gmm_points(rng, n, cfg["dim"], cfg["n_comp"], cfg["sd"])


def make_problem(name: str, n: int | None = None) -> Problem:
    """Config c1..c4 at its full size (or the first n draws of the same recipe)."""
    cfg = CONFIGS[name]
    rng = np.random.default_rng(1000 * cfg["cid"])
    n_full = cfg["n"]
    n = n_full if n is None else int(n)
    dim = cfg["dim"]
    if cfg["points"] == "uniform":
        x = uniform_points(rng, n, dim)
    else:
        x = gmm_points(rng, n, dim, cfg["n_comp"], cfg["sd"])
    if "radius" in cfg:
        radius = float(cfg["radius"])
    else:
        radii = load_radii()
        if name not in radii:
            raise KeyError(f"radius for {name} not calibrated; run workloads/calibrate_radius.py")
        radius = float(radii[name]["radius"])
    P = cfg["n_bumps"]
    centers = f32(rng.random((P, dim)))
    weights = rng.uniform(0.5, 1.5, size=P)
    y = target_function(x) + NOISE_SD * rng.standard_normal(n)
    return Problem(name, x, y, radius, BUMP_WIDTH, centers, weights, NOISE_VAR,
                   cfg["n_probes"], dict(cfg))


def make_random_problem(seed: int, n: int, dim: int, radius: float, n_bumps: int = 4,
                        bump_width: float = BUMP_WIDTH, noise_var: float = NOISE_VAR,
                        points: str = "uniform", n_probes: int = 8) -> Problem:
    """Small ad-hoc instance for tests (uniform or clustered points)."""
    rng = np.random.default_rng(seed)
    if points == "uniform":
        x = uniform_points(rng, n, dim)
    else:
        x = gmm_points(rng, n, dim, 8, (0.02, 0.08))
    centers = f32(rng.random((n_bumps, dim)))
    weights = rng.uniform(0.5, 1.5, size=n_bumps)
    y = target_function(x) + NOISE_SD * rng.standard_normal(n)
    return Problem(f"rand{seed}", x, y, float(radius), float(bump_width), centers, weights,
                   float(noise_var), n_probes, {})


C5_INSTANCES = 64


def c5_instance_specs():
    """Per-instance (n, dim, target row count, noise variance) for the batched config."""
    specs = []
    for i in range(C5_INSTANCES):
        rng = np.random.default_rng(5000 + i)
        n = int(round(np.exp(rng.uniform(np.log(5e3), np.log(1e5)))))
        dim = int(rng.integers(2, 4))
        target = float(rng.uniform(20.0, 120.0))
        noise_var = float(np.exp(rng.uniform(np.log(1e-5), np.log(1e-3))))
        specs.append(dict(n=n, dim=dim, target_row=target, noise_var=noise_var, seed=5000 + i))
    return specs


def c5_points(i: int) -> np.ndarray:
    spec = c5_instance_specs()[i]
    rng = np.random.default_rng(spec["seed"] + 100_000)
    return uniform_points(rng, spec["n"], spec["dim"])


def make_c5(max_instances: int | None = None) -> list[Problem]:
    radii = load_radii().get("c5")
    if radii is None:
        raise KeyError("radii for c5 not calibrated; run workloads/calibrate_radius.py")
    out = []
    specs = c5_instance_specs()
    for i, spec in enumerate(specs[:max_instances]):
        rng = np.random.default_rng(spec["seed"] + 100_000)
        x = uniform_points(rng, spec["n"], spec["dim"])
        P = 8
        centers = f32(rng.random((P, spec["dim"])))
        weights = rng.uniform(0.5, 1.5, size=P)
        y = target_function(x) + np.sqrt(spec["noise_var"]) * rng.standard_normal(spec["n"])
        out.append(Problem(f"c5_{i}", x, y, float(radii[i]), BUMP_WIDTH, centers, weights,
                           spec["noise_var"], 16, dict(spec)))
    return out


def mcmc_draws(seed: int, n_iter: int, block_sizes) -> list:
    """Seeded random inputs of a block Metropolis-Hastings run: for every iteration and
    block, the standard-normal proposal offsets (one per parameter of the block) and the
    uniform acceptance draw. Shared by the sampler and its oracle so that both take the
    same decisions; holds none of the sampler's arithmetic."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_iter):
        out.append([(rng.standard_normal(int(k)), float(rng.random())) for k in block_sizes])
    return out
