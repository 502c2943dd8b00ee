"""Find the Wendland radius r for the workloads whose row density is specified
rather than their radius, and store it in radii.json.

Bisection (on log r) until the mean number of points within r of a point,
itself included, is within 0.5% of the target; counts come from the oracle's
k-d tree pair count. Run once: `python workloads/calibrate_radius.py [c3 c4 c5]`.
"""
from __future__ import annotations

import json
import math
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
import workloads  # noqa: E402


def bisect_radius(x, target, r0, rel=0.005, max_steps=40):
    dim = x.shape[1]
    lo, hi = r0 / 2.0, r0 * 2.0
    while oracle.mean_row_count(x, lo) > target:
        lo /= 2.0
    while oracle.mean_row_count(x, hi) < target:
        hi *= 2.0
    r, m = r0, None
    for _ in range(max_steps):
        r = math.sqrt(lo * hi)
        m = oracle.mean_row_count(x, r)
        if abs(m - target) <= rel * target:
            break
        if m < target:
            lo = r
        else:
            hi = r
    return r, m


def main(names):
    radii = workloads.load_radii()
    for name in names:
        if name == "c5":
            out = []
            for i, spec in enumerate(workloads.c5_instance_specs()):
                x = workloads.c5_points(i)
                n, dim = x.shape
                r0 = (spec["target_row"] / n / (math.pi if dim == 2 else 4 * math.pi / 3)) ** (1 / dim)
                r, m = bisect_radius(x, spec["target_row"], r0)
                out.append(r)
                print(f"c5[{i}] n={n} d={dim} target={spec['target_row']:.1f} r={r:.6g} mean={m:.2f}",
                      flush=True)
            radii["c5"] = out
        else:
            cfg = workloads.CONFIGS[name]
            x = workloads.make_points(name)
            n, dim = x.shape
            r0 = (cfg["target_row"] / n / (math.pi if dim == 2 else 4 * math.pi / 3)) ** (1 / dim)
            r, m = bisect_radius(x, cfg["target_row"], r0)
            radii[name] = dict(radius=r, mean_row=m, target_row=cfg["target_row"], n=n)
            print(f"{name}: r={r:.6g} mean={m:.3f}", flush=True)
        with open(workloads.RADII_FILE, "w") as fh:
            json.dump(radii, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c3", "c4", "c5"])
