"""Kernel pieces in float64: Wendland function, bump functions, the bump mask g.

Parity pinned by closed-form values, integrals and finite differences in
tests/test_oracle_kernel.py.
"""
from __future__ import annotations

import numpy as np


def wendland_c2(rho):
    """C^2 Wendland function W(rho) = (1 - rho)^4 (4 rho + 1) for rho < 1, else 0.

    Sec. 4.1: the paper prints the C^6 member (Eq. wendland) and uses "small
    variations thereof"; the workloads use this C^2 member. The support is strict
    (the equation's condition is ||x_i - x_j|| < r_0).
    """
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    inside = rho < 1.0
    q = 1.0 - rho[inside]
    out[inside] = q ** 4 * (4.0 * rho[inside] + 1.0)
    return out


def wendland_c2_dr(rho, r):
    """Derivative of W(d / r) with respect to the radius r, at rho = d / r.

    dW/drho = -20 rho (1 - rho)^3 and drho/dr = -rho / r, so the product is
    20 rho^2 (1 - rho)^3 / r inside the support and 0 outside.
    """
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    inside = rho < 1.0
    q = 1.0 - rho[inside]
    out[inside] = 20.0 * rho[inside] ** 2 * q ** 3 / r
    return out


def wendland_c6(rho):
    """The Wendland member printed in Sec. 4.1, Eq. wendland:
    (1 - rho)^8 (32 rho^3 + 25 rho^2 + 8 rho + 1) for rho < 1, else 0."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    inside = rho < 1.0
    p = rho[inside]
    out[inside] = (1.0 - p) ** 8 * (32.0 * p ** 3 + 25.0 * p ** 2 + 8.0 * p + 1.0)
    return out


def wendland_c6_dr(rho, r):
    """Derivative of the C^6 member W(d / r) (Eq. wendland) with respect to r, at rho = d / r.

    dW/drho = -22 rho (1 - rho)^7 (16 rho^2 + 7 rho + 1) (product rule on the printed
    form), drho/dr = -rho / r, so the product is 22 rho^2 (1 - rho)^7 (16 rho^2 + 7 rho
    + 1) / r inside the support and 0 outside.
    """
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    inside = rho < 1.0
    p = rho[inside]
    out[inside] = 22.0 * p ** 2 * (1.0 - p) ** 7 * (16.0 * p ** 2 + 7.0 * p + 1.0) / r
    return out


KERNELS = ("c2", "c6")


def wendland_dlog(rho, kernel="c2"):
    """D(rho) = -W'(rho) / rho inside the support (0 outside): 20 (1 - rho)^3 for the C^2
    member, 22 (1 - rho)^7 (16 rho^2 + 7 rho + 1) for the C^6 member. Finite at rho = 0;
    the radius derivative is D(rho) rho^2 / r."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    inside = rho < 1.0
    p = rho[inside]
    q = 1.0 - p
    if kernel == "c2":
        out[inside] = 20.0 * q ** 3
    elif kernel == "c6":
        out[inside] = 22.0 * q ** 7 * (16.0 * p * p + 7.0 * p + 1.0)
    else:
        raise ValueError(f"unknown Wendland member {kernel!r}")
    return out


def wendland(rho, kernel="c2"):
    """The Wendland member selected by `kernel`: "c2" (the workloads' member) or "c6"
    (Eq. wendland as printed)."""
    if kernel == "c2":
        return wendland_c2(rho)
    if kernel == "c6":
        return wendland_c6(rho)
    raise ValueError(f"unknown kernel {kernel!r}")


def wendland_dr(rho, r, kernel="c2"):
    """d/dr of the selected member at rho = d / r."""
    if kernel == "c2":
        return wendland_c2_dr(rho, r)
    if kernel == "c6":
        return wendland_c6_dr(rho, r)
    raise ValueError(f"unknown kernel {kernel!r}")


def kernel_params_check(dim, radius, bump_width, centers, weights, noise_var):
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, dim)
    weights = np.asarray(weights, dtype=np.float64).reshape(-1)
    if centers.shape[0] != weights.shape[0]:
        raise ValueError("centers and weights disagree on the bump count")
    if not (radius > 0 and bump_width > 0 and noise_var >= 0):
        raise ValueError("radius and bump width must be positive, noise variance >= 0")
    return centers, weights


def bump_values(x, centers, bump_width, weights, chunk=1 << 16):
    """Bump functions of Sec. 4.3, Eq. bump, and their weighted sum g.

    For bump k with centre c_k, width w and amplitude a_k (the weight), with the
    shape parameter beta fixed to 1:
        s_ik  = ||x_i - c_k||^2 / w^2
        b_ik  = exp(1 - 1 / (1 - s_ik))      if ||x_i - c_k||^2 < w^2, else 0
        g_i   = sum_k a_k b_ik               (g as a sum of P bumps, Sec. 4.3)
        gamma_i = [some bump has x_i strictly inside its support]
    The printed support condition compares a squared distance with r; it is read
    as the strict ball ||x - c_k|| < w, matching the r^2 inside the exponent.

    Returns (g, b, gamma) with b the unweighted bump values, shape (n, P).
    """
    x = np.asarray(x, dtype=np.float64)
    n, dim = x.shape
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, dim)
    weights = np.asarray(weights, dtype=np.float64).reshape(-1)
    P = centers.shape[0]
    w2 = float(bump_width) ** 2
    b = np.zeros((n, P))
    gamma = np.zeros(n, dtype=bool)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        diff = x[lo:hi, None, :] - centers[None, :, :]
        d2 = np.einsum("ipk,ipk->ip", diff, diff)
        inside = d2 < w2
        s = d2[inside] / w2
        blk = np.zeros((hi - lo, P))
        blk[inside] = np.exp(1.0 - 1.0 / (1.0 - s))
        b[lo:hi] = blk
        gamma[lo:hi] = inside.any(axis=1)
    g = b @ weights
    return g, b, gamma
