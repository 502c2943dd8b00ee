// Device helpers shared by the training assembly and the test-point (posterior)
// cross-covariance: bins, the bump mask, the support test and the entry value. One
// definition keeps a test point that coincides with a training point bitwise
// identical to it.
#pragma once

#include "gp2s_internal.h"

namespace gp2s {

__device__ inline int32_t bin_coord(double v, double o, double inv_h, int32_t nb) {
  double f = floor((v - o) * inv_h);
  int32_t c = (int32_t)fmax(0.0, fmin(f, (double)(nb - 1)));
  return c;
}

// Bin of a point (coordinates beyond the grid are clamped to its edge bins, which
// still holds every point within r of them).
__device__ inline int64_t bin_index(const double (&xi)[3], const GridDev& g) {
  int64_t b = 0;
  for (int k = g.dim - 1; k >= 0; --k) b = b * g.nb[k] + bin_coord(xi[k], g.origin[k], g.inv_h[k], g.nb[k]);
  return b;
}

// g(x) = sum_k a_k exp(1 - 1/(1 - s_k)), s_k = ||x - c_k||^2 / w^2, over the bumps with
// s_k < 1 (Sec. 4.3, Eq. bump with shape parameter 1); `inside` marks a point strictly
// inside at least one bump.
__device__ inline void bump_mask(const double (&xi)[3], int dim, const double* __restrict__ centers,
                                 const double* __restrict__ weights, int P, double bump_w2, double& gsum,
                                 bool& inside) {
  gsum = 0.0;
  inside = false;
  for (int p = 0; p < P; ++p) {
    double d2 = 0.0;
    for (int k = 0; k < dim; ++k) {
      double d = xi[k] - centers[p * dim + k];
      d2 += d * d;
    }
    if (d2 < bump_w2) {
      inside = true;
      double s = d2 / bump_w2;
      gsum += weights[p] * exp(1.0 - 1.0 / (1.0 - s));
    }
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that consecutive
// rows (which share neighbour bins) land on the same XCD and its L2.
__device__ inline int64_t xcd_block(int64_t nblocks_padded) {
  int64_t b = blockIdx.x;
  int64_t per = nblocks_padded / 8;
  return (b % 8) * per + b / 8;
}

__device__ inline uint32_t lane_prefix(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int DIM>
__device__ inline void decode_bin(int32_t b, const GridDev& g, int& bx, int& by, int& bz) {
  bx = b % g.nb[0];
  int t = b / g.nb[0];
  if (DIM == 3) {
    by = t % g.nb[1];
    bz = t / g.nb[1];
  } else {
    by = t;
    bz = 0;
  }
}

// Squared distances for the support test. Explicit rounding intrinsics fix the
// evaluation order, so the count pass and the fill pass (separate instantiations)
// take bitwise the same decision, and K stays symmetric: swapping i and j only
// negates the differences.
template <int DIM>
__device__ inline float sqdist_f32(const float4& a, const float4& b) {
  const float dx = a.x - b.x, dy = a.y - b.y;
  float d2 = __fmaf_rn(dy, dy, __fmul_rn(dx, dx));
  if (DIM == 3) {
    const float dz = a.z - b.z;
    d2 = __fmaf_rn(dz, dz, d2);
  }
  return d2;
}
template <int DIM>
__device__ inline double sqdist_f64(const double4& a, const double4& b) {
  const double dx = a.x - b.x, dy = a.y - b.y;
  double d2 = __fma_rn(dy, dy, __dmul_rn(dx, dx));
  if (DIM == 3) {
    const double dz = a.z - b.z;
    d2 = __fma_rn(dz, dz, d2);
  }
  return d2;
}

// Wendland members (Sec. 4.1): kern 0 is the C^2 member (1 - rho)^4 (4 rho + 1), the
// variant the workloads use; kern 1 is the C^6 member of Eq. wendland as printed,
// (1 - rho)^8 (32 rho^3 + 25 rho^2 + 8 rho + 1). om = 1 - rho is passed in, formed
// from 1 - rho^2 without cancellation near the support boundary.
template <typename T>
__device__ inline T wendland_w(int kern, T rho, T om) {
  const T om2 = om * om, om4 = om2 * om2;
  if (kern == 1) return om4 * om4 * ((((T)32 * rho + (T)25) * rho + (T)8) * rho + (T)1);
  return om4 * ((T)4 * rho + (T)1);
}
// W and its derivative in the radius at rho = d / r: dW/dr = -(rho / r) dW/drho, i.e.
// 20 rho^2 (1 - rho)^3 / r (C^2) and 22 rho^2 (1 - rho)^7 (16 rho^2 + 7 rho + 1) / r (C^6).
template <typename T>
__device__ inline void wendland_w_dr(int kern, T rho, T om, T inv_r, T& W, T& dW) {
  const T om2 = om * om, om4 = om2 * om2;
  if (kern == 1) {
    W = om4 * om4 * ((((T)32 * rho + (T)25) * rho + (T)8) * rho + (T)1);
    dW = (T)22 * rho * rho * om4 * om2 * om * (((T)16 * rho + (T)7) * rho + (T)1) * inv_r;
  } else {
    W = om4 * ((T)4 * rho + (T)1);
    dW = (T)20 * rho * rho * om2 * om * inv_r;
  }
}

__device__ inline double entry_f64(const double4& pi, const double4& pj, double r2, double inv_r2, int kern) {
  double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
  double d2 = dx * dx + dy * dy + dz * dz;
  double t = fmax((r2 - d2) * inv_r2, 0.0);
  double rho = sqrt(d2 * inv_r2);
  double om = t / (1.0 + rho);
  return pi.w * pj.w * wendland_w<double>(kern, rho, om);
}

__device__ inline double4 promote(const float4& p) { return make_double4(p.x, p.y, p.z, p.w); }

// Float32-stored entry value of a surviving off-diagonal pair: the float64 evaluation
// from the float32 coordinates and g, rounded once. Rounding after each float32 step
// (square root, reciprocal, polynomial) left entry errors of ~14 ulp; summed over the
// thousands of entries of a row inside dense clusters they moved the smallest
// eigenvalue of the stored matrix below zero (measured on the densest regions of a
// 10 M-point clustered cloud: -7.5e-5 against sigma_n^2 = 1e-4), while one rounding
// per entry kept it at 0.91 sigma_n^2. The support test stays in float32.
// In float64, 1 - rho = 1 - sqrt(rho^2) is accurate to ~2e-16 absolute, so W's relative
// error, about 8e-16 / (1 - rho), stays below the float32 rounding (6e-8) wherever
// 1 - rho > 1.3e-8 (W > 1.4e-31): the division of the float64 path's t / (1 + rho) is
// not needed for a float32-stored value.
__device__ inline float entry_f32(const float4& pi, const float4& pj, double r2, double inv_r2, int kern) {
  const double dx = (double)pi.x - (double)pj.x, dy = (double)pi.y - (double)pj.y, dz = (double)pi.z - (double)pj.z;
  const double d2 = dx * dx + dy * dy + dz * dz;
  const double rho = sqrt(d2 * inv_r2);
  const double om = fmax(1.0 - rho, 0.0);
  return (float)((double)pi.w * (double)pj.w * wendland_w<double>(kern, rho, om));
}

// ---- general kernel (Eq. wendconv with axis radii and the length-scale field) ------
// li, lj are l(x)^2 of the two points (1 without the field).

// Support test: sum_k ((x_ik - x_jk) / r_k)^2 < m_ij, in float32 with fixed rounding
// (symmetric in i, j: the differences only change sign).
template <int DIM>
__device__ inline bool gen_pass_f32(const float4& a, const float4& b, const KernGeom& kg, double li, double lj) {
  const float dx = __fmul_rn(a.x - b.x, kg.inv_rf[0]), dy = __fmul_rn(a.y - b.y, kg.inv_rf[1]);
  float d2 = __fmaf_rn(dy, dy, __fmul_rn(dx, dx));
  if (DIM == 3) {
    const float dz = __fmul_rn(a.z - b.z, kg.inv_rf[2]);
    d2 = __fmaf_rn(dz, dz, d2);
  }
  const float m = kg.lsq ? __fmul_rn(0.5f, __fadd_rn((float)li, (float)lj)) : 1.0f;
  return d2 < m;
}
template <int DIM>
__device__ inline bool gen_pass_f64(const double4& a, const double4& b, const KernGeom& kg, double li, double lj) {
  const double dx = __dmul_rn(a.x - b.x, kg.inv_r[0]), dy = __dmul_rn(a.y - b.y, kg.inv_r[1]);
  double d2 = __fma_rn(dy, dy, __dmul_rn(dx, dx));
  if (DIM == 3) {
    const double dz = __dmul_rn(a.z - b.z, kg.inv_r[2]);
    d2 = __fma_rn(dz, dz, d2);
  }
  const double m = kg.lsq ? __dmul_rn(0.5, __dadd_rn(li, lj)) : 1.0;
  return d2 < m;
}

// Float64 geometry of a stored pair: scaled squared differences ds[k], m, t = 1 - Q
// (formed as (m - d) / m, accurate near the support boundary), Q = d / m, and the
// prefactor p = (l_i l_j / m)^{DIM/2}.
template <int DIM>
__device__ inline void gen_geom(double ax, double ay, double az, double bx, double by, double bz, const KernGeom& kg,
                                double li, double lj, double (&ds)[3], double& m, double& t, double& Q, double& p) {
  const double dx = (ax - bx) * kg.inv_r[0], dy = (ay - by) * kg.inv_r[1], dz = DIM == 3 ? (az - bz) * kg.inv_r[2] : 0.0;
  ds[0] = dx * dx;
  ds[1] = dy * dy;
  ds[2] = dz * dz;
  const double d2 = ds[0] + ds[1] + ds[2];
  m = kg.lsq ? 0.5 * (li + lj) : 1.0;
  t = fmax((m - d2) / m, 0.0);
  Q = d2 / m;
  p = 1.0;
  if (kg.lsq) {
    const double q = sqrt(li * lj) / m;
    p = DIM == 3 ? q * sqrt(q) : q;
  }
}

template <int DIM>
__device__ inline double gen_entry_f64(const double4& pi, const double4& pj, const KernGeom& kg, double li, double lj,
                                       int kern) {
  double ds[3], m, t, Q, p;
  gen_geom<DIM>(pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, kg, li, lj, ds, m, t, Q, p);
  const double rho = sqrt(Q);
  const double om = t / (1.0 + rho);
  return pi.w * pj.w * p * wendland_w<double>(kern, rho, om);
}

// Float32-stored value of the general kernel: float64 evaluation, one rounding (as
// entry_f32).
template <int DIM>
__device__ inline float gen_entry_f32(const float4& pi, const float4& pj, const KernGeom& kg, double li, double lj,
                                      int kern) {
  return (float)gen_entry_f64<DIM>(promote(pi), promote(pj), kg, li, lj, kern);
}

// D(rho) = -W'(rho) / rho: 20 (1 - rho)^3 (C^2), 22 (1 - rho)^7 (16 rho^2 + 7 rho + 1) (C^6).
template <typename T>
__device__ inline T wendland_dlog(int kern, T rho, T om) {
  const T om2 = om * om, om3 = om2 * om;
  if (kern == 1) return (T)22 * om3 * om3 * om * (((T)16 * rho + (T)7) * rho + (T)1);
  return (T)20 * om3;
}

}  // namespace gp2s
