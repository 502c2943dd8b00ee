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
  for (int k = g.dim - 1; k >= 0; --k) b = b * g.nb[k] + bin_coord(xi[k], g.origin[k], g.inv_h, g.nb[k]);
  return b;
}

// g(x) = sum_k a_k exp(1 - 1/(1 - s_k)), s_k = ||x - c_k||^2 / w^2, over the bumps with
// s_k < 1 (Sec. 3.3, Eq. bump with shape parameter 1); `inside` marks a point strictly
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

// Wendland members (Sec. 3.1): kern 0 is the C^2 member (1 - rho)^4 (4 rho + 1), the
// workloads' "small variation"; kern 1 is the C^6 member of Eq. wendland as printed,
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

// Float32 entry value for a surviving off-diagonal pair.
__device__ inline float entry_f32(const float4& pi, const float4& pj, double r2, double inv_r2, int kern) {
  double dx = (double)pi.x - (double)pj.x;
  double dy = (double)pi.y - (double)pj.y;
  double dz = (double)pi.z - (double)pj.z;
  double d2 = dx * dx + dy * dy + dz * dz;
  float t = (float)((r2 - d2) * inv_r2);          // 1 - rho^2, accurate near rho -> 1
  t = fmaxf(t, 0.0f);
  float rho = __builtin_amdgcn_sqrtf((float)(d2 * inv_r2));
  float om = t * __builtin_amdgcn_rcpf(1.0f + rho);  // 1 - rho
  return pi.w * pj.w * wendland_w<float>(kern, rho, om);
}

__device__ inline double entry_f64(const double4& pi, const double4& pj, double r2, double inv_r2, int kern) {
  double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
  double d2 = dx * dx + dy * dy + dz * dz;
  double t = fmax((r2 - d2) * inv_r2, 0.0);
  double rho = sqrt(d2 * inv_r2);
  double om = t / (1.0 + rho);
  return pi.w * pj.w * wendland_w<double>(kern, rho, om);
}

}  // namespace gp2s
