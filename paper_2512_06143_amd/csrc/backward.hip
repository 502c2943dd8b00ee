// Gradient of the log marginal likelihood with respect to theta = (r, a_1..a_P, sigma_n^2).
//
// dLML/dtheta = 1/2 a^T dK a - 1/2 tr(K^-1 dK), a = K^-1 y (Sec. 3 log density); the
// trace is estimated with the probe solutions q_s = K^-1 L z_s and w_s = L^-T z_s
// (M = L L^T the preconditioner: L = D^1/2, w_s recomputed from the signs, or the
// blockwise Cholesky factor, w_s read from memory) as (1/S) sum_s q_s^T dK w_s. With
// the symmetrised weight
//   P_ij = a_i a_j - (1/2S) sum_s (q_si w_sj + q_sj w_si)
// every component reduces to per-row sums over the stored pattern:
//   dK_ij/dr      = g_i g_j dW/dr,    dW/dr = 20 rho^2 (1 - rho)^3 / r for the C^2
//                                     member, 22 rho^2 (1 - rho)^7 (16 rho^2 + 7 rho + 1) / r for C^6
//   dK_ij/da_k    = (b_k(x_i) g_j + g_i b_k(x_j)) W_ij          (b_k: unweighted bump)
//   dK_ij/dsigma2 = [i == j]
//   R_i = sum_j g_j W_ij P_ij,  T_i = sum_j g_j dW/dr_ij P_ij,
//   U_i = sum_s q_si w_si,
//   dLML/dr = 1/2 sum_i g_i T_i,  dLML/da_k = sum_i b_k(x_i) R_i,
//   dLML/dsigma2 = 1/2 sum_i (a_i^2 - U_i / S).
// W and dW/dr are recomputed from the coordinates for every stored entry: no
// per-parameter matrix is ever formed.
#include "gp2s_internal.h"
#include "pair.h"

namespace gp2s {

__device__ inline double bcast64(double v, int l) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, l);
  p.y = __builtin_amdgcn_readlane(p.y, l);
  return __builtin_bit_cast(double, p);
}
__device__ inline float bcast32(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ inline uint64_t bcastu64(uint64_t v, int l) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__builtin_amdgcn_readlane((int)lo, l);
  hi = (uint32_t)__builtin_amdgcn_readlane((int)hi, l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// W and dW/dr for a stored pair of the float32-assembled path, evaluated in float64 from
// the float32 coordinates: the trace term sums q_i dK_ij w_j over terms that cancel
// heavily, so dK is not rounded to float32 here (one pass per gradient; the float32
// values are the CG operator's business only).
__device__ inline void w_dw_mixed(const float4& pi, const float4& pj, double r2, double inv_r2, double inv_r,
                                  int kern, double& W, double& dW) {
  double dx = (double)pi.x - (double)pj.x;
  double dy = (double)pi.y - (double)pj.y;
  double dz = (double)pi.z - (double)pj.z;
  double d2 = dx * dx + dy * dy + dz * dz;
  double t = fmax((r2 - d2) * inv_r2, 0.0);
  double rho = sqrt(d2 * inv_r2);
  double om = t / (1.0 + rho);
  wendland_w_dr<double>(kern, rho, om, inv_r, W, dW);
}
__device__ inline void w_dw_f64(const double4& pi, const double4& pj, double r2, double inv_r2, double inv_r, int kern,
                                double& W, double& dW) {
  double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
  double d2 = dx * dx + dy * dy + dz * dz;
  double t = fmax((r2 - d2) * inv_r2, 0.0);
  double rho = sqrt(d2 * inv_r2);
  double om = t / (1.0 + rho);
  wendland_w_dr<double>(kern, rho, om, inv_r, W, dW);
}

template <bool F32>
__global__ __launch_bounds__(kBlock) void k_backward_rows(BackwardArgs b, double* __restrict__ Rrow,
                                                          double* __restrict__ Trow,
                                                          double* __restrict__ Urow) {
  const int lane = threadIdx.x & (kWave - 1);
  const XcdRows rr = xcd_rows(b.n, threadIdx.x / kWave, kBlock / kWave);
  const int S = b.S;
  const bool active = lane < S;
  const double inv_r = 1.0 / b.radius;
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    float4 pi32;
    double4 pi64;
    if (F32) pi32 = b.pts32[row];
    else pi64 = b.pts64[row];
    const double ai = b.a[row];
    const uint64_t mi = b.mask[row];
    const double dsi = sqrt(b.dinv[row]);
    const double qi = active ? b.Q[row * S + lane] : 0.0;
    const double wi = !active ? 0.0 : b.W ? b.W[row * S + lane] : (((mi >> lane) & 1ull) ? -dsi : dsi);
    double accR = 0.0, accT = 0.0, aR = 0.0, aT = 0.0;
    const int64_t s0 = b.rp[row], e0 = b.rp[row + 1];
    for (int64_t k0 = s0; k0 < e0; k0 += kWave) {
      const int64_t k = k0 + lane;
      const bool valid = k < e0;
      const int32_t j = valid ? b.col[k] : (int32_t)row;
      double gW = 0.0, gWp = 0.0;
      if (valid) {
        if (F32) {
          double W, dW;
          w_dw_mixed(pi32, b.pts32[j], b.r2, b.inv_r2, inv_r, b.kern, W, dW);
          const double gj = b.g64[j];
          gW = gj * W;
          gWp = gj * dW;
        } else {
          const double4 pj = b.pts64[j];
          double W, dW;
          w_dw_f64(pi64, pj, b.r2, b.inv_r2, inv_r, b.kern, W, dW);
          const double gj = pt_g(pj.w);
          gW = gj * W;
          gWp = gj * dW;
        }
        const double aj = b.a[j];
        aR += gW * aj;
        aT += gWp * aj;
      }
      const uint64_t mj = valid ? b.mask[j] : 0ull;
      const double dsj = valid ? sqrt(b.dinv[j]) : 0.0;
      const int cnt = (int)((e0 - k0) < kWave ? (e0 - k0) : kWave);
      for (int l = 0; l < cnt; ++l) {
        const int32_t jj = __builtin_amdgcn_readlane(j, l);
        const double gw = bcast64(gW, l);
        const double gwp = bcast64(gWp, l);
        const uint64_t mm = bcastu64(mj, l);
        const double ds = bcast64(dsj, l);
        if (active) {
          const double qj = b.Q[(int64_t)jj * S + lane];
          const double wj = b.W ? b.W[(int64_t)jj * S + lane] : (((mm >> lane) & 1ull) ? -ds : ds);
          const double c = qi * wj + qj * wi;
          accR += gw * c;
          accT += gwp * c;
        }
      }
    }
    const double sR = wave_sum(aR), sT = wave_sum(aT);
    const double pR = wave_sum(accR), pT = wave_sum(accT);
    const double U = wave_sum(qi * wi);
    if (lane == 0) {
      const double inv2S = 0.5 / (double)S;
      Rrow[row] = ai * sR - inv2S * pR;
      Trow[row] = ai * sT - inv2S * pT;
      Urow[row] = U;
    }
  }
}

// General kernel (Eq. wendconv with axis radii r_k and the length-scale field l): per
// row, with p, Q, m, W and D(rho) = -W'(rho)/rho of the pair (pair.h gen_geom),
//   R_i  = sum_j g_j p_ij W_ij P_ij                                     (amplitudes)
//   T_ik = sum_j g_j p_ij D_ij ((x_ik - x_jk)/r_k)^2 / (r_k m_ij) P_ij    (axis radius k;
//          one isotropic radius: sum_j g_j p_ij D_ij Q_ij / r P_ij)
//   V_i  = sum_j g_j E_ij P_ij,  E_ij = p_ij [(d/2)(1 - l_i^2/m_ij) W_ij + D_ij Q_ij l_i^2/(2 m_ij)]
//          = d(p W)/d ln l_i                                            (length-scale weights)
//   U_i  as above; dLML/dr_k = 1/2 sum_i g_i T_ik, dLML/dc_q = sum_i bhat_q(x_i) g_i V_i.
// Everything in float64 (the float32 path's coordinates promoted).
template <int DIM, bool F32>
__global__ __launch_bounds__(kBlock) void k_backward_gen(BackwardArgs b, double* __restrict__ Rrow,
                                                         double* __restrict__ Trow, double* __restrict__ Urow,
                                                         double* __restrict__ Vrow) {
  const int lane = threadIdx.x & (kWave - 1);
  const XcdRows rr = xcd_rows(b.n, threadIdx.x / kWave, kBlock / kWave);
  const int S = b.S;
  const bool active = lane < S;
  const int nr = b.nr;
  const bool ls = b.kg.lsq != nullptr;
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    double xi, yi, zi;
    if (F32) {
      const float4 v = b.pts32[row];
      xi = v.x, yi = v.y, zi = v.z;
    } else {
      const double4 v = b.pts64[row];
      xi = v.x, yi = v.y, zi = v.z;
    }
    const double li = ls ? b.kg.lsq[row] : 1.0;
    const double ai = b.a[row];
    const uint64_t mi = b.mask[row];
    const double dsi = sqrt(b.dinv[row]);
    const double qi = active ? b.Q[row * S + lane] : 0.0;
    const double wi = !active ? 0.0 : b.W ? b.W[row * S + lane] : (((mi >> lane) & 1ull) ? -dsi : dsi);
    double accR = 0.0, accV = 0.0, aR = 0.0, aV = 0.0;
    double accT[DIM], aT[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) accT[k] = aT[k] = 0.0;
    const int64_t s0 = b.rp[row], e0 = b.rp[row + 1];
    for (int64_t k0 = s0; k0 < e0; k0 += kWave) {
      const int64_t k = k0 + lane;
      const bool valid = k < e0;
      const int32_t j = valid ? b.col[k] : (int32_t)row;
      double gW = 0.0, gE = 0.0, gT[DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) gT[c] = 0.0;
      if (valid) {
        double xj, yj, zj;
        if (F32) {
          const float4 v = b.pts32[j];
          xj = v.x, yj = v.y, zj = v.z;
        } else {
          const double4 v = b.pts64[j];
          xj = v.x, yj = v.y, zj = v.z;
        }
        const double lj = ls ? b.kg.lsq[j] : 1.0;
        double ds[3], m, t, Q, p;
        gen_geom<DIM>(xi, yi, zi, xj, yj, zj, b.kg, li, lj, ds, m, t, Q, p);
        const double rho = sqrt(Q), om = t / (1.0 + rho);
        const double W = wendland_w<double>(b.kern, rho, om), D = wendland_dlog<double>(b.kern, rho, om);
        const double gj = b.g64[j];
        gW = gj * p * W;
        if (nr == 1) {
          gT[0] = gj * p * D * Q * b.kg.inv_r[0];
        } else {
#pragma unroll
          for (int c = 0; c < DIM; ++c) gT[c] = gj * p * D * ds[c] * b.kg.inv_r[c] / m;
        }
        if (ls) gE = gj * p * (0.5 * DIM * (1.0 - li / m) * W + D * Q * li / (2.0 * m));
        const double aj = b.a[j];
        aR += gW * aj;
        aV += gE * aj;
#pragma unroll
        for (int c = 0; c < DIM; ++c) aT[c] += gT[c] * aj;
      }
      const uint64_t mj = valid ? b.mask[j] : 0ull;
      const double dsj = valid ? sqrt(b.dinv[j]) : 0.0;
      const int cnt = (int)((e0 - k0) < kWave ? (e0 - k0) : kWave);
      for (int l = 0; l < cnt; ++l) {
        const int32_t jj = __builtin_amdgcn_readlane(j, l);
        const double gw = bcast64(gW, l), ge = bcast64(gE, l);
        double gt[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) gt[c] = bcast64(gT[c], l);
        const uint64_t mm = bcastu64(mj, l);
        const double ds = bcast64(dsj, l);
        if (active) {
          const double qj = b.Q[(int64_t)jj * S + lane];
          const double wj = b.W ? b.W[(int64_t)jj * S + lane] : (((mm >> lane) & 1ull) ? -ds : ds);
          const double c = qi * wj + qj * wi;
          accR += gw * c;
          accV += ge * c;
#pragma unroll
          for (int q = 0; q < DIM; ++q) accT[q] += gt[q] * c;
        }
      }
    }
    const double inv2S = 0.5 / (double)S;
    const double sR = wave_sum(aR), pR = wave_sum(accR);
    const double sV = wave_sum(aV), pV = wave_sum(accV);
    const double U = wave_sum(qi * wi);
    double sT[DIM], pT[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      sT[c] = wave_sum(aT[c]);
      pT[c] = wave_sum(accT[c]);
    }
    if (lane == 0) {
      Rrow[row] = ai * sR - inv2S * pR;
      for (int c = 0; c < nr; ++c) Trow[(int64_t)c * b.n + row] = ai * sT[c] - inv2S * pT[c];
      Urow[row] = U;
      if (Vrow) Vrow[row] = ai * sV - inv2S * pV;
    }
  }
}

hipError_t launch_backward_rows(const BackwardArgs& b, int prec, double* Rrow, double* Trow, double* Urow,
                                double* Vrow, hipStream_t st) {
  int64_t blocks = (b.n + (kBlock / kWave) - 1) / (kBlock / kWave);
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) return hipSuccess;
  blocks = round_up8(blocks);
  const dim3 g((unsigned)blocks), t(kBlock);
  if (b.kg.general) {
    if (b.dim == 3) {
      if (prec == GP2S_MIXED) hipLaunchKernelGGL((k_backward_gen<3, true>), g, t, 0, st, b, Rrow, Trow, Urow, Vrow);
      else hipLaunchKernelGGL((k_backward_gen<3, false>), g, t, 0, st, b, Rrow, Trow, Urow, Vrow);
    } else {
      if (prec == GP2S_MIXED) hipLaunchKernelGGL((k_backward_gen<2, true>), g, t, 0, st, b, Rrow, Trow, Urow, Vrow);
      else hipLaunchKernelGGL((k_backward_gen<2, false>), g, t, 0, st, b, Rrow, Trow, Urow, Vrow);
    }
  } else if (prec == GP2S_MIXED) {
    hipLaunchKernelGGL(k_backward_rows<true>, g, t, 0, st, b, Rrow, Trow, Urow);
  } else {
    hipLaunchKernelGGL(k_backward_rows<false>, g, t, 0, st, b, Rrow, Trow, Urow);
  }
  return hipGetLastError();
}

// Per-point reduction to the gradient components (bump values recomputed in float64
// from the coordinates, as in the prologue): nr radius components, P amplitudes, P
// length-scale weights when Vrow is given, the noise variance. Deterministic two-level
// sum.
constexpr int kGradChunk = 16;

__global__ __launch_bounds__(kBlock) void k_grad_reduce(int64_t n, int dim, int P, int S, int nr,
                                                        const double* __restrict__ x64,
                                                        const double* __restrict__ g64,
                                                        const double* __restrict__ a,
                                                        const double* __restrict__ Rrow,
                                                        const double* __restrict__ Trow,
                                                        const double* __restrict__ Urow,
                                                        const double* __restrict__ Vrow,
                                                        const double* __restrict__ Hrow,
                                                        const int32_t* __restrict__ group, int U,
                                                        const double* __restrict__ centers,
                                                        double bump_w2, double* __restrict__ partial,
                                                        uint32_t* __restrict__ ticket,
                                                        double* __restrict__ grad) {
  __shared__ double sh[kBlock];
  __shared__ int am_last;
  const int nc = Vrow ? P : 0;
  const int ncomp = nr + P + nc + 1;
  // radius and noise components
  double cr = 0.0, cr1 = 0.0, cr2 = 0.0, cs2 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    cr += 0.5 * g64[i] * Trow[i];
    if (nr > 1) cr1 += 0.5 * g64[i] * Trow[n + i];
    if (nr > 2) cr2 += 0.5 * g64[i] * Trow[2 * n + i];
    cs2 += 0.5 * (a[i] * a[i] - Urow[i] / (double)S);
  }
  auto block_sum = [&](double v) -> double {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    double t = sh[0];
    __syncthreads();
    return t;
  };
  double t = block_sum(cr);
  if (threadIdx.x == 0) partial[blockIdx.x * (int64_t)ncomp + 0] = t;
  if (nr > 1) {
    t = block_sum(cr1);
    if (threadIdx.x == 0) partial[blockIdx.x * (int64_t)ncomp + 1] = t;
  }
  if (nr > 2) {
    t = block_sum(cr2);
    if (threadIdx.x == 0) partial[blockIdx.x * (int64_t)ncomp + 2] = t;
  }
  t = block_sum(cs2);
  if (threadIdx.x == 0) partial[blockIdx.x * (int64_t)ncomp + ncomp - 1] = t;
  for (int k0 = 0; k0 < P; k0 += kGradChunk) {
    double acc[kGradChunk], accc[kGradChunk];
#pragma unroll
    for (int q = 0; q < kGradChunk; ++q) acc[q] = accc[q] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const double R = Rrow[i];
      const double GV = Vrow ? g64[i] * Vrow[i] : 0.0;
#pragma unroll
      for (int q = 0; q < kGradChunk; ++q) {
        const int k = k0 + q;
        if (k < P) {
          double d2 = 0.0;
          for (int c = 0; c < dim; ++c) {
            const double d = x64[i * dim + c] - centers[k * dim + c];
            d2 += d * d;
          }
          if (d2 < bump_w2) {
            const double bk = exp(1.0 - 1.0 / (1.0 - d2 / bump_w2));
            acc[q] += bk * (Hrow ? Hrow[i * U + group[k]] : R);
            accc[q] += bk * GV;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kGradChunk; ++q) {
      if (k0 + q < P) {
        double v = block_sum(acc[q]);
        if (threadIdx.x == 0) partial[blockIdx.x * (int64_t)ncomp + nr + k0 + q] = v;
        if (Vrow) {
          v = block_sum(accc[q]);
          if (threadIdx.x == 0) partial[blockIdx.x * (int64_t)ncomp + nr + P + k0 + q] = v;
        }
      }
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) am_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  for (int c = threadIdx.x; c < ncomp; c += blockDim.x) {
    double v = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) v += partial[b * (int64_t)ncomp + c];
    grad[c] = v;
  }
  if (threadIdx.x == 0) *ticket = 0u;
}

hipError_t launch_grad_reduce(int64_t n, int dim, int P, int S, int nr, const double* x64, const double* g64,
                              const double* a, const double* Rrow, const double* Trow, const double* Urow,
                              const double* Vrow, const double* Hrow, const int32_t* group, int U,
                              const double* centers, double bump_w2, double* partial,
                              uint32_t* ticket, double* grad, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, dim, P, S, nr, x64, g64, a,
                     Rrow, Trow, Urow, Vrow, Hrow, group, U, centers, bump_w2, partial, ticket, grad);
  return hipGetLastError();
}

}  // namespace gp2s
