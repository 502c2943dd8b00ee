// CSR products with the assembled covariance: single right-hand side (vector CSR,
// a group of G lanes per row) and blocks of up to 64 right-hand sides (one wave per
// row, one lane per column). These drive the solve K a = y and the probe solves of
// the log-determinant (Sec. 3.5; App. B.6 "MINRES", "LOGDET"). Stored values
// (float32 or float64) multiply float64 vectors and accumulate in float64.
//
// The CG variants also produce p^T q per column from fixed per-workgroup partial
// sums; the last workgroup to finish (ticket counter) reduces them in workgroup
// order, so results are bitwise reproducible.
#include "gp2s_internal.h"

namespace gp2s {

template <typename V>
__device__ inline double ld(const V* p, int64_t k) {
  return (double)p[k];
}

// ---- single right-hand side -----------------------------------------------------------
template <int G, typename V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv(const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const V* __restrict__ val, int64_t n,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y, CgState cs) {
  const int lane = threadIdx.x & (G - 1);
  const int64_t group = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / G;
  double dot = 0.0;
  for (int64_t row = group; row < n; row += ngroups) {
    const int64_t s = rp[row], e = rp[row + 1];
    double acc = 0.0;
    for (int64_t k = s + lane; k < e; k += G) acc += ld(val, k) * x[col[k]];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (lane == 0) {
      y[row] = acc;
      if (DOT) dot += acc * x[row];
    }
  }
  if (!DOT) return;
  // p^T q partial of this workgroup, then alpha in the last workgroup.
  __shared__ double sh[kBlock];
  __shared__ int am_last;
  sh[threadIdx.x] = dot;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cs.partial[blockIdx.x] = sh[0];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) am_last = atomicAdd(&cs.ticket[0], 1u) == gridDim.x - 1;
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  if (threadIdx.x == 0) {
    double pq = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) pq += cs.partial[b];
    double a = 0.0;
    if (!cs.done[0]) {
      if (!(pq > 0.0) || !isfinite(pq)) {
        cs.flags[0] = 1;
      } else {
        a = cs.rz[0] / pq;
      }
    }
    cs.alpha[0] = a;
    cs.ticket[0] = 0u;
  }
}

static int pick_group(double mean_row) {
  if (mean_row <= 6) return 4;
  if (mean_row <= 12) return 8;
  if (mean_row <= 24) return 16;
  if (mean_row <= 48) return 32;
  return 64;
}

template <typename V, bool DOT>
static hipError_t spmv_dispatch(const int64_t* rp, const int32_t* col, const V* val, int64_t n,
                                double mean_row, const double* x, double* y, const CgState& cs,
                                hipStream_t st) {
  const int G = pick_group(mean_row);
  int64_t groups_per_block = kBlock / G;
  int64_t blocks = (n + groups_per_block - 1) / groups_per_block;
  if (DOT && blocks > kReduceBlocks) blocks = kReduceBlocks;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (blocks < 1) blocks = 1;
  dim3 grid((unsigned)blocks), block(kBlock);
  switch (G) {
    case 4: hipLaunchKernelGGL((k_spmv<4, V, DOT>), grid, block, 0, st, rp, col, val, n, x, y, cs); break;
    case 8: hipLaunchKernelGGL((k_spmv<8, V, DOT>), grid, block, 0, st, rp, col, val, n, x, y, cs); break;
    case 16: hipLaunchKernelGGL((k_spmv<16, V, DOT>), grid, block, 0, st, rp, col, val, n, x, y, cs); break;
    case 32: hipLaunchKernelGGL((k_spmv<32, V, DOT>), grid, block, 0, st, rp, col, val, n, x, y, cs); break;
    default: hipLaunchKernelGGL((k_spmv<64, V, DOT>), grid, block, 0, st, rp, col, val, n, x, y, cs); break;
  }
  return hipGetLastError();
}

hipError_t launch_spmv(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t n,
                       double mean_row, const double* x, double* y, hipStream_t st) {
  CgState cs{};
  if (prec == GP2S_MIXED)
    return spmv_dispatch<float, false>(rp, col, static_cast<const float*>(val), n, mean_row, x, y, cs, st);
  return spmv_dispatch<double, false>(rp, col, static_cast<const double*>(val), n, mean_row, x, y, cs, st);
}

// ---- blocks of S <= 64 right-hand sides --------------------------------------------------
// X, Y row-major [n * S]. One wave per row; lane s owns column s. The row's column
// indices and values are loaded 64 at a time (one per lane) and broadcast with
// readlane, so every lane streams X[j * S + s] for the same j: one coalesced row of X.
__device__ inline double bcast_f64(double v, int l) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, l);
  p.y = __builtin_amdgcn_readlane(p.y, l);
  return __builtin_bit_cast(double, p);
}

template <typename V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm(const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const V* __restrict__ val, int64_t n, int S,
                                                 const double* __restrict__ X,
                                                 double* __restrict__ Y, CgState cs) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t wave = blockIdx.x * (int64_t)(kBlock / kWave) + wid;
  const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
  const bool active = lane < S;
  double dot = 0.0;
  for (int64_t row = wave; row < n; row += nwaves) {
    const int64_t s = rp[row], e = rp[row + 1];
    double acc = 0.0;
    for (int64_t k0 = s; k0 < e; k0 += kWave) {
      const int64_t k = k0 + lane;
      const int32_t cj = k < e ? col[k] : 0;
      const double vj = k < e ? ld(val, k) : 0.0;
      const int cnt = (int)((e - k0) < kWave ? (e - k0) : kWave);
      for (int l = 0; l < cnt; ++l) {
        const int32_t j = __builtin_amdgcn_readlane(cj, l);
        const double v = bcast_f64(vj, l);
        if (active) acc += v * X[(int64_t)j * S + lane];
      }
    }
    if (active) {
      Y[row * S + lane] = acc;
      if (DOT) dot += acc * X[row * S + lane];
    }
  }
  if (!DOT) return;
  __shared__ double sh[kBlock / kWave][kWave];
  __shared__ int am_last;
  sh[wid][lane] = dot;
  __syncthreads();
  if (wid == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w][lane];
    if (active) cs.partial[blockIdx.x * (int64_t)S + lane] = t;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) am_last = atomicAdd(&cs.ticket[0], 1u) == gridDim.x - 1;
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  if (wid == 0 && active) {
    double pq = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) pq += cs.partial[b * (int64_t)S + lane];
    double a = 0.0;
    if (!cs.done[lane]) {
      if (!(pq > 0.0) || !isfinite(pq)) {
        cs.flags[0] = 1;
      } else {
        a = cs.rz[lane] / pq;
      }
    }
    cs.alpha[lane] = a;
  }
  if (threadIdx.x == 0) cs.ticket[0] = 0u;
}

template <typename V, bool DOT>
static hipError_t spmm_dispatch(const int64_t* rp, const int32_t* col, const V* val, int64_t n, int S,
                                const double* X, double* Y, const CgState& cs, hipStream_t st) {
  int64_t blocks = (n + (kBlock / kWave) - 1) / (kBlock / kWave);
  const int64_t cap = DOT ? kReduceBlocks : (1 << 20);
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_spmm<V, DOT>), dim3((unsigned)blocks), dim3(kBlock), 0, st, rp, col, val, n, S,
                     X, Y, cs);
  return hipGetLastError();
}

hipError_t launch_spmm(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t n,
                       int S, const double* X, double* Y, hipStream_t st) {
  CgState cs{};
  if (prec == GP2S_MIXED)
    return spmm_dispatch<float, false>(rp, col, static_cast<const float*>(val), n, S, X, Y, cs, st);
  return spmm_dispatch<double, false>(rp, col, static_cast<const double*>(val), n, S, X, Y, cs, st);
}

hipError_t launch_cg_matvec(int prec, const int64_t* rp, const int32_t* col, const void* val,
                            int64_t n, int S, double mean_row, const double* P, double* Q,
                            const CgState& cs, hipStream_t st) {
  if (S == 1) {
    if (prec == GP2S_MIXED)
      return spmv_dispatch<float, true>(rp, col, static_cast<const float*>(val), n, mean_row, P, Q, cs, st);
    return spmv_dispatch<double, true>(rp, col, static_cast<const double*>(val), n, mean_row, P, Q, cs, st);
  }
  if (prec == GP2S_MIXED)
    return spmm_dispatch<float, true>(rp, col, static_cast<const float*>(val), n, S, P, Q, cs, st);
  return spmm_dispatch<double, true>(rp, col, static_cast<const double*>(val), n, S, P, Q, cs, st);
}

}  // namespace gp2s
