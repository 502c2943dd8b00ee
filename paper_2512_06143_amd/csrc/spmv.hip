// CSR products with the assembled covariance: single right-hand side (vector CSR,
// a group of G lanes per row) and blocks of up to 64 right-hand sides (one wave per
// row, one lane per column). These drive the solve K a = y and the probe solves of
// the log-determinant (Sec. 3.5; App. B.6 "MINRES", "LOGDET"). Stored values
// (float32 or float64) multiply the vectors and accumulate in float64.
//
// Both are bandwidth kernels: loads are issued in independent groups of four or
// eight so that enough gathers are in flight per wave, and grids are large enough to
// keep every CU's wave slots busy. The CG variants also write p^T q per column as
// fixed per-workgroup partial sums; a finalize kernel (pcg.hip) reduces them in
// workgroup order, so results are bitwise reproducible.
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
  const XcdRows rr = xcd_rows(n, threadIdx.x / G, kBlock / G);
  double dot = 0.0;
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    const int64_t s = rp[row], e = rp[row + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t k = s + lane;
    for (; k + 3 * G < e; k += 4 * G) {
      const int32_t c0 = col[k], c1 = col[k + G], c2 = col[k + 2 * G], c3 = col[k + 3 * G];
      const double v0 = ld(val, k), v1 = ld(val, k + G), v2 = ld(val, k + 2 * G), v3 = ld(val, k + 3 * G);
      const double x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
      a0 += v0 * x0;
      a1 += v1 * x1;
      a2 += v2 * x2;
      a3 += v3 * x3;
    }
    for (; k < e; k += G) a0 += ld(val, k) * x[col[k]];
    double acc = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (lane == 0) {
      y[row] = acc;
      if (DOT) dot += acc * x[row];
    }
  }
  if (!DOT) return;
  // p^T q partial of this workgroup; alpha is formed by launch_cg_alpha.
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = dot;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cs.partial[blockIdx.x] = sh[0];
}

// Lanes per row: about half the mean row length, a power of two in [4, 64].
static int pick_group(double mean_row) {
  int g = 4;
  while (g < 64 && 2 * g <= mean_row / 2.0 + 1e-9) g *= 2;
  return g;
}

template <typename V, bool DOT>
static hipError_t spmv_dispatch(const int64_t* rp, const int32_t* col, const V* val, int64_t n,
                                double mean_row, const double* x, double* y, const CgState& cs,
                                hipStream_t st, int* nblocks = nullptr) {
  const int G = pick_group(mean_row);
  int64_t groups_per_block = kBlock / G;
  int64_t blocks = (n + groups_per_block - 1) / groups_per_block;
  const int64_t cap = DOT ? kReduceBlocks : (1 << 20);
  if (blocks > cap) blocks = cap;
  blocks = round_up8(blocks < 1 ? 1 : blocks);
  if (nblocks) *nblocks = (int)blocks;
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
// X, Y row-major [n * S] (float32 or float64 vectors). One wave per row; lane s owns
// column s. The row's column offsets (j * S) and values are loaded 64 at a time (one
// per lane) and broadcast with readlane, so every lane reads X[j * S + s] for the
// same j: one coalesced row of X per stored entry, eight rows in flight per wave.
// The loop is bound by vector-instruction issue, not memory. Search directions may be
// float32 (the probe block of the mixed path); products accumulate and are stored in
// float64 either way.
__device__ inline double bcast_acc(double v, int l) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, l);
  p.y = __builtin_amdgcn_readlane(p.y, l);
  return __builtin_bit_cast(double, p);
}
__device__ inline float bcast_acc(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

constexpr int kSpmmUnroll = 8;

template <typename V, typename PT, typename QT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm(const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const V* __restrict__ val, int64_t n, int S,
                                                 const PT* __restrict__ X,
                                                 QT* __restrict__ Y, CgState cs) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const XcdRows rr = xcd_rows(n, wid, kBlock / kWave);
  const bool active = lane < S;
  const int ls = active ? lane : 0;
  const PT* __restrict__ Xl = X + ls;  // this lane's column
  double dot = 0.0;
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    const int64_t s = rp[row], e = rp[row + 1];
    double acc = 0.0;
    for (int64_t k0 = s; k0 < e; k0 += kWave) {
      // one stored entry per lane: row offset of its column in X (n * S < 2^31) and value
      const int64_t k = k0 + lane;
      const int32_t off = k < e ? col[k] * S : 0;
      const V vj = k < e ? val[k] : (V)0;
      const int cnt = (int)((e - k0) < kWave ? (e - k0) : kWave);
      int l = 0;
      for (; l + kSpmmUnroll <= cnt; l += kSpmmUnroll) {
        double xv[kSpmmUnroll], vv[kSpmmUnroll];
#pragma unroll
        for (int u = 0; u < kSpmmUnroll; ++u) {
          vv[u] = (double)bcast_acc(vj, l + u);
          xv[u] = (double)Xl[__builtin_amdgcn_readlane(off, l + u)];
        }
#pragma unroll
        for (int u = 0; u < kSpmmUnroll; ++u) acc += vv[u] * xv[u];
      }
      for (; l < cnt; ++l) acc += (double)bcast_acc(vj, l) * (double)Xl[__builtin_amdgcn_readlane(off, l)];
    }
    if (active) {
      const QT q = (QT)acc;
      Y[row * S + lane] = q;
      if (DOT) dot += (double)q * (double)X[row * S + lane];
    }
  }
  if (!DOT) return;
  // per-column p^T q partials of this workgroup; alpha is formed by launch_cg_alpha.
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = dot;
  __syncthreads();
  if (wid == 0 && active) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w * kWave + lane];
    cs.partial[blockIdx.x * (int64_t)S + lane] = t;
  }
}

template <typename V, typename PT, typename QT, bool DOT>
static hipError_t spmm_dispatch(const int64_t* rp, const int32_t* col, const V* val, int64_t n, int S,
                                const PT* X, QT* Y, const CgState& cs, hipStream_t st,
                                int* nblocks = nullptr) {
  int64_t blocks = (n + (kBlock / kWave) - 1) / (kBlock / kWave);
  const int64_t cap = DOT ? kReduceBlocks : (1 << 20);
  if (blocks > cap) blocks = cap;
  blocks = round_up8(blocks < 1 ? 1 : blocks);
  if (nblocks) *nblocks = (int)blocks;
  hipLaunchKernelGGL((k_spmm<V, PT, QT, DOT>), dim3((unsigned)blocks), dim3(kBlock), 0, st, rp, col, val, n, S,
                     X, Y, cs);
  return hipGetLastError();
}

hipError_t launch_spmm(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t n,
                       int S, const double* X, double* Y, hipStream_t st) {
  CgState cs{};
  if (prec == GP2S_MIXED)
    return spmm_dispatch<float, double, double, false>(rp, col, static_cast<const float*>(val), n, S, X, Y, cs, st);
  return spmm_dispatch<double, double, double, false>(rp, col, static_cast<const double*>(val), n, S, X, Y, cs, st);
}

hipError_t launch_cg_matvec(int prec, const int64_t* rp, const int32_t* col, const void* val,
                            int64_t n, int S, double mean_row, const void* P, void* Q, bool f32vec,
                            const CgState& cs, hipStream_t st) {
  int nb = 0;
  hipError_t e;
  if (S == 1) {
    // single right-hand side: always float64 vectors
    if (prec == GP2S_MIXED)
      e = spmv_dispatch<float, true>(rp, col, static_cast<const float*>(val), n, mean_row,
                                     static_cast<const double*>(P), static_cast<double*>(Q), cs, st, &nb);
    else
      e = spmv_dispatch<double, true>(rp, col, static_cast<const double*>(val), n, mean_row,
                                      static_cast<const double*>(P), static_cast<double*>(Q), cs, st, &nb);
  } else if (prec == GP2S_MIXED) {
    if (f32vec)
      e = spmm_dispatch<float, float, double, true>(rp, col, static_cast<const float*>(val), n, S,
                                                    static_cast<const float*>(P), static_cast<double*>(Q), cs, st,
                                                    &nb);
    else
      e = spmm_dispatch<float, double, double, true>(rp, col, static_cast<const float*>(val), n, S,
                                                     static_cast<const double*>(P), static_cast<double*>(Q), cs, st,
                                                     &nb);
  } else {
    e = spmm_dispatch<double, double, double, true>(rp, col, static_cast<const double*>(val), n, S,
                                                    static_cast<const double*>(P), static_cast<double*>(Q), cs, st,
                                                    &nb);
  }
  if (e != hipSuccess) return e;
  return launch_cg_alpha(cs, nb, S, st);
}

}  // namespace gp2s
