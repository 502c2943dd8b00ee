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
#include "spmm_rows.h"

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
    cs.partial[(int64_t)lane * gridDim.x + blockIdx.x] = t;
  }
}

// Entry-parallel block product (spmm_rows.h) for S in {8, 16, 32, 64}: G lanes per row,
// CW = min(S, 16) columns per pass over the row. p^T q partials per workgroup and
// column as in k_spmm.
template <int G, int S, typename V, typename PT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm_e(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const V* __restrict__ val, int64_t n, const PT* __restrict__ X,
                                                   double* __restrict__ Y, CgState cs) {
  constexpr int CW = S < 16 ? S : 16;
  constexpr int NP = S / CW;
  constexpr int OW = CW / G;
  const int lane = threadIdx.x % G;
  const XcdRows rr = xcd_rows(n, threadIdx.x / G, kBlock / G);
  double dot[NP * OW];
#pragma unroll
  for (int j = 0; j < NP * OW; ++j) dot[j] = 0.0;
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    const int64_t s = rp[row], e = rp[row + 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      double q[OW];
      row_cols_product<G, CW>(col, val, s, e, lane, X, S, p * CW, q);
      const int64_t o = row * S + p * CW + lane * OW;
#pragma unroll
      for (int j = 0; j < OW; ++j) {
        Y[o + j] = q[j];
        if (DOT) dot[p * OW + j] += q[j] * (double)X[o + j];
      }
    }
  }
  if (!DOT) return;
  __shared__ double sh[kBlock / kWave][S];
  const int wid = threadIdx.x / kWave, wl = threadIdx.x % kWave;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int j = 0; j < OW; ++j) {
      const double t = wave_sum_strided<G>(dot[p * OW + j]);
      if (wl < G) sh[wid][p * CW + wl * OW + j] = t;
    }
  __syncthreads();
  if ((int)threadIdx.x < S) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w][threadIdx.x];
    cs.partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// Slice-per-lane block product (spmm_rows.h) for S in {8, 16, 32, 64}: one wave per
// row, 16-byte column slices per lane. p^T q partials per workgroup and column as in k_spmm.
template <int S, typename V, typename PT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm_s(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const V* __restrict__ val, int64_t n, const PT* __restrict__ X,
                                                   double* __restrict__ Y, CgState cs) {
  constexpr int VW = 16 / sizeof(PT);
  constexpr int LE = S / VW;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cq = lane % LE;
  const XcdRows rr = xcd_rows(n, wid, kBlock / kWave);
  double dot[VW];
#pragma unroll
  for (int c = 0; c < VW; ++c) dot[c] = 0.0;
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    double acc[VW];
    row_slices_product<S>(col, val, rp[row], rp[row + 1], lane, X, acc);
    if (lane < LE) {
      const int64_t o = row * S + cq * VW;
#pragma unroll
      for (int c = 0; c < VW; ++c) {
        Y[o + c] = acc[c];
        if (DOT) dot[c] += acc[c] * (double)X[o + c];
      }
    }
  }
  if (!DOT) return;
  __shared__ double sh[kBlock / kWave][S];
  if (lane < LE)
#pragma unroll
    for (int c = 0; c < VW; ++c) sh[wid][cq * VW + c] = dot[c];
  __syncthreads();
  if ((int)threadIdx.x < S) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w][threadIdx.x];
    cs.partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// LDS-staged block product over row tiles (S in {8, 16, 32, 64}). A workgroup takes the
// tiles of an XCD-contiguous range in turn: it copies the rows of X in the tile's column
// intervals into LDS (as many whole intervals as fit in kTileLdsBytes), then each wave
// multiplies whole rows with row_tiled_product, reading staged rows from LDS and the
// rest from X. p^T q partials per workgroup and column as in k_spmm.
template <int S, typename V, typename PT, bool DOT>
__global__ __launch_bounds__(kTileBlock) void k_spmm_t(const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col, const V* __restrict__ val,
                                                       const RowTile* __restrict__ tiles, int64_t ntiles,
                                                       const PT* __restrict__ X, double* __restrict__ Y, CgState cs) {
  constexpr int VW = 16 / sizeof(PT);
  constexpr int LE = S / VW;
  constexpr int NW = kTileBlock / kWave;
  constexpr int BUDGET = kTileLdsBytes / (S * (int)sizeof(PT));  // rows of X
  __shared__ __align__(16) PT lds[BUDGET * S];
  __shared__ int32_t iv_lo[kTileMaxIv], iv_len[kTileMaxIv], iv_base[kTileMaxIv];
  __shared__ int64_t t_rp[kTileMaxRows + 1];
  __shared__ int64_t t_row0;
  __shared__ int32_t t_rows, t_niv;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cq = lane % LE;
  const XcdRows tr = xcd_rows(ntiles, 0, 1);
  double dot[VW];
#pragma unroll
  for (int c = 0; c < VW; ++c) dot[c] = 0.0;
  for (int64_t t = tr.first; t < tr.end; t += tr.step) {
    if (threadIdx.x == 0) {
      const RowTile& T = tiles[t];
      t_row0 = T.row0;
      t_rows = T.rows < kTileMaxRows ? T.rows : kTileMaxRows;
      const int niv = T.niv < kTileMaxIv ? T.niv : kTileMaxIv;
      t_niv = niv;
      int cum = 0;
      for (int k = 0; k < niv; ++k) {
        iv_lo[k] = T.lo[k];
        iv_len[k] = T.len[k];
        if (T.len[k] > 0 && cum + T.len[k] <= BUDGET) {
          iv_base[k] = cum;
          cum += T.len[k];
        } else {
          iv_base[k] = -1;
        }
      }
    }
    __syncthreads();
    const int niv = t_niv;
    const int64_t r0 = t_row0;
    const int nrows = t_rows;
    if ((int)threadIdx.x <= nrows) t_rp[threadIdx.x] = rp[r0 + threadIdx.x];
    for (int k = 0; k < niv; ++k) {
      if (iv_base[k] < 0) continue;
      const float4* __restrict__ src = reinterpret_cast<const float4*>(X + (int64_t)iv_lo[k] * S);
      float4* dst = reinterpret_cast<float4*>(lds + (int64_t)iv_base[k] * S);
      const int nvec = iv_len[k] * (S * (int)sizeof(PT) / 16);
      int i = threadIdx.x;
      for (; i + kTileBlock < nvec; i += 2 * kTileBlock) {  // two loads in flight per thread
        const float4 a = src[i], b = src[i + kTileBlock];
        dst[i] = a;
        dst[i + kTileBlock] = b;
      }
      if (i < nvec) dst[i] = src[i];
    }
    __syncthreads();
    for (int rl = wid; rl < nrows; rl += NW) {
      double acc[VW];
      row_tiled_product<S>(col, val, t_rp[rl], t_rp[rl + 1], lane, X, lds, niv, iv_lo, iv_len, iv_base, acc);
      if (lane < LE) {
        const int64_t o = (r0 + rl) * S + cq * VW;
#pragma unroll
        for (int c = 0; c < VW; ++c) {
          Y[o + c] = acc[c];
          if (DOT) dot[c] += acc[c] * (double)X[o + c];
        }
      }
    }
    __syncthreads();  // the next tile overwrites LDS and the descriptors
  }
  if (!DOT) return;
  double* sh = reinterpret_cast<double*>(lds);  // LDS is free now (NW * S doubles)
  if (lane < LE)
#pragma unroll
    for (int c = 0; c < VW; ++c) sh[wid * S + cq * VW + c] = dot[c];
  __syncthreads();
  if ((int)threadIdx.x < S) {
    double tsum = 0.0;
    for (int w = 0; w < NW; ++w) tsum += sh[w * S + threadIdx.x];
    cs.partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = tsum;
  }
}

// Lanes per row of the entry-parallel product: about a sixth of the mean row length,
// a power of two in [4, min(16, S)].
static int pick_entry_group(double mean_row, int S) {
  int g = 4;
  const int gmax = S < 16 ? S : 16;
  while (g < gmax && 2 * g <= mean_row / 6.0 + 1e-9) g *= 2;
  return g;
}

// Launches k_spmm_e with G lanes per row when (S, G) has an instance and X is 16-byte
// aligned; returns false otherwise.
template <typename V, typename PT, bool DOT>
static bool spmm_entry(int G, const int64_t* rp, const int32_t* col, const V* val, int64_t n, int S, const PT* X,
                       double* Y, const CgState& cs, hipStream_t st, int64_t blocks) {
  if (!entry_product_ok(S, G) || (reinterpret_cast<uintptr_t>(X) & 15) != 0) return false;
  dim3 grid((unsigned)blocks), block(kBlock);
#define GP2S_SPMM_E(GG, SS)                                                                            \
  if (G == GG && S == SS) {                                                                           \
    hipLaunchKernelGGL((k_spmm_e<GG, SS, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs); \
    return true;                                                                                      \
  }
  GP2S_SPMM_E(4, 8) GP2S_SPMM_E(8, 8)
  GP2S_SPMM_E(4, 16) GP2S_SPMM_E(8, 16) GP2S_SPMM_E(16, 16)
  GP2S_SPMM_E(4, 32) GP2S_SPMM_E(8, 32) GP2S_SPMM_E(16, 32)
  GP2S_SPMM_E(4, 64) GP2S_SPMM_E(8, 64) GP2S_SPMM_E(16, 64)
#undef GP2S_SPMM_E
  return false;
}

// Row-grouped block product (S in {32, 64}): one wave per group of kGrp consecutive
// rows. NSUB lane sets walk interleaved union columns (LE lanes cover one row of X with
// 16-byte slices, so every load instruction moves NSUB distinct rows of X) and apply
// each gathered slice to all kGrp rows of the group with their values (zero where a
// row has no entry): a row of X is read once per group instead of once per stored
// entry. The union columns are fetched 64 at a time, one per lane, and handed to the
// lane sets by shuffles, so the gathers do not wait on dependent loads. The NSUB
// partial sums are combined by a fixed butterfly; products accumulate in float64.
template <int S, typename V, typename PT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm_g(const int64_t* __restrict__ gptr, const int32_t* __restrict__ gcol,
                                                   const V* __restrict__ gval, int64_t ngroups, int64_t n,
                                                   const PT* __restrict__ X, double* __restrict__ Y, CgState cs) {
  constexpr int VW = 16 / sizeof(PT);  // elements of X per lane
  constexpr int LE = S / VW;           // lanes per row of X
  constexpr int NSUB = kWave / LE;     // union columns per step
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cq = lane % LE, sub = lane / LE;
  const XcdRows rr = xcd_rows(ngroups, wid, kBlock / kWave);
  double dot[VW];
#pragma unroll
  for (int c = 0; c < VW; ++c) dot[c] = 0.0;
  for (int64_t g = rr.first; g < rr.end; g += rr.step) {
    double acc[kGrp][VW];
#pragma unroll
    for (int r = 0; r < kGrp; ++r)
#pragma unroll
      for (int c = 0; c < VW; ++c) acc[r][c] = 0.0;
    const int64_t b = gptr[g], e = gptr[g + 1];
    for (int64_t k0 = b; k0 < e; k0 += kWave) {
      const int cnt = (int)((e - k0) < kWave ? (e - k0) : kWave);
      const int32_t colreg = lane < cnt ? gcol[k0 + lane] : 0;
#pragma unroll 2
      for (int j = 0; j < cnt; j += NSUB) {
        const int idx = j + sub;
        const int32_t c = __shfl(colreg, idx, kWave);
        if (idx < cnt) {
          PT x[VW];
          *reinterpret_cast<float4*>(x) = *reinterpret_cast<const float4*>(X + (int64_t)c * S + cq * VW);
          V v[kGrp];
#pragma unroll
          for (int q = 0; q < kGrp * (int)sizeof(V) / 16; ++q)
            reinterpret_cast<float4*>(v)[q] = reinterpret_cast<const float4*>(gval + (k0 + idx) * kGrp)[q];
#pragma unroll
          for (int r = 0; r < kGrp; ++r)
#pragma unroll
            for (int cc = 0; cc < VW; ++cc) acc[r][cc] = fma((double)v[r], (double)x[cc], acc[r][cc]);
        }
      }
    }
#pragma unroll
    for (int off = LE; off < kWave; off <<= 1)
#pragma unroll
      for (int r = 0; r < kGrp; ++r)
#pragma unroll
        for (int c = 0; c < VW; ++c) acc[r][c] += __shfl_xor(acc[r][c], off, kWave);
    if (sub == 0) {
#pragma unroll
      for (int r = 0; r < kGrp; ++r) {
        const int64_t row = g * kGrp + r;
        if (row < n) {
          const int64_t o = row * S + cq * VW;
#pragma unroll
          for (int c = 0; c < VW; ++c) {
            Y[o + c] = acc[r][c];
            if (DOT) dot[c] += acc[r][c] * (double)X[o + c];
          }
        }
      }
    }
  }
  if (!DOT) return;
  __shared__ double sh[kBlock / kWave][S];
  if (sub == 0)
#pragma unroll
    for (int c = 0; c < VW; ++c) sh[wid][cq * VW + c] = dot[c];
  __syncthreads();
  if ((int)threadIdx.x < S) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w][threadIdx.x];
    cs.partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// Launches k_spmm_g when S has an instance, the grouped copy exists and X is 16-byte aligned.
template <typename V, typename PT, bool DOT>
static bool spmm_grouped(int64_t n, int S, const TileSet& ts, const PT* X, double* Y, const CgState& cs,
                         hipStream_t st, int64_t blocks) {
  if ((S != 32 && S != 64) || !ts.gptr || ts.ngroups < 1 || (reinterpret_cast<uintptr_t>(X) & 15) != 0) return false;
  const V* gv = static_cast<const V*>(ts.gval);
  dim3 grid((unsigned)blocks), block(kBlock);
  if (S == 32)
    hipLaunchKernelGGL((k_spmm_g<32, V, PT, DOT>), grid, block, 0, st, ts.gptr, ts.gcol, gv, ts.ngroups, n, X, Y, cs);
  else
    hipLaunchKernelGGL((k_spmm_g<64, V, PT, DOT>), grid, block, 0, st, ts.gptr, ts.gcol, gv, ts.ngroups, n, X, Y, cs);
  return true;
}

// Launches k_spmm_s when S has an instance and X is 16-byte aligned.
template <typename V, typename PT, bool DOT>
static bool spmm_slices(const int64_t* rp, const int32_t* col, const V* val, int64_t n, int S, const PT* X, double* Y,
                        const CgState& cs, hipStream_t st, int64_t blocks) {
  if ((S != 8 && S != 16 && S != 32 && S != 64) || (reinterpret_cast<uintptr_t>(X) & 15) != 0) return false;
  dim3 grid((unsigned)blocks), block(kBlock);
  switch (S) {
    case 8: hipLaunchKernelGGL((k_spmm_s<8, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs); break;
    case 16: hipLaunchKernelGGL((k_spmm_s<16, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs); break;
    case 32: hipLaunchKernelGGL((k_spmm_s<32, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs); break;
    default: hipLaunchKernelGGL((k_spmm_s<64, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs); break;
  }
  return true;
}

// Launches k_spmm_t when S has an instance, tiles exist and X is 16-byte aligned.
template <typename V, typename PT, bool DOT>
static bool spmm_tiles(const int64_t* rp, const int32_t* col, const V* val, int S, const TileSet& tiles,
                       const PT* X, double* Y, const CgState& cs, hipStream_t st, int64_t blocks) {
  if ((S != 8 && S != 16 && S != 32 && S != 64) || !tiles.t || tiles.n < 1 ||
      (reinterpret_cast<uintptr_t>(X) & 15) != 0)
    return false;
  dim3 grid((unsigned)blocks), block(kTileBlock);
  switch (S) {
    case 8:
      hipLaunchKernelGGL((k_spmm_t<8, V, PT, DOT>), grid, block, 0, st, rp, col, val, tiles.t, tiles.n, X, Y, cs);
      break;
    case 16:
      hipLaunchKernelGGL((k_spmm_t<16, V, PT, DOT>), grid, block, 0, st, rp, col, val, tiles.t, tiles.n, X, Y, cs);
      break;
    case 32:
      hipLaunchKernelGGL((k_spmm_t<32, V, PT, DOT>), grid, block, 0, st, rp, col, val, tiles.t, tiles.n, X, Y, cs);
      break;
    default:
      hipLaunchKernelGGL((k_spmm_t<64, V, PT, DOT>), grid, block, 0, st, rp, col, val, tiles.t, tiles.n, X, Y, cs);
      break;
  }
  return true;
}

// variant: 0 lane per column, 1 slice per lane, 2 LDS-staged row tiles, 3 row groups,
// G > 3 entry-parallel with G lanes per row, -1 heuristic (entry-parallel up to 32
// columns, else one lane per column).
template <typename V, typename PT, bool DOT>
static hipError_t spmm_dispatch(const int64_t* rp, const int32_t* col, const V* val, int64_t n, int S,
                                double mean_row, int variant, const TileSet& tiles, const PT* X, double* Y,
                                const CgState& cs, hipStream_t st, int* nblocks = nullptr) {
  const int64_t cap = DOT ? kReduceBlocks : (1 << 20);
  auto grid_for = [&](int64_t rows_per_block) {
    int64_t b = (n + rows_per_block - 1) / rows_per_block;
    if (b > cap) b = cap;
    return round_up8(b < 1 ? 1 : b);
  };
  const int G = variant >= 0 ? variant : (S <= 32 ? pick_entry_group(mean_row, S) : 0);
  if (G == 1) {
    const int64_t sb = grid_for(kBlock / kWave);
    if (spmm_slices<V, PT, DOT>(rp, col, val, n, S, X, Y, cs, st, sb)) {
      if (nblocks) *nblocks = (int)sb;
      return hipGetLastError();
    }
  } else if (G == 2) {
    int64_t tb = tiles.n < cap ? tiles.n : cap;
    tb = round_up8(tb < 1 ? 1 : tb);
    if (spmm_tiles<V, PT, DOT>(rp, col, val, S, tiles, X, Y, cs, st, tb)) {
      if (nblocks) *nblocks = (int)tb;
      return hipGetLastError();
    }
  } else if (G == 3) {
    int64_t gb = (tiles.ngroups + kBlock / kWave - 1) / (kBlock / kWave);
    if (gb > cap) gb = cap;
    gb = round_up8(gb < 1 ? 1 : gb);
    if (spmm_grouped<V, PT, DOT>(n, S, tiles, X, Y, cs, st, gb)) {
      if (nblocks) *nblocks = (int)gb;
      return hipGetLastError();
    }
  } else if (G > 3) {
    const int64_t eb = grid_for(kBlock / G);
    if (spmm_entry<V, PT, DOT>(G, rp, col, val, n, S, X, Y, cs, st, eb)) {
      if (nblocks) *nblocks = (int)eb;
      return hipGetLastError();
    }
  }
  const int64_t blocks = grid_for(kBlock / kWave);
  if (nblocks) *nblocks = (int)blocks;
  hipLaunchKernelGGL((k_spmm<V, PT, double, DOT>), dim3((unsigned)blocks), dim3(kBlock), 0, st, rp, col, val, n, S,
                     X, Y, cs);
  return hipGetLastError();
}

hipError_t launch_spmm(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t n,
                       int S, double mean_row, int variant, const TileSet& tiles, const double* X, double* Y,
                       hipStream_t st) {
  CgState cs{};
  if (prec == GP2S_MIXED)
    return spmm_dispatch<float, double, false>(rp, col, static_cast<const float*>(val), n, S, mean_row, variant,
                                               tiles, X, Y, cs, st);
  return spmm_dispatch<double, double, false>(rp, col, static_cast<const double*>(val), n, S, mean_row, variant,
                                              tiles, X, Y, cs, st);
}

hipError_t launch_cg_matvec(int prec, const int64_t* rp, const int32_t* col, const void* val,
                            int64_t n, int S, double mean_row, int variant, const TileSet& tiles, const void* P,
                            void* Q, bool f32vec, const CgState& cs, hipStream_t st) {
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
      e = spmm_dispatch<float, float, true>(rp, col, static_cast<const float*>(val), n, S, mean_row, variant, tiles,
                                            static_cast<const float*>(P), static_cast<double*>(Q), cs, st, &nb);
    else
      e = spmm_dispatch<float, double, true>(rp, col, static_cast<const float*>(val), n, S, mean_row, variant, tiles,
                                             static_cast<const double*>(P), static_cast<double*>(Q), cs, st, &nb);
  } else {
    e = spmm_dispatch<double, double, true>(rp, col, static_cast<const double*>(val), n, S, mean_row, variant, tiles,
                                            static_cast<const double*>(P), static_cast<double*>(Q), cs, st, &nb);
  }
  if (e != hipSuccess) return e;
  return launch_cg_alpha(cs, nb, S, st);
}

}  // namespace gp2s
