// CSR products with the assembled covariance: single right-hand side (k_spmv_a,
// nnz-balanced row blocks streamed as 16-byte quads, for matrix handles; k_spmv, a
// group of G lanes per row, for other CSRs) and blocks of up to 64 right-hand sides
// (several variants, picked per matrix by timing). These drive the solve K a = y and
// the probe solves of the log-determinant (Sec. 4.6; App. B.6 "MINRES", "LOGDET").
// Stored values (float32 or float64) multiply the vectors and accumulate in float64.
//
// The single-RHS products stream the CSR from HBM; the block products are bound by the
// vector-memory units that serve their gathered rows of X. The CG variants also write
// p^T q per column as fixed per-workgroup partial sums; a finalize kernel (pcg.hip)
// reduces them in workgroup order, so results are bitwise reproducible.
#include "gp2s_internal.h"
#include "spmm_rows.h"

namespace gp2s {

template <typename V>
__device__ inline double ld(const V* p, int64_t k) {
  return (double)p[k];
}

// ---- single right-hand side -----------------------------------------------------------
// G lanes per row, for CSRs without row blocks such as the posterior's cross-covariance
// (the batched solves have their own kernel). A row's entries take three dependent trips
// to memory (row pointers, then columns and values, then the gathered x), so a group
// issues all of a row's column and value loads at once (kWave / G per lane: rows up to
// 64 entries in one pass) before any gather, and loads the next row's pointers before
// it multiplies the current row. Every load is
// unconditional, at an index clamped into the row (lanes past its end reread its last
// entry and their products are dropped by a select): a predicated load would become a
// branch, and the compiler then waits for each load inside its branch.
template <int G, typename V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv(const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const V* __restrict__ val, int64_t n,
                                                 const double* __restrict__ x,
                                                 double* __restrict__ y, CgState cs) {
  constexpr int U = kWave / G;
  const int lane = threadIdx.x & (G - 1);
  const XcdRows rr = xcd_rows(n, threadIdx.x / G, kBlock / G);
  double dot = 0.0;
  if (rr.first >= rr.end) {
    if (!DOT) return;
  } else {
    int64_t s = rp[rr.first], e = rp[rr.first + 1];
    for (int64_t row = rr.first; row < rr.end; row += rr.step) {
      // the next row's extent (this row's again past the range: a valid index)
      const int64_t nrow = row + rr.step < rr.end ? row + rr.step : row;
      const int64_t ns = rp[nrow], ne = rp[nrow + 1];
      double acc = 0.0;
      for (int64_t k0 = s + lane; k0 < e; k0 += (int64_t)U * G) {
        int32_t c[U];
        V v[U];
        bool in[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int64_t k = k0 + (int64_t)j * G;
          in[j] = k < e;
          const int64_t kk = in[j] ? k : e - 1;  // e - 1 >= k0 >= s: inside the row
          c[j] = col[kk];
          v[j] = val[kk];
        }
        double xv[U];
#pragma unroll
        for (int j = 0; j < U; ++j) xv[j] = x[c[j]];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const double t = (double)v[j] * xv[j];
          acc += in[j] ? t : 0.0;
        }
      }
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
      if (lane == 0) {
        y[row] = acc;
        if (DOT) dot += acc * x[row];
      }
      s = ns;
      e = ne;
    }
    if (!DOT) return;
  }
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

// nnz-balanced streaming product (single right-hand side; matrix handles only). The
// rows are cut into blocks by where they start: block b holds the rows whose first
// entry lies in [b C, (b + 1) C), C = kStreamChunk (the block boundaries rowblk[] come
// from launch_rowblocks). Every row of a block but the last ends inside that span, so
// one pass of C entries from the block's first entry covers all of them; only the last
// row can run on, over further passes. A workgroup streams a pass's columns and values
// as aligned 16-byte quads (4 entries per thread and load: far more bytes in flight
// than lane groups per row issuing 4-byte loads), gathers x and writes the products to
// LDS; the rows are then summed in a fixed order by L lanes each (L = 256 / rows, a
// power of two up to 64, or one lane and several rows per thread), and a last row that
// runs on is summed by the whole workgroup across passes. The work per workgroup is
// balanced by entries whatever the row lengths (clustered clouds have rows from 1 to
// thousands of entries). Quads past the block's last entry are clamped onto that
// entry's quad (a cached reread, never summed); col and val must be 16-byte aligned
// and hold kQuadPad valid entries past nnz.
constexpr int kStreamChunk = 2048;  // entries per pass (16 KB of float64 products)

__device__ inline void load_quad(const float* p, double (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
__device__ inline void load_quad(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}

template <typename V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv_a(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const V* __restrict__ val, const int32_t* __restrict__ rowblk,
                                                   int64_t nblk, const double* __restrict__ x,
                                                   double* __restrict__ y, CgState cs) {
  constexpr int NU = kStreamChunk / (4 * kBlock);
  __shared__ double prod[kStreamChunk];
  __shared__ double red[kBlock];
  const int t = threadIdx.x;
  double dot = 0.0;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t r0 = rowblk[b], r1 = rowblk[b + 1];
    if (r0 == r1) continue;  // uniform: no row starts in this span
    const int64_t E0 = rp[r0], E1 = rp[r1];
    const int64_t A0 = E0 & ~(int64_t)3;
    const int64_t qlast = (E1 - 1) & ~(int64_t)3;  // quad holding the block's last entry
    const bool runs_on = E1 > A0 + kStreamChunk;    // the last row needs further passes
    // rows summed after the first pass: all, or all but a last row that runs on
    const int64_t nf = (r1 - r0) - (runs_on ? 1 : 0);
    const int L = nf >= kBlock ? 1 : (nf <= kBlock / kWave ? kWave : kBlock / (int)nf);
    const int Lp = 1 << (31 - __clz(L));  // power of two, divides 64
    const int lane = t % Lp;
    const int64_t grp = t / Lp, ngrp = kBlock / Lp;
    double acc_last = 0.0;
    for (int64_t c0 = A0; c0 < E1; c0 += kStreamChunk) {
      int32_t c[NU][4];
      double v[NU][4];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int64_t q = min(c0 + 4 * t + (int64_t)(4 * kBlock) * u, qlast);
        const int4 cq = *reinterpret_cast<const int4*>(col + q);
        c[u][0] = cq.x;
        c[u][1] = cq.y;
        c[u][2] = cq.z;
        c[u][3] = cq.w;
        load_quad(val + q, v[u]);
      }
      double xv[NU][4];
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[u][i] = x[c[u][i]];
#pragma unroll
      for (int u = 0; u < NU; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) prod[4 * t + 4 * kBlock * u + i] = v[u][i] * xv[u][i];
      __syncthreads();
      if (c0 == A0) {
        // rows r0 .. r0 + nf - 1 lie inside this pass
        for (int64_t g = grp; g < nf; g += ngrp) {
          const int64_t row = r0 + g;
          const int64_t s = rp[row], e = rp[row + 1];
          double acc = 0.0;
          for (int64_t k = s + lane; k < e; k += Lp) acc += prod[k - c0];
          for (int o = Lp / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
          if (lane == 0) {
            y[row] = acc;
            if (DOT) dot += acc * x[row];
          }
        }
      }
      if (runs_on) {
        const int64_t s = rp[r1 - 1];
        const int64_t lo = max(s, c0), hi = min(E1, c0 + kStreamChunk);
        for (int64_t k = lo + t; k < hi; k += kBlock) acc_last += prod[k - c0];
      }
      __syncthreads();
    }
    if (runs_on) {  // uniform per block
      red[t] = acc_last;
      __syncthreads();
      for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
      }
      if (t == 0) {
        y[r1 - 1] = red[0];
        if (DOT) dot += red[0] * x[r1 - 1];
      }
      __syncthreads();
    }
  }
  if (!DOT) return;
  red[t] = dot;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) cs.partial[blockIdx.x] = red[0];
}

// rowblk[b] = the first row whose first entry is at or past b C (b < nblk), rowblk[nblk] = n.
__global__ void k_rowblocks(const int64_t* __restrict__ rp, int64_t n, int64_t nblk, int32_t* __restrict__ rowblk) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b <= nblk; b += (int64_t)gridDim.x * blockDim.x) {
    if (b == nblk) {
      rowblk[b] = (int32_t)n;
      continue;
    }
    const int64_t target = b * kStreamChunk;
    int64_t lo = 0, hi = n;  // first i in [0, n] with rp[i] >= target
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (rp[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    rowblk[b] = (int32_t)lo;
  }
}

int64_t rowblocks_count(int64_t nnz) { return (nnz + kStreamChunk - 1) / kStreamChunk; }

hipError_t launch_rowblocks(const int64_t* rp, int64_t n, int64_t nnz, int32_t* rowblk, hipStream_t st) {
  const int64_t nblk = rowblocks_count(nnz);
  int64_t blocks = (nblk + 1 + kBlock - 1) / kBlock;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_rowblocks, dim3((unsigned)blocks), dim3(kBlock), 0, st, rp, n, nblk, rowblk);
  return hipGetLastError();
}

// Lanes per row: about half the mean row length, a power of two in [4, 64].
static int pick_group(double mean_row) {
  int g = 4;
  while (g < 64 && 2 * g <= mean_row / 2.0 + 1e-9) g *= 2;
  return g;
}

template <typename V, bool DOT>
static hipError_t spmv_dispatch(const int64_t* rp, const int32_t* col, const V* val, int64_t n,
                                double mean_row, const RowBlocks& rb, const double* x, double* y, const CgState& cs,
                                hipStream_t st, int* nblocks = nullptr) {
  const int64_t cap = DOT ? kReduceBlocks : (1 << 20);
  if (rb.blk && rb.n > 0 && ((reinterpret_cast<uintptr_t>(col) | reinterpret_cast<uintptr_t>(val)) & 15) == 0) {
    int64_t blocks = rb.n < cap ? rb.n : cap;
    blocks = round_up8(blocks < 1 ? 1 : blocks);
    if (nblocks) *nblocks = (int)blocks;
    hipLaunchKernelGGL((k_spmv_a<V, DOT>), dim3((unsigned)blocks), dim3(kBlock), 0, st, rp, col, val, rb.blk, rb.n,
                       x, y, cs);
    return hipGetLastError();
  }
  const int G = pick_group(mean_row);
  int64_t groups_per_block = kBlock / G;
  int64_t blocks = (n + groups_per_block - 1) / groups_per_block;
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
                       double mean_row, const double* x, double* y, hipStream_t st, const RowBlocks& rb) {
  CgState cs{};
  if (prec == GP2S_MIXED)
    return spmv_dispatch<float, false>(rp, col, static_cast<const float*>(val), n, mean_row, rb, x, y, cs, st);
  return spmv_dispatch<double, false>(rp, col, static_cast<const double*>(val), n, mean_row, rb, x, y, cs, st);
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
// With npart > 1 a launch covers part `part` of each XCD's row range (the ranges split
// into npart consecutive pieces), so that the rows of X one XCD gathers in a launch fit
// its L2; the partials of launch `part` sit at part * gridDim.x in a row of npart *
// gridDim.x per column.
template <int S, typename V, typename PT, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm_s(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const V* __restrict__ val, int64_t n, const PT* __restrict__ X,
                                                   double* __restrict__ Y, CgState cs, int part, int npart) {
  constexpr int VW = 16 / sizeof(PT);
  constexpr int LE = S / VW;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cq = lane % LE;
  XcdRows rr = xcd_rows(n, wid, kBlock / kWave);
  if (npart > 1) {
    const int64_t x = blockIdx.x % 8, lo = n * x / 8, len = n * (x + 1) / 8 - lo;
    const int64_t sub = lo + len * part / npart;
    rr.first = sub + (rr.first - lo);
    rr.end = lo + len * (part + 1) / npart;
  }
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
    cs.partial[(int64_t)threadIdx.x * gridDim.x * npart + (int64_t)part * gridDim.x + blockIdx.x] = t;
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
                        const CgState& cs, hipStream_t st, int64_t blocks, int npart = 1) {
  if ((S != 8 && S != 16 && S != 32 && S != 64) || (reinterpret_cast<uintptr_t>(X) & 15) != 0) return false;
  dim3 grid((unsigned)blocks), block(kBlock);
  for (int part = 0; part < npart; ++part) {
    switch (S) {
      case 8:
        hipLaunchKernelGGL((k_spmm_s<8, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs, part, npart);
        break;
      case 16:
        hipLaunchKernelGGL((k_spmm_s<16, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs, part, npart);
        break;
      case 32:
        hipLaunchKernelGGL((k_spmm_s<32, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs, part, npart);
        break;
      default:
        hipLaunchKernelGGL((k_spmm_s<64, V, PT, DOT>), grid, block, 0, st, rp, col, val, n, X, Y, cs, part, npart);
        break;
    }
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
// 5 block split (bsplit.hip), G in {4, 8, 16} entry-parallel with G lanes per row, -1 heuristic (entry-parallel up to 32
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
  } else if (G == 6) {
    // column slices in two launches over halves of each XCD's rows (L2-sized gathers)
    int64_t sb = grid_for(kBlock / kWave);
    if (sb > cap / 2) sb = round_up8(cap / 2 - 7);
    if (spmm_slices<V, PT, DOT>(rp, col, val, n, S, X, Y, cs, st, sb, 2)) {
      if (nblocks) *nblocks = (int)(2 * sb);
      return hipGetLastError();
    }
  } else if (G == 5) {
    if (spmm_split<V, PT, DOT>(rp, col, val, n, S, tiles, X, Y, cs, st, grid_for(kBlock / kWave), nblocks))
      return hipGetLastError();
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
                            void* Q, bool f32vec, const CgState& cs, hipStream_t st, const RowBlocks& rb) {
  int nb = 0;
  hipError_t e;
  if (S == 1) {
    // single right-hand side: always float64 vectors
    if (prec == GP2S_MIXED)
      e = spmv_dispatch<float, true>(rp, col, static_cast<const float*>(val), n, mean_row, rb,
                                     static_cast<const double*>(P), static_cast<double*>(Q), cs, st, &nb);
    else
      e = spmv_dispatch<double, true>(rp, col, static_cast<const double*>(val), n, mean_row, rb,
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
