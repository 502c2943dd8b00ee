// Block-split multi-RHS product: K = B + R, B the 64 x 64 diagonal blocks of K over runs
// of 64 consecutive rows (dense, zero where K stores no entry), R every other stored
// entry. Consecutive rows of the internal order are spatial neighbours, so B holds about
// half of K's entries (53% on the 200 000-point uniform workload). Y = K X is then
//   1. R X: the column-slice gather product (spmm_rows.h) over each row's entries outside
//      its block, written to Y;
//   2. Y += B X_b per block on the float64 matrix cores: the block's 64 rows of X are read
//      once (one contiguous 64 x S tile) instead of once per stored entry, which removes
//      the gathers of B's entries, and the per-column p^T q partials of the CG are taken
//      here from the finished Y.
// Columns ascend within a row, so a row's in-block entries (columns r0 .. r0 + 63 of its
// block) form one contiguous run [s + lo, s + hi) of the row; R's entries are the row
// minus that run. Products of stored values with X accumulate in float64 in both parts
// (float32 values and directions are exact in float64), as in the other variants.
//
// Measured on the 200 000-point workload (64 float32 columns, inside CG): the column-slice
// product takes 0.235 ms; the split's R pass 0.190 ms for 47% of the entries plus 0.095 ms
// for the matrix-core pass. The in-block entries are the gathers that hit in cache (the
// same 64 rows of X serve a whole run of rows), so removing them saves little; the cost
// sits in the out-of-block gathers. The tuner therefore does not offer this variant; it
// can be pinned (gp2s_matrix_set_block_product).
#include "bj_apply.h"
#include "spmm_rows.h"

namespace gp2s {

// Per block: B in the operand order of the f64 16x16x4 instruction (wave w's 16 rows at
// w * 1024; for k-step kk lane l holds B[16w + l % 16][4kk + l / 16] at kk * 64 + l), and
// per row the run [lo, hi) of its in-block entries as offsets from the row start
// (lo = hi when the row has none). VALUES_ONLY refreshes B after a refill (the runs
// depend only on the pattern).
template <typename V, bool VALUES_ONLY>
__global__ __launch_bounds__(kBJThreads) void k_bs_build(int64_t n, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col, const V* __restrict__ val,
                                                         V* __restrict__ Bv, int2* __restrict__ seg) {
  __shared__ V A[kBJ * (kBJ + 1)];
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  const int64_t nblk = (n + kBJ - 1) / kBJ;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = blk * kBJ;
    const int m = (int)((n - r0) < kBJ ? (n - r0) : kBJ);
    for (int e = t; e < kBJ * (kBJ + 1); e += kBJThreads) A[e] = (V)0;
    __syncthreads();
    for (int i = wave; i < m; i += kBJThreads / kWave) {
      const int64_t s = rp[r0 + i], e = rp[r0 + i + 1];
      int lo = INT32_MAX, hi = -1;
      for (int64_t k = s + lane; k < e; k += kWave) {
        const int64_t c = (int64_t)col[k] - r0;
        if (c >= 0 && c < kBJ) {
          A[i * (kBJ + 1) + (int)c] = val[k];
          const int off = (int)(k - s);
          lo = off < lo ? off : lo;
          hi = off > hi ? off : hi;
        }
      }
      if (!VALUES_ONLY) {
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const int l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
          lo = l2 < lo ? l2 : lo;
          hi = h2 > hi ? h2 : hi;
        }
        if (lane == 0) seg[r0 + i] = hi < 0 ? make_int2(0, 0) : make_int2(lo, hi + 1);
      }
    }
    __syncthreads();
    V* Bb = Bv + blk * (int64_t)(kBJ * kBJ);
    for (int e = t; e < kBJ * kBJ; e += kBJThreads) {
      const int w = e >> 10, kk = (e >> 6) & 15, l = e & 63;
      Bb[e] = A[(16 * w + (l & 15)) * (kBJ + 1) + 4 * kk + (l >> 4)];
    }
    __syncthreads();
  }
}

// R X: one wave per row as k_spmm_s, over the row's entries before and after its
// in-block run.
template <int S, typename V, typename PT>
__global__ __launch_bounds__(kBlock) void k_spmm_sr(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                    const V* __restrict__ val, const int2* __restrict__ seg,
                                                    int64_t n, const PT* __restrict__ X, double* __restrict__ Y) {
  constexpr int VW = 16 / sizeof(PT);
  constexpr int LE = S / VW;
  const int lane = threadIdx.x & (kWave - 1);
  const int cq = lane % LE;
  const XcdRows rr = xcd_rows(n, threadIdx.x / kWave, kBlock / kWave);
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    const int64_t s = rp[row], e = rp[row + 1];
    const int2 sg = seg[row];
    double a1[VW], a2[VW];
    row_slices_product<S>(col, val, s, s + sg.x, lane, X, a1);
    row_slices_product<S>(col, val, s + sg.y, e, lane, X, a2);
    if (lane < LE) {
      const int64_t o = row * S + cq * VW;
#pragma unroll
      for (int c = 0; c < VW; ++c) Y[o + c] = a1[c] + a2[c];
    }
  }
}

// Y += B X_b for one block, on the matrix cores: Xs is the block's X in LDS ([row][column],
// column stride 64, rows past m and columns past S zero); wave w computes rows 16w .. 16w + 15.
// With DOT, adds X . Y (the finished row values) to dot[jt] for column 16 jt + lane % 16.
template <typename V, bool DOT>
__device__ inline void bs_apply_block(const double* Xs, const V* __restrict__ Bb, int m, int S, int64_t r0,
                                      double* __restrict__ Y, double (&dot)[kBJ / 16]) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int ntile = (S + 15) / 16;
  const V* F = Bb + wave * 1024;
  double af[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) af[kk] = (double)F[kk * 64 + lane];
  const int row_base = 16 * wave + (lane >> 4);
#pragma unroll
  for (int jt = 0; jt < kBJ / 16; ++jt) {
    if (jt < ntile) {
      const int c = 16 * jt + (lane & 15);
      v4d_bj acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double bv = c < S ? Xs[(4 * kk + (lane >> 4)) * kBJ + c] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk], bv, acc, 0, 0, 0);
      }
      if (c < S) {
        double part = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row_base + 4 * v;
          if (row < m) {
            const int64_t g = (r0 + row) * S + c;
            const double q = Y[g] + acc[v];
            Y[g] = q;
            if (DOT) part += Xs[row * kBJ + c] * q;
          }
        }
        if (DOT) dot[jt] += part;
      }
    }
  }
}

template <typename V, typename PT, bool DOT>
__global__ __launch_bounds__(kBJThreads) void k_spmm_bb(int64_t n, int S, const V* __restrict__ Bv,
                                                        const PT* __restrict__ X, double* __restrict__ Y,
                                                        CgState cs) {
  __shared__ double Xs[kBJ * kBJ];
  __shared__ double red[kBJThreads / kWave][kBJ];
  const int t = threadIdx.x;
  const int64_t nblk = (n + kBJ - 1) / kBJ;
  double dot[kBJ / 16] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = blk * kBJ;
    const int m = (int)((n - r0) < kBJ ? (n - r0) : kBJ);
    for (int e = t; e < kBJ * kBJ; e += kBJThreads) {
      const int i = e / kBJ, c = e % kBJ;
      Xs[e] = (i < m && c < S) ? (double)X[(r0 + i) * S + c] : 0.0;
    }
    __syncthreads();
    bs_apply_block<V, DOT>(Xs, Bv + blk * (int64_t)(kBJ * kBJ), m, S, r0, Y, dot);
    __syncthreads();
  }
  if (!DOT) return;
  const double tot = bj_rz_total<kBJThreads / kWave>(dot, red, S);
  if (t < S) cs.partial[(int64_t)t * gridDim.x + blockIdx.x] = tot;
}

hipError_t launch_bs_build(int64_t n, const int64_t* rp, const int32_t* col, const void* val, int prec, void* Bv,
                           int2* seg, bool values_only, hipStream_t st) {
  int64_t nblk = (n + kBJ - 1) / kBJ;
  const unsigned g = (unsigned)(nblk < 8192 ? (nblk < 1 ? 1 : nblk) : 8192);
#define GP2S_BSB(V, VO)                                                                                       \
  hipLaunchKernelGGL((k_bs_build<V, VO>), dim3(g), dim3(kBJThreads), 0, st, n, rp, col, static_cast<const V*>(val), \
                     static_cast<V*>(Bv), seg)
  if (prec == GP2S_MIXED) {
    if (values_only) GP2S_BSB(float, true);
    else GP2S_BSB(float, false);
  } else {
    if (values_only) GP2S_BSB(double, true);
    else GP2S_BSB(double, false);
  }
#undef GP2S_BSB
  return hipGetLastError();
}

// Both parts. The partials of p^T q (DOT) come from the matrix-core pass, whose grid
// (at most kDotBlocks workgroups) is returned in *nblocks.
template <typename V, typename PT, bool DOT>
bool spmm_split(const int64_t* rp, const int32_t* col, const V* val, int64_t n, int S, const TileSet& tiles,
                const PT* X, double* Y, const CgState& cs, hipStream_t st, int64_t row_blocks, int* nblocks) {
  if ((S != 8 && S != 16 && S != 32 && S != 64) || !tiles.bval || !tiles.bseg ||
      (reinterpret_cast<uintptr_t>(X) & 15) != 0)
    return false;
  const V* Bv = static_cast<const V*>(tiles.bval);
  dim3 grid((unsigned)row_blocks), block(kBlock);
  switch (S) {
    case 8: hipLaunchKernelGGL((k_spmm_sr<8, V, PT>), grid, block, 0, st, rp, col, val, tiles.bseg, n, X, Y); break;
    case 16: hipLaunchKernelGGL((k_spmm_sr<16, V, PT>), grid, block, 0, st, rp, col, val, tiles.bseg, n, X, Y); break;
    case 32: hipLaunchKernelGGL((k_spmm_sr<32, V, PT>), grid, block, 0, st, rp, col, val, tiles.bseg, n, X, Y); break;
    default: hipLaunchKernelGGL((k_spmm_sr<64, V, PT>), grid, block, 0, st, rp, col, val, tiles.bseg, n, X, Y); break;
  }
  int64_t nblk = (n + kBJ - 1) / kBJ;
  if (nblk > kDotBlocks) nblk = kDotBlocks;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL((k_spmm_bb<V, PT, DOT>), dim3((unsigned)nblk), dim3(kBJThreads), 0, st, n, S, Bv, X, Y, cs);
  if (nblocks) *nblocks = (int)nblk;
  return true;
}

template bool spmm_split<float, float, true>(const int64_t*, const int32_t*, const float*, int64_t, int,
                                             const TileSet&, const float*, double*, const CgState&, hipStream_t,
                                             int64_t, int*);
template bool spmm_split<float, float, false>(const int64_t*, const int32_t*, const float*, int64_t, int,
                                              const TileSet&, const float*, double*, const CgState&, hipStream_t,
                                              int64_t, int*);
template bool spmm_split<float, double, true>(const int64_t*, const int32_t*, const float*, int64_t, int,
                                              const TileSet&, const double*, double*, const CgState&, hipStream_t,
                                              int64_t, int*);
template bool spmm_split<float, double, false>(const int64_t*, const int32_t*, const float*, int64_t, int,
                                               const TileSet&, const double*, double*, const CgState&, hipStream_t,
                                               int64_t, int*);
template bool spmm_split<double, double, true>(const int64_t*, const int32_t*, const double*, int64_t, int,
                                               const TileSet&, const double*, double*, const CgState&, hipStream_t,
                                               int64_t, int*);
template bool spmm_split<double, double, false>(const int64_t*, const int32_t*, const double*, int64_t, int,
                                                const TileSet&, const double*, double*, const CgState&, hipStream_t,
                                                int64_t, int*);

}  // namespace gp2s
