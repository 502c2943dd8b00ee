// Block-Jacobi preconditioner application shared by the single-matrix and batched CG
// updates: z = M^-1 r for one block of BJ rows (128 for a matrix handle, 64 for the
// instances of a batch) on the float64 matrix cores.
#pragma once

#include "gp2s_internal.h"

namespace gp2s {

typedef double v4d_bj __attribute__((ext_vector_type(4)));

constexpr int kBJThreads = 256;  // threads of a 64-row block kernel: four waves of 16 rows
constexpr int kRsStride = 64;    // column stride of the LDS residual block (S <= 64)

// Rs: the block's residual in LDS ([row][column], column stride kRsStride, rows past m
// zero); Mb: the block's M^-1 in operand order (wave w's 16 rows at w * 16 BJ: for k-step
// kk, lane l holds M^-1[16w + l % 16][4kk + l / 16] at kk * 64 + l). BJ / 16 waves; wave w
// writes z for its rows 16w .. 16w + 15 (those below m) to Z (rows from r0, row stride S)
// and adds this lane's share of r^T z for column 16 jt + lane % 16 to rz[jt].
// Operands of the f64 16x16x4 instruction: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16] of a 16 x 4 by 4 x 16 step; the result of lane l, register v, is row
// l / 16 + 4 v, column l % 16 of the 16 x 16 tile.
// MT: float64, or float32 for solves whose preconditioner does not enter an estimator
// (the y and refinement solves: a symmetric float32 rounding of M^-1 is still positive
// definite and halves the bytes that dominate a single-column update).
// ZT: the stored z (float64, or float32 where only the float32 search directions are
// formed from it); r^T z is taken from the float64 value either way.
template <int BJ, typename MT, typename ZT>
__device__ inline void bj_apply_block(const double* Rs, const MT* __restrict__ Mb, int m, int S, int64_t r0,
                                      ZT* __restrict__ Z, double (&rz)[kRsStride / 16]) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int ntile = (S + 15) / 16;
  const MT* F = Mb + wave * (16 * BJ);
  double af[BJ / 4];
#pragma unroll
  for (int kk = 0; kk < BJ / 4; ++kk) af[kk] = (double)F[kk * 64 + lane];
  const int row_base = 16 * wave + (lane >> 4);
#pragma unroll
  for (int jt = 0; jt < kRsStride / 16; ++jt) {
    if (jt < ntile) {
      const int c = 16 * jt + (lane & 15);
      v4d_bj acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < BJ / 4; ++kk) {
        const double bv = c < S ? Rs[(4 * kk + (lane >> 4)) * kRsStride + c] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk], bv, acc, 0, 0, 0);
      }
      if (c < S) {
        double part = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = row_base + 4 * v;
          if (row < m) {
            Z[(r0 + row) * S + c] = (ZT)acc[v];
            part += Rs[row * kRsStride + c] * acc[v];
          }
        }
        rz[jt] += part;
      }
    }
  }
}

// Workgroup totals of the rz[] partials (NW waves): thread t < S returns column t's r^T z
// (red is LDS scratch of NW rows of 64). Every thread of the workgroup calls it.
template <int NW>
__device__ inline double bj_rz_total(const double (&rz)[kRsStride / 16], double (*red)[kRsStride], int S) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int jt = 0; jt < kRsStride / 16; ++jt) {
    double v = rz[jt];
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    if (lane < 16) red[wave][16 * jt + lane] = v;
  }
  __syncthreads();
  double v = 0.0;
  if ((int)threadIdx.x < S)
    for (int w = 0; w < NW; ++w) v += red[w][threadIdx.x];
  __syncthreads();
  return v;
}

}  // namespace gp2s
