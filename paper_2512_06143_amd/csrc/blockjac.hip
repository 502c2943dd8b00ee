// Block-Jacobi preconditioner of the CG solves: M = the block diagonal of K over runs
// of BJ consecutive rows of the internal (bin-sorted) order, M = L L^T blockwise (BJ = 128
// for a matrix handle, 64 for the instances of a batch).
//
// The log-determinant and trace estimators use M through its Cholesky factor (the
// probe right-hand sides are L z, the gradient's trace vectors L^-T z, and
// ln|K| = ln|M| + ln|L^-1 K L^-T|), so one kernel per matrix factors every block and
// stores, per block:
//   - L (row-major BJ x BJ, zero above the diagonal)      for the probe right-hand sides,
//   - M^-1 = L^-T L^-1 in the operand order of the f64 matrix-core instruction,
//   - the pivots L_ii^2 (sum of logs = ln|M|).
// Applying M^-1 to a BJ-row block of S residual columns is a dense BJ x BJ by BJ x S
// product: it runs on the matrix cores (v_mfma_f64_16x16x4), fused with the CG
// solution/residual update so that the residual block is read once.
//
// A ragged last block (n not a multiple of BJ) is padded with identity rows and
// columns; padded rows are never read or written outside the workgroup.
#include "bj_apply.h"

namespace gp2s {

constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;  // the GPU's last-level cache (MI355X)

constexpr int kBJStride = kBJ + 1;  // LDS row stride of the factor kernel (doubles)

// Block b: rows r0 .. r0 + m - 1; consecutive 64-row runs from row 0 unless a block list
// is given (the batched path: runs of 64 inside each instance).
__device__ inline int64_t bj_count(const BjBlocks& bl, int64_t n) { return bl.r0 ? bl.n : (n + kBJ - 1) / kBJ; }
__device__ inline int64_t bj_row0(const BjBlocks& bl, int64_t blk) { return bl.r0 ? bl.r0[blk] : blk * kBJ; }
__device__ inline int bj_rows(const BjBlocks& bl, int64_t n, int64_t blk) {
  if (bl.r0) return bl.m[blk];
  const int64_t r0 = blk * kBJ;
  return (int)((n - r0) < kBJ ? (n - r0) : kBJ);
}

// Operand order of M^-1 (per block, 4096 doubles): wave w = i / 16 owns rows
// 16w..16w+15; for k-step kk (columns 4kk..4kk+3) lane l holds M^-1[16w + l % 16][4kk + l / 16]
// at offset w * 1024 + kk * 64 + l, so every wave reads its operands as whole cache lines.
template <typename V>
__global__ __launch_bounds__(kBJThreads) void k_bj_factor(int64_t n, const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ col,
                                                          const V* __restrict__ val, const double* __restrict__ G,
                                                          int U, BjBlocks bl, double* __restrict__ Lout,
                                                          double* __restrict__ Mfrag, float* __restrict__ M32,
                                                          double* __restrict__ piv, int32_t* __restrict__ bad) {
  __shared__ double A[kBJ * kBJStride];   // block of K, then its factor L (lower part)
  __shared__ double Li[kBJ * kBJStride];  // L^-1 (lower part)
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  const int64_t nblk = bj_count(bl, n);
  bool failed = false;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = bj_row0(bl, blk);
    const int m = bj_rows(bl, n, blk);
    for (int e = t; e < kBJ * kBJ; e += kBJThreads) {
      const int i = e / kBJ, j = e % kBJ;
      A[i * kBJStride + j] = (i == j && i >= m) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int i = wave; i < m; i += kBJThreads / kWave) {
      const int64_t s = rp[r0 + i], e = rp[r0 + i + 1];
      for (int64_t k = s + lane; k < e; k += kWave) {
        const int64_t c = (int64_t)col[k] - r0;
        if (c >= 0 && c < m) A[i * kBJStride + (int)c] = (double)val[k];
      }
    }
    __syncthreads();
    if (G) {  // far-field kernel: the block of K_loc + G G^T
      for (int e = t; e < kBJ * kBJ; e += kBJThreads) {
        const int i = e / kBJ, j = e % kBJ;
        if (i < m && j < m) {
          double s = 0.0;
          for (int u = 0; u < U; ++u) s += G[(r0 + i) * U + u] * G[(r0 + j) * U + u];
          A[i * kBJStride + j] += s;
        }
      }
      __syncthreads();
    }
    // right-looking Cholesky on the lower triangle
    for (int k = 0; k < kBJ; ++k) {
      if (t == 0) {
        double d = A[k * kBJStride + k];
        if (!(d > 0.0) || !isfinite(d)) {
          failed = true;
          d = 1.0;
        }
        A[k * kBJStride + k] = sqrt(d);
      }
      __syncthreads();
      const double dk = A[k * kBJStride + k];
      for (int i = k + 1 + t; i < kBJ; i += kBJThreads) A[i * kBJStride + k] /= dk;
      __syncthreads();
      // trailing update of the lower triangle: wave w takes rows k+1+w, k+5+w, ..., its
      // lanes the columns of a row
      for (int i = k + 1 + wave; i < kBJ; i += kBJThreads / kWave) {
        const double lik = A[i * kBJStride + k];
        for (int j = k + 1 + lane; j <= i; j += kWave) A[i * kBJStride + j] -= lik * A[j * kBJStride + k];
      }
      __syncthreads();
    }
    if (t < m) {
      const double l = A[t * kBJStride + t];
      piv[r0 + t] = l * l;
    }
    double* Lb = Lout + blk * (int64_t)(kBJ * kBJ);
    for (int e = t; e < kBJ * kBJ; e += kBJThreads) {
      const int i = e / kBJ, j = e % kBJ;
      Lb[e] = j <= i ? A[i * kBJStride + j] : 0.0;
    }
    // L^-1 by forward substitution, one column per thread
    if (t < kBJ) {
      const int j = t;
      for (int i = 0; i < kBJ; ++i) {
        double v;
        if (i < j) {
          v = 0.0;
        } else if (i == j) {
          v = 1.0 / A[j * kBJStride + j];
        } else {
          // four independent partial sums, so that the LDS reads of a chain overlap
          double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
          int k = j;
          for (; k + 4 <= i; k += 4) {
            a0 += A[i * kBJStride + k] * Li[k * kBJStride + j];
            a1 += A[i * kBJStride + k + 1] * Li[(k + 1) * kBJStride + j];
            a2 += A[i * kBJStride + k + 2] * Li[(k + 2) * kBJStride + j];
            a3 += A[i * kBJStride + k + 3] * Li[(k + 3) * kBJStride + j];
          }
          for (; k < i; ++k) a0 += A[i * kBJStride + k] * Li[k * kBJStride + j];
          v = -((a0 + a1) + (a2 + a3)) / A[i * kBJStride + i];
        }
        Li[i * kBJStride + j] = v;
      }
    }
    __syncthreads();
    // M^-1[i][j] = sum_{k >= max(i, j)} Li[k][i] Li[k][j] (the same sum for (j, i): exactly symmetric)
    double* Mb = Mfrag + blk * (int64_t)(kBJ * kBJ);
    for (int e = t; e < kBJ * kBJ; e += kBJThreads) {
      const int w = e >> 10, kk = (e >> 6) & 15, l = e & 63;
      const int i = 16 * w + (l & 15), j = 4 * kk + (l >> 4);
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int k = i > j ? i : j;
      for (; k + 3 < kBJ; k += 4) {
        a0 += Li[k * kBJStride + i] * Li[k * kBJStride + j];
        a1 += Li[(k + 1) * kBJStride + i] * Li[(k + 1) * kBJStride + j];
        a2 += Li[(k + 2) * kBJStride + i] * Li[(k + 2) * kBJStride + j];
        a3 += Li[(k + 3) * kBJStride + i] * Li[(k + 3) * kBJStride + j];
      }
      for (; k < kBJ; ++k) a0 += Li[k * kBJStride + i] * Li[k * kBJStride + j];
      const double s = (a0 + a1) + (a2 + a3);
      Mb[e] = s;
      if (M32) M32[blk * (int64_t)(kBJ * kBJ) + e] = (float)s;
    }
    __syncthreads();
  }
  if (failed) atomicOr(bad, 1);
}

// The factor of one 128-row block for a matrix handle (consecutive 128-row runs from row
// 0). Two 128 x 129 float64 arrays would exceed the LDS, so the block is factored and then
// inverted in place: after the Cholesky factor L is written out, column j of L^-1 (for
// j = 127 down to 0) is formed from the columns of L^-1 to its right and column j of L,
// L^-1[i][j] = -(1 / L_jj) sum_{k = j+1..i} L^-1[i][k] L[k][j], L^-1[j][j] = 1 / L_jj.
// The far-field kernel adds its rank-U term to the block as in k_bj_factor.
template <typename V>
__global__ __launch_bounds__(kBJM * 4) void k_bj_factor_big(int64_t n, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const V* __restrict__ val, const double* __restrict__ G,
                                                           int U, double* __restrict__ Lout,
                                                           double* __restrict__ Mfrag, float* __restrict__ M32,
                                                           double* __restrict__ piv, int32_t* __restrict__ bad) {
  constexpr int B = kBJM, ST = kBJM + 1, NT = kBJM * 4;
  __shared__ double A[B * ST];  // the block of K, then L, then L^-1 (lower parts)
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  const int64_t nblk = (n + B - 1) / B;
  bool failed = false;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = blk * B;
    const int m = (int)((n - r0) < B ? (n - r0) : B);
    for (int e = t; e < B * B; e += NT) {
      const int i = e / B, j = e % B;
      A[i * ST + j] = (i == j && i >= m) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int i = wave; i < m; i += NT / kWave) {
      const int64_t s = rp[r0 + i], e = rp[r0 + i + 1];
      for (int64_t k = s + lane; k < e; k += kWave) {
        const int64_t c = (int64_t)col[k] - r0;
        if (c >= 0 && c < m) A[i * ST + (int)c] = (double)val[k];
      }
    }
    __syncthreads();
    if (G) {
      for (int e = t; e < B * B; e += NT) {
        const int i = e / B, j = e % B;
        if (i < m && j < m) {
          double acc = 0.0;
          for (int u = 0; u < U; ++u) acc += G[(r0 + i) * U + u] * G[(r0 + j) * U + u];
          A[i * ST + j] += acc;
        }
      }
      __syncthreads();
    }
    // right-looking Cholesky on the lower triangle
    for (int k = 0; k < B; ++k) {
      if (t == 0) {
        double d = A[k * ST + k];
        if (!(d > 0.0) || !isfinite(d)) {
          failed = true;
          d = 1.0;
        }
        A[k * ST + k] = sqrt(d);
      }
      __syncthreads();
      const double dk = A[k * ST + k];
      for (int i = k + 1 + t; i < B; i += NT) A[i * ST + k] /= dk;
      __syncthreads();
      // trailing update of the lower triangle: wave w takes rows k+1+w, k+1+w+8, ..., its
      // lanes the columns of a row
      for (int i = k + 1 + wave; i < B; i += NT / kWave) {
        const double lik = A[i * ST + k];
        for (int j = k + 1 + lane; j <= i; j += kWave) A[i * ST + j] -= lik * A[j * ST + k];
      }
      __syncthreads();
    }
    if (t < m) {
      const double l = A[t * ST + t];
      piv[r0 + t] = l * l;
    }
    double* Lb = Lout + blk * (int64_t)(B * B);
    for (int e = t; e < B * B; e += NT) {
      const int i = e / B, j = e % B;
      Lb[e] = j <= i ? A[i * ST + j] : 0.0;
    }
    __syncthreads();
    // L^-1 in place, column by column from the right
    for (int j = B - 1; j >= 0; --j) {
      const double ljj = A[j * ST + j];
      double v = 0.0;
      const int i = j + 1 + t;
      if (i < B) {
        // four independent partial sums, so that the LDS reads of a chain overlap
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int k = j + 1;
        for (; k + 3 <= i; k += 4) {
          a0 += A[i * ST + k] * A[k * ST + j];
          a1 += A[i * ST + k + 1] * A[(k + 1) * ST + j];
          a2 += A[i * ST + k + 2] * A[(k + 2) * ST + j];
          a3 += A[i * ST + k + 3] * A[(k + 3) * ST + j];
        }
        for (; k <= i; ++k) a0 += A[i * ST + k] * A[k * ST + j];
        v = -((a0 + a1) + (a2 + a3)) / ljj;
      }
      __syncthreads();
      if (i < B) A[i * ST + j] = v;
      if (t == 0) A[j * ST + j] = 1.0 / ljj;
      __syncthreads();
    }
    // M^-1[i][j] = sum_{k >= max(i, j)} L^-1[k][i] L^-1[k][j] (the same sum for (j, i)),
    // stored in operand order: wave w's 16 rows at w * 16 B, k-step kk at kk * 64 + lane
    double* Mb = Mfrag + blk * (int64_t)(B * B);
    for (int e = t; e < B * B; e += NT) {
      const int w = e / (16 * B), kk = (e >> 6) % (B / 4), l = e & 63;
      const int i = 16 * w + (l & 15), j = 4 * kk + (l >> 4);
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int k = i > j ? i : j;
      for (; k + 3 < B; k += 4) {
        a0 += A[k * ST + i] * A[k * ST + j];
        a1 += A[(k + 1) * ST + i] * A[(k + 1) * ST + j];
        a2 += A[(k + 2) * ST + i] * A[(k + 2) * ST + j];
        a3 += A[(k + 3) * ST + i] * A[(k + 3) * ST + j];
      }
      for (; k < B; ++k) a0 += A[k * ST + i] * A[k * ST + j];
      const double acc = (a0 + a1) + (a2 + a3);
      Mb[e] = acc;
      if (M32) M32[blk * (int64_t)(B * B) + e] = (float)acc;
    }
    __syncthreads();
  }
  if (failed) atomicOr(bad, 1);
}

// One CG update with the block preconditioner, per BJ-row block of a matrix handle:
//   INIT:  r = b, x = 0;  otherwise  x += alpha p, r -= alpha q   (columns with alpha = 0 keep r)
//   z = M^-1 r (matrix cores), and the per-column partials of r^T z (which 0) and r^T r (which 1).
// Thread t of the elementwise phase owns column t % S; waves own 16 rows of z each.
template <int BJ, int kU, typename VEC, bool WANTX, bool INIT, typename MT, typename ZT>
__global__ __launch_bounds__(BJ * 4) void k_bj_update(int64_t n, int S, const double* __restrict__ B,
                                                      double* __restrict__ X, double* __restrict__ R,
                                                      const VEC* __restrict__ P, const double* __restrict__ Q,
                                                      const MT* __restrict__ Mfrag, ZT* __restrict__ Z,
                                                      CgState cs) {
  constexpr int NT = BJ * 4;
  __shared__ double Rs[BJ * kRsStride];  // residual block [row][column], column stride 64
  __shared__ double red[NT / kWave][kRsStride];
  const int t = threadIdx.x;
  const int nth = (NT / S) * S;
  const int s_me = t % S;
  const double a = (INIT || t >= nth) ? 0.0 : cs.alpha[s_me];
  const int64_t nblk = (n + BJ - 1) / BJ;
  double rr = 0.0;
  double rz[kRsStride / 16] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = blk * BJ;
    const int m = (int)((n - r0) < BJ ? (n - r0) : BJ);
    if (t < nth) {
      // kU elements per thread and pass. Their loads are unconditional (elements past the
      // block's last row read its last element instead, and a finished column still reads
      // its p, q, x), so all 4 kU of them are in flight before the first use. kU = 4 pays
      // where the vectors sit in the Infinity Cache and the loads wait on latency; where
      // they stream from HBM the extra streams per wave cost more than they hide.
      const int elast = m * S - 1;
      for (int e0 = t; e0 < BJ * S; e0 += kU * nth) {
        double rv[kU], qv[kU], xv[kU];
        VEC pv[kU];  // converted where used
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int e = e0 + u * nth;
          const int64_t g = r0 * S + (e < elast ? e : elast);
          if (INIT) {
            rv[u] = B[g];
          } else {
            rv[u] = R[g];
            qv[u] = Q[g];
            if (WANTX) {
              pv[u] = P[g];
              xv[u] = X[g];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int e = e0 + u * nth;
          if (e < BJ * S) {
            const int i = e / S;
            double r = i < m ? rv[u] : 0.0;
            if (i < m) {
              const int64_t g = r0 * S + e;
              if (INIT) {
                R[g] = r;
                if (WANTX) X[g] = 0.0;
              } else if (a != 0.0) {
                if (WANTX) X[g] = xv[u] + a * (double)pv[u];
                r -= a * qv[u];
                R[g] = r;
              }
              rr += r * r;
            }
            Rs[i * kRsStride + s_me] = r;
          }
        }
      }
    }
    __syncthreads();
    bj_apply_block<BJ>(Rs, Mfrag + blk * (int64_t)(BJ * BJ), m, S, r0, Z, rz);
    __syncthreads();
  }
  // r^T z: lanes sharing a column (lane % 16) across row groups, then across waves
  const double rzt = bj_rz_total<NT / kWave>(rz, red, S);
  if (t < S) cs.partial[(int64_t)t * gridDim.x + blockIdx.x] = rzt;
  // r^T r: thread t holds column t % S (threads >= nth hold zero)
  Rs[t] = rr;
  __syncthreads();
  if (t < S) {
    double v = 0.0;
    for (int k = t; k < NT; k += S) v += Rs[k];
    cs.partial[((int64_t)S + t) * gridDim.x + blockIdx.x] = v;
  }
}

// Single-column form of the same update (the y and refinement solves, float64 search
// direction, z stored in float64). z = M^-1 r runs on the vector ALUs from the same
// operand-order M^-1: lane l of wave w holds row 16w + l % 16 at the columns congruent to
// l / 16 modulo 4, sums them against r from LDS, and the four lane groups combine by
// shuffles. The workgroup keeps only BJ doubles of r in LDS (the column-block form keeps
// BJ x 64), so many more workgroups stay resident, and the next block's M^-1 is loaded
// before the barrier that publishes r. Partials: r^T z at [b], r^T r at [gridDim + b].
template <int BJ, bool WANTX, bool INIT, typename MT>
__global__ __launch_bounds__(BJ * 4) void k_bj_update1(int64_t n, const double* __restrict__ B,
                                                       double* __restrict__ X, double* __restrict__ R,
                                                       const double* __restrict__ P, const double* __restrict__ Q,
                                                       const MT* __restrict__ Mfrag, double* __restrict__ Z,
                                                       CgState cs) {
  constexpr int NW = BJ * 4 / kWave;
  __shared__ double Rs[BJ];
  __shared__ double red[NW][2];
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  const int q = lane >> 4, row = 16 * wave + (lane & 15);
  const double a = INIT ? 0.0 : cs.alpha[0];
  const int64_t nblk = (n + BJ - 1) / BJ;
  double rr = 0.0, rz = 0.0;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = blk * BJ;
    const int m = (int)((n - r0) < BJ ? (n - r0) : BJ);
    const MT* F = Mfrag + blk * (int64_t)(BJ * BJ) + wave * (16 * BJ);
    MT af[BJ / 4];
#pragma unroll
    for (int kk = 0; kk < BJ / 4; ++kk) af[kk] = F[kk * 64 + lane];
    if (t < BJ) {
      double r = 0.0;
      if (t < m) {
        const int64_t g = r0 + t;
        if (INIT) {
          r = B[g];
          R[g] = r;
          if (WANTX) X[g] = 0.0;
        } else {
          r = R[g];
          if (a != 0.0) {
            if (WANTX) X[g] += a * P[g];
            r -= a * Q[g];
            R[g] = r;
          }
        }
        rr += r * r;
      }
      Rs[t] = r;
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < BJ / 4; ++kk) acc += (double)af[kk] * Rs[4 * kk + q];
    acc += __shfl_xor(acc, 16, kWave);
    acc += __shfl_xor(acc, 32, kWave);
    if (q == 0 && row < m) {
      Z[r0 + row] = acc;
      rz += Rs[row] * acc;
    }
    __syncthreads();  // Rs is rewritten by the next block
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    rz += __shfl_xor(rz, o, kWave);
    rr += __shfl_xor(rr, o, kWave);
  }
  if (lane == 0) {
    red[wave][0] = rz;
    red[wave][1] = rr;
  }
  __syncthreads();
  if (t < 2) {
    double v = 0.0;
    for (int w = 0; w < NW; ++w) v += red[w][t];
    cs.partial[(int64_t)t * gridDim.x + blockIdx.x] = v;
  }
}

// Probe right-hand sides B = L z (z = +-1 from the sign masks), per block of BJ rows.
template <int BJ>
__global__ __launch_bounds__(kBJThreads) void k_bj_rhs(int64_t n, int S, BjBlocks bl, const uint64_t* __restrict__ mask,
                                                       const double* __restrict__ Lg, double* __restrict__ B) {
  __shared__ double Ls[BJ * BJ];
  __shared__ uint64_t ms[BJ];
  const int t = threadIdx.x;
  const int64_t nblk = bl.r0 ? bl.n : (n + BJ - 1) / BJ;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t r0 = bl.r0 ? bl.r0[blk] : blk * BJ;
    const int m = bl.r0 ? bl.m[blk] : (int)((n - r0) < BJ ? (n - r0) : BJ);
    const double* Lb = Lg + blk * (int64_t)(BJ * BJ);
    for (int e = t; e < BJ * BJ; e += kBJThreads) Ls[e] = Lb[e];
    for (int k = t; k < BJ; k += kBJThreads) ms[k] = k < m ? mask[r0 + k] : 0ull;
    __syncthreads();
    for (int e = t; e < m * S; e += kBJThreads) {
      const int i = e / S, s = e % S;
      double v = 0.0;
      for (int k = 0; k <= i; ++k) {
        const double l = Ls[i * BJ + k];
        v += ((ms[k] >> s) & 1ull) ? -l : l;
      }
      B[r0 * S + e] = v;
    }
    __syncthreads();
  }
}

template <typename VEC>
__global__ void k_copy_dir(int64_t total, const double* __restrict__ Z, VEC* __restrict__ P) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    P[e] = (VEC)Z[e];
}

static unsigned bj_grid_blocks(int64_t nblk, int64_t cap) {
  if (nblk > cap) nblk = cap;
  if (nblk < 1) nblk = 1;
  return (unsigned)nblk;
}
static unsigned bj_grid(int64_t n, int64_t cap, int bj) { return bj_grid_blocks((n + bj - 1) / bj, cap); }
static int64_t bj_count_host(const BjBlocks& bl, int64_t n, int bj) { return bl.r0 ? bl.n : (n + bj - 1) / bj; }

hipError_t launch_bj_factor(int64_t n, const int64_t* rp, const int32_t* col, const void* val, int prec,
                            const double* G, int U, double* L, double* Mfrag, float* M32, double* piv, int32_t* bad,
                            hipStream_t st, const BjBlocks& bl, int bj) {
  if (bj == kBJM) {
    if (bl.r0) return hipErrorInvalidValue;  // 128-row blocks are consecutive runs only
    const unsigned g = bj_grid_blocks(bj_count_host(bl, n, bj), 8192);
    if (prec == GP2S_MIXED)
      hipLaunchKernelGGL(k_bj_factor_big<float>, dim3(g), dim3(kBJM * 4), 0, st, n, rp, col,
                         static_cast<const float*>(val), G, U, L, Mfrag, M32, piv, bad);
    else
      hipLaunchKernelGGL(k_bj_factor_big<double>, dim3(g), dim3(kBJM * 4), 0, st, n, rp, col,
                         static_cast<const double*>(val), G, U, L, Mfrag, M32, piv, bad);
    return hipGetLastError();
  }
  const unsigned g = bj_grid_blocks(bj_count_host(bl, n, kBJ), 8192);
  if (prec == GP2S_MIXED)
    hipLaunchKernelGGL(k_bj_factor<float>, dim3(g), dim3(kBJThreads), 0, st, n, rp, col,
                       static_cast<const float*>(val), G, U, bl, L, Mfrag, M32, piv, bad);
  else
    hipLaunchKernelGGL(k_bj_factor<double>, dim3(g), dim3(kBJThreads), 0, st, n, rp, col,
                       static_cast<const double*>(val), G, U, bl, L, Mfrag, M32, piv, bad);
  return hipGetLastError();
}

unsigned bj_update_blocks(int64_t n, int bj) { return bj_grid(n, kDotBlocks, bj); }

hipError_t launch_bj_update(int64_t n, int S, const double* B, double* X, double* R, const void* P, const void* Q,
                            bool f32vec, const double* Mfrag, double* Z, const CgState& cs, hipStream_t st,
                            const float* M32, float* Z32, int bj) {
  const unsigned g = bj_update_blocks(n, bj);
  const bool wx = X != nullptr;
  const bool cached = (double)n * S * sizeof(double) <= kInfinityCacheBytes;
  const double* Qd = static_cast<const double*>(Q);
#define GP2S_BJU(BJ, U, VEC, WX, INIT)                                                                          \
  do {                                                                                                         \
    if (Z32)                                                                                                   \
      hipLaunchKernelGGL((k_bj_update<BJ, U, VEC, WX, INIT, double, float>), dim3(g), dim3(BJ * 4), 0, st, n,  \
                         S, B, X, R, static_cast<const VEC*>(P), Qd, Mfrag, Z32, cs);                         \
    else                                                                                                       \
      hipLaunchKernelGGL((k_bj_update<BJ, U, VEC, WX, INIT, double, double>), dim3(g), dim3(BJ * 4), 0, st, n, \
                         S, B, X, R, static_cast<const VEC*>(P), Qd, Mfrag, Z, cs);                           \
  } while (0)
#define GP2S_BJS(BJ, VEC, WX, INIT)       \
  do {                                    \
    if (cached)                           \
      GP2S_BJU(BJ, 4, VEC, WX, INIT);     \
    else                                  \
      GP2S_BJU(BJ, 1, VEC, WX, INIT);     \
  } while (0)
#define GP2S_BJ(VEC, WX, INIT)             \
  do {                                     \
    if (bj == kBJM)                        \
      GP2S_BJS(kBJM, VEC, WX, INIT);       \
    else                                   \
      GP2S_BJS(kBJ, VEC, WX, INIT);        \
  } while (0)
  if (S == 1 && !f32vec && !Z32) {
#define GP2S_BJ1(BJ, WX, INIT)                                                                                   \
  do {                                                                                                         \
    if (M32)                                                                                                   \
      hipLaunchKernelGGL((k_bj_update1<BJ, WX, INIT, float>), dim3(g), dim3(BJ * 4), 0, st, n, B, X, R,        \
                         static_cast<const double*>(P), Qd, M32, Z, cs);                                      \
    else                                                                                                       \
      hipLaunchKernelGGL((k_bj_update1<BJ, WX, INIT, double>), dim3(g), dim3(BJ * 4), 0, st, n, B, X, R,       \
                         static_cast<const double*>(P), Qd, Mfrag, Z, cs);                                    \
  } while (0)
#define GP2S_BJ1R(WX, INIT)          \
  do {                               \
    if (bj == kBJM)                  \
      GP2S_BJ1(kBJM, WX, INIT);      \
    else                             \
      GP2S_BJ1(kBJ, WX, INIT);       \
  } while (0)
    if (B) {
      if (wx) GP2S_BJ1R(true, true);
      else GP2S_BJ1R(false, true);
    } else {
      if (wx) GP2S_BJ1R(true, false);
      else GP2S_BJ1R(false, false);
    }
#undef GP2S_BJ1R
#undef GP2S_BJ1
  } else if (M32) {
    return hipErrorInvalidValue;  // the float32 M^-1 serves single-column solves only
  } else if (B) {
    if (wx) GP2S_BJ(double, true, true);
    else GP2S_BJ(double, false, true);
  } else if (f32vec) {
    if (wx) GP2S_BJ(float, true, false);
    else GP2S_BJ(float, false, false);
  } else {
    if (wx) GP2S_BJ(double, true, false);
    else GP2S_BJ(double, false, false);
  }
#undef GP2S_BJU
#undef GP2S_BJS
#undef GP2S_BJ
  return hipGetLastError();
}

hipError_t launch_bj_rhs(int64_t n, int S, const uint64_t* mask, const double* L, double* B, hipStream_t st,
                         const BjBlocks& bl, int bj) {
  const dim3 g(bj_grid_blocks(bj_count_host(bl, n, bj), 8192));
  if (bj == kBJM) {
    if (bl.r0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bj_rhs<kBJM>, g, dim3(kBJThreads), 0, st, n, S, bl, mask, L, B);
  } else {
    hipLaunchKernelGGL(k_bj_rhs<kBJ>, g, dim3(kBJThreads), 0, st, n, S, bl, mask, L, B);
  }
  return hipGetLastError();
}

hipError_t launch_copy_dir(int64_t n, int S, const double* Z, void* P, bool f32vec, hipStream_t st) {
  int64_t total = n * (int64_t)S;
  int64_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) return hipSuccess;
  if (f32vec)
    hipLaunchKernelGGL(k_copy_dir<float>, dim3((unsigned)blocks), dim3(kBlock), 0, st, total, Z,
                       static_cast<float*>(P));
  else
    hipLaunchKernelGGL(k_copy_dir<double>, dim3((unsigned)blocks), dim3(kBlock), 0, st, total, Z,
                       static_cast<double*>(P));
  return hipGetLastError();
}

}  // namespace gp2s
