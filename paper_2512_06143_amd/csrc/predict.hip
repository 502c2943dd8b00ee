// Posterior mean and variance of the latent function at test points (Sec. 3,
// Eq. posterior, zero prior mean):
//
//   mean_t = k(X, x*_t)^T a,                 a = K^{-1} y (kept from training, App. B.7)
//   var_t  = k(x*_t, x*_t) - k(X, x*_t)^T K^{-1} k(X, x*_t),   k(x*, x*) = g(x*)^2
//
// The cross-covariance K* (test rows x training columns, internal column order) is
// assembled like K: test points are binned on the training grid, each test row
// tests the training points of its 3^d neighbouring bins, and survivors are
// compacted into CSR with a wave ballot. The mean is one CSR SpMV of K* with a.
// The variance needs K^{-1} k(X, x*_t) for every test point: test points are
// solved 64 at a time as one block (preconditioned CG with the training matrix) whose
// right-hand sides are the scattered rows of K*, then var_t = g*_t^2 minus the dot of
// row t of K* with its solution column.
#include "gp2s_internal.h"
#include "pair.h"

namespace gp2s {

// Bump mask, support flag and bin of every test point, in the training path's point
// formats (w = g, or -1 outside every bump). Non-finite coordinates set *nonfinite.
__global__ __launch_bounds__(kBlock) void k_test_prologue(const double* __restrict__ x, int64_t nt, GridDev g,
                                                          const double* __restrict__ centers,
                                                          const double* __restrict__ weights, int P, double bump_w2,
                                                          float4* __restrict__ pts32, double4* __restrict__ pts64,
                                                          double* __restrict__ g64, int32_t* __restrict__ bin,
                                                          int32_t* __restrict__ nonfinite, int unit) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const int dim = g.dim;
  double xi[3] = {0.0, 0.0, 0.0};
  bool bad = false;
  for (int k = 0; k < dim; ++k) {
    xi[k] = x[i * dim + k];
    bad = bad || !isfinite(xi[k]);
  }
  if (bad) {
    atomicOr(nonfinite, 1);
    xi[0] = xi[1] = xi[2] = 0.0;
  }
  const int64_t b = bin_index(xi, g);
  double gs = 0.0;
  bool inside = false;
  bump_mask(xi, dim, centers, weights, P, bump_w2, gs, inside);
  if (unit) {  // far-field kernel: no bump mask on the Wendland term
    gs = 1.0;
    inside = true;
  }
  if (bad) inside = false;
  if (pts32) pts32[i] = make_float4((float)xi[0], (float)xi[1], (float)xi[2], inside ? (float)gs : pt_out_f32());
  if (pts64) pts64[i] = make_double4(xi[0], xi[1], xi[2], inside ? gs : pt_out_f64());
  g64[i] = inside ? gs : 0.0;
  bin[i] = (int32_t)b;
}

hipError_t launch_test_prologue(const double* x, int64_t nt, const GridDev& g, const double* centers,
                                const double* weights, int P, double bump_w2, float4* pts32, double4* pts64,
                                double* g64, int32_t* bin, int32_t* nonfinite, hipStream_t st, bool unit) {
  const int64_t blocks = (nt + kBlock - 1) / kBlock;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_test_prologue, dim3((unsigned)blocks), dim3(kBlock), 0, st, x, nt, g, centers, weights, P,
                     bump_w2, pts32, pts64, g64, bin, nonfinite, unit ? 1 : 0);
  return hipGetLastError();
}

// Count (FILL = false) or fill the cross-covariance rows: one wave per test row, the
// same candidate sequence and support test as the training assembly, without the
// diagonal (no test point is a training point, even where they coincide).
template <int DIM, bool FILL, bool F32>
__global__ __launch_bounds__(kBlock) void k_cross(CrossArgs a, int64_t nblocks_padded, int32_t* __restrict__ row_cnt,
                                                  const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                  void* __restrict__ val) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lb = xcd_block(nblocks_padded);
  const int64_t row = lb * (kBlock / kWave) + threadIdx.x / kWave;
  if (row >= a.nt) return;  // uniform per wave
  float4 pi32;
  double4 pi64;
  bool in_i;
  if (F32) {
    pi32 = a.test32[row];
    in_i = pt_in(pi32.w);
  } else {
    pi64 = a.test64[row];
    in_i = pt_in(pi64.w);
  }
  if (!in_i) {
    if (!FILL && lane == 0) row_cnt[row] = 0;
    return;
  }
  const int64_t base = FILL ? row_ptr[row] : 0;
  const int64_t end = FILL ? row_ptr[row + 1] : 0;
  int bx, by, bz;
  decode_bin<DIM>(a.test_bin[row], a.grid, bx, by, bz);
  const int nbx = a.grid.nb[0], nby = a.grid.nb[1], nbz = a.grid.nb[2];
  const int x0 = bx > 0 ? bx - 1 : 0;
  const int x1 = bx + 1 < nbx ? bx + 1 : nbx - 1;
  int64_t cnt = 0;
  const bool gen = a.kg.general != 0;
  const double li = a.lsq_test ? a.lsq_test[row] : 1.0;
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
    const int zz = bz + dz;
    if (zz < 0 || zz >= nbz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int yy = by + dy;
      if (yy < 0 || yy >= nby) continue;
      const int64_t rb = ((int64_t)zz * nby + yy) * nbx;
      const int64_t s = a.bin_start[rb + x0];
      const int64_t e = a.bin_start[rb + x1 + 1];
      for (int64_t c = s; c < e; c += kWave) {
        const int64_t j = c + lane;
        const bool ok = j < e;
        bool pass;
        float4 pj32;
        double4 pj64;
        const double lj = (a.kg.lsq && ok) ? a.kg.lsq[j] : 1.0;
        if (F32) {
          pj32 = ok ? a.pts32[j] : make_float4(0.f, 0.f, 0.f, pt_out_f32());
          pass = ok && pt_in(pj32.w) &&
                 (gen ? gen_pass_f32<DIM>(pi32, pj32, a.kg, li, lj) : sqdist_f32<DIM>(pi32, pj32) < a.r2f);
        } else {
          pj64 = ok ? a.pts64[j] : make_double4(0., 0., 0., pt_out_f64());
          pass = ok && pt_in(pj64.w) &&
                 (gen ? gen_pass_f64<DIM>(pi64, pj64, a.kg, li, lj) : sqdist_f64<DIM>(pi64, pj64) < a.r2);
        }
        const uint64_t m = __ballot(pass);
        const int64_t pos = base + cnt + lane_prefix(m);
        if (FILL && pass && pos < end) {  // never past the row counted by the first pass
          col[pos] = (int32_t)j;
          if (F32)
            static_cast<float*>(val)[pos] = gen ? gen_entry_f32<DIM>(pi32, pj32, a.kg, li, lj, a.kern)
                                                : entry_f32(pi32, pj32, a.r2, a.inv_r2, a.kern);
          else
            static_cast<double*>(val)[pos] = gen ? gen_entry_f64<DIM>(pi64, pj64, a.kg, li, lj, a.kern)
                                                 : entry_f64(pi64, pj64, a.r2, a.inv_r2, a.kern);
        }
        cnt += __popcll(m);
      }
    }
  }
  if (!FILL && lane == 0) row_cnt[row] = (int32_t)cnt;
}

template <bool FILL>
static hipError_t launch_cross_t(const CrossArgs& a, int prec, int32_t* row_cnt, const int64_t* row_ptr, int32_t* col,
                                 void* val, hipStream_t st) {
  const int rows_per_block = kBlock / kWave;
  const int64_t nblocks = (a.nt + rows_per_block - 1) / rows_per_block;
  if (nblocks == 0) return hipSuccess;
  const int64_t padded = (nblocks + 7) / 8 * 8;
  dim3 grid((unsigned)padded), block(kBlock);
  const bool f32 = prec == GP2S_MIXED;
  if (a.grid.dim == 2) {
    if (f32)
      hipLaunchKernelGGL((k_cross<2, FILL, true>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val);
    else
      hipLaunchKernelGGL((k_cross<2, FILL, false>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val);
  } else {
    if (f32)
      hipLaunchKernelGGL((k_cross<3, FILL, true>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val);
    else
      hipLaunchKernelGGL((k_cross<3, FILL, false>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val);
  }
  return hipGetLastError();
}

hipError_t launch_cross_count(const CrossArgs& a, int prec, int32_t* row_cnt, hipStream_t st) {
  return launch_cross_t<false>(a, prec, row_cnt, nullptr, nullptr, nullptr, st);
}
hipError_t launch_cross_fill(const CrossArgs& a, int prec, const int64_t* row_ptr, int32_t* col, void* val,
                             hipStream_t st) {
  return launch_cross_t<true>(a, prec, nullptr, row_ptr, col, val, st);
}

template <typename V>
__device__ inline double ldv(const void* val, int64_t k) {
  return (double)static_cast<const V*>(val)[k];
}

// B[j * S + s] = K*[t0 + s, j] / c_s for the S test rows of a block, c_s = max_j
// |K*[t0 + s, j]| (c_s = 0 leaves the column zero). The scaling keeps right-hand sides
// built from tiny bump values (which can sit near the float32 underflow threshold)
// well inside range for the float32 search directions; CG is invariant to it. B is
// zeroed beforehand; each column is written by one wave only.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_cross_block(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                        const void* __restrict__ val, int64_t t0, int S,
                                                        double* __restrict__ B, double* __restrict__ cs, int raw) {
  const int lane = threadIdx.x & (kWave - 1);
  const int s = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (s >= S) return;
  const int64_t b = rp[t0 + s], e = rp[t0 + s + 1];
  if (raw) {
    for (int64_t k = b + lane; k < e; k += kWave) B[(int64_t)col[k] * S + s] = ldv<V>(val, k);
    return;
  }
  double mx = 0.0;
  for (int64_t k = b + lane; k < e; k += kWave) mx = fmax(mx, fabs(ldv<V>(val, k)));
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if (lane == 0) cs[s] = mx;
  if (!(mx > 0.0)) return;
  const double inv = 1.0 / mx;
  for (int64_t k = b + lane; k < e; k += kWave) B[(int64_t)col[k] * S + s] = ldv<V>(val, k) * inv;
}

// var[t0 + s] = g*^2 - c_s sum_j K*[t0 + s, j] V[j * S + s] (V solves K V = B; one wave
// per test row; the lane partial sums are combined in a fixed order).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_cross_var(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      const void* __restrict__ val, int64_t t0, int S,
                                                      const double* __restrict__ Vs, const double* __restrict__ cs,
                                                      const double* __restrict__ g64t, double* __restrict__ var) {
  const int lane = threadIdx.x & (kWave - 1);
  const int s = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (s >= S) return;
  const int64_t b = rp[t0 + s], e = rp[t0 + s + 1];
  double acc = 0.0;
  for (int64_t k = b + lane; k < e; k += kWave) acc += ldv<V>(val, k) * Vs[(int64_t)col[k] * S + s];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) {
    const double gs = g64t[t0 + s];
    var[t0 + s] = gs * gs - cs[s] * acc;
  }
}

hipError_t launch_cross_block(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t t0, int S,
                              double* B, double* cs, hipStream_t st, bool raw) {
  const int blocks = (S + kBlock / kWave - 1) / (kBlock / kWave);
  if (prec == GP2S_MIXED)
    hipLaunchKernelGGL(k_cross_block<float>, dim3(blocks), dim3(kBlock), 0, st, rp, col, val, t0, S, B, cs, raw ? 1 : 0);
  else
    hipLaunchKernelGGL(k_cross_block<double>, dim3(blocks), dim3(kBlock), 0, st, rp, col, val, t0, S, B, cs, raw ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_cross_var(int prec, const int64_t* rp, const int32_t* col, const void* val, int64_t t0, int S,
                            const double* Vs, const double* cs, const double* g64t, double* var, hipStream_t st) {
  const int blocks = (S + kBlock / kWave - 1) / (kBlock / kWave);
  if (prec == GP2S_MIXED)
    hipLaunchKernelGGL(k_cross_var<float>, dim3(blocks), dim3(kBlock), 0, st, rp, col, val, t0, S, Vs, cs, g64t,
                       var);
  else
    hipLaunchKernelGGL(k_cross_var<double>, dim3(blocks), dim3(kBlock), 0, st, rp, col, val, t0, S, Vs, cs, g64t,
                       var);
  return hipGetLastError();
}

}  // namespace gp2s
