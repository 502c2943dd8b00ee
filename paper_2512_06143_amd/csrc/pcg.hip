// Jacobi-preconditioned conjugate gradients over a block of S independent columns,
// plus the small streaming kernels the runtime needs (permutations, dots, logs); the
// block-Jacobi update lives in blockjac.hip and shares the finalizers here.
//
// Per iteration: Q = K P (spmv.hip, yields alpha = r^T z / p^T q per column), then
// this file's update (x += alpha p, r -= alpha q, z = r / diag(K), new r^T z and
// r^T r, beta, convergence) and direction update (p = z + beta p). All sums are
// float64 and reduced in a fixed workgroup order. The alpha and beta of every
// iteration are kept: they are the Lanczos coefficients of the preconditioned
// operator used by the log-determinant quadrature (slq.hip).
#include "gp2s_internal.h"

namespace gp2s {

static inline int cols_block(int S) { return (kBlock / S) * S; }

// Per-column sums of the block's values (thread t belongs to column t % S), written to
// partial[(which * S + column) * gridDim + blockIdx] (column-major, so that the
// finalize kernels read each column's partials contiguously).
__device__ inline void block_cols_to_partial(double* sh, int S, double v, double* partial, int which) {
  const int nth = blockDim.x;
  const int per = nth / S;  // threads per column
  sh[threadIdx.x] = v;
  __syncthreads();
  if ((per & (per - 1)) == 0) {
    // power-of-two threads per column: tree over strides that keep columns aligned
    for (int o = (per / 2) * S; o >= S; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if ((int)threadIdx.x < S) partial[((int64_t)which * S + threadIdx.x) * gridDim.x + blockIdx.x] = sh[threadIdx.x];
  } else if ((int)threadIdx.x < S) {
    double t = 0.0;
    for (int k = threadIdx.x; k < nth; k += S) t += sh[k];
    partial[((int64_t)which * S + threadIdx.x) * gridDim.x + blockIdx.x] = t;
  }
  __syncthreads();
}

template <typename VEC>
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t n, int S, const double* __restrict__ B,
                                                    const double* __restrict__ dinv,
                                                    double* __restrict__ X, double* __restrict__ R,
                                                    VEC* __restrict__ P, CgState cs, double tol) {
  __shared__ double sh[kBlock];
  const int nth = blockDim.x;
  const int64_t total = n * (int64_t)S;
  double rz = 0.0, bb = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)nth + threadIdx.x; e < total; e += (int64_t)gridDim.x * nth) {
    const int64_t i = e / S;
    const double b = B[e];
    const double z = b * dinv[i];
    if (X) X[e] = 0.0;
    R[e] = b;
    P[e] = (VEC)z;
    rz += b * z;
    bb += b * b;
  }
  block_cols_to_partial(sh, S, rz, cs.partial, 0);
  block_cols_to_partial(sh, S, bb, cs.partial, 1);
}

// WANTX = false skips the solution update (the probe block of an LML without gradient
// needs only the CG coefficients).
template <typename VEC, bool WANTX>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, int S, double* __restrict__ X,
                                                      double* __restrict__ R, const VEC* __restrict__ P,
                                                      const double* __restrict__ Q,
                                                      const double* __restrict__ dinv, CgState cs,
                                                      int32_t iter) {
  __shared__ double sh[kBlock];
  const int nth = blockDim.x;
  const int64_t total = n * (int64_t)S;
  const int s_me = threadIdx.x % S;
  const double a = cs.alpha[s_me];
  double rz = 0.0, rr = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)nth + threadIdx.x; e < total; e += (int64_t)gridDim.x * nth) {
    const int64_t i = e / S;
    double r = R[e];
    if (a != 0.0) {
      if (WANTX) X[e] += a * (double)P[e];
      r -= a * Q[e];
      R[e] = r;
    }
    rz += r * (r * dinv[i]);
    rr += r * r;
  }
  block_cols_to_partial(sh, S, rz, cs.partial, 0);
  block_cols_to_partial(sh, S, rr, cs.partial, 1);
}

// ---- finalizers: one workgroup per column, fixed-order sums of the partials ----------
// Sum of partial[(which * S + s) * nb + b] over b < nb (all threads of the workgroup);
// W (partials per block and column) is implied by the layout and kept for clarity.
__device__ inline double column_sum(const double* partial, int nb, int W, int which, int S, int s, double* sh) {
  double v = 0.0;
  (void)W;
  const double* __restrict__ col = partial + ((int64_t)which * S + s) * nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) v += col[b];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double t = sh[0];
  __syncthreads();
  return t;
}

// alpha = r^T z / p^T q for every unfinished column; p^T q <= 0 flags a breakdown
// (flags[0] = 1, flags[3] = the column).
__global__ __launch_bounds__(kBlock) void k_cg_alpha(CgState cs, int nb, int S) {
  __shared__ double sh[kBlock];
  const int s = blockIdx.x;
  double pq = column_sum(cs.partial, nb, 1, 0, S, s, sh);
  if (threadIdx.x == 0) {
    if (cs.lrC)  // far-field kernel: p^T G G^T p = |G^T p|^2
      for (int u = 0; u < cs.lrU; ++u) pq += cs.lrC[u * S + s] * cs.lrC[u * S + s];
    double a = 0.0;
    if (!cs.done[s]) {
      if (!(pq > 0.0) || !isfinite(pq)) {
        cs.flags[0] = 1;
        cs.flags[3] = s;
      } else {
        a = cs.rz[s] / pq;
      }
    }
    cs.alpha[s] = a;
  }
}

__global__ __launch_bounds__(kBlock) void k_cg_init_fin(CgState cs, int nb, int S, double tol) {
  __shared__ double sh[kBlock];
  const int s = blockIdx.x;
  const double rz = column_sum(cs.partial, nb, 2, 0, S, s, sh);
  const double bb = column_sum(cs.partial, nb, 2, 1, S, s, sh);
  if (threadIdx.x == 0) {
    cs.rz[s] = rz;
    cs.bb[s] = bb;
    cs.rr[s] = bb;
    cs.tol2[s] = tol * tol;
    cs.iters[s] = 0;
    cs.alpha[s] = 0.0;
    cs.beta[s] = 0.0;
    cs.done[s] = (bb == 0.0) ? 1 : 0;
    if (!isfinite(rz) || !isfinite(bb)) cs.flags[2] = 1;
  }
}

// beta = new r^T z / old r^T z, coefficient history, convergence test.
__global__ __launch_bounds__(kBlock) void k_cg_beta(CgState cs, int nb, int S, int32_t iter) {
  __shared__ double sh[kBlock];
  const int s = blockIdx.x;
  const double rzn = column_sum(cs.partial, nb, 2, 0, S, s, sh);
  const double rrn = column_sum(cs.partial, nb, 2, 1, S, s, sh);
  if (threadIdx.x != 0) return;
  double beta = 0.0;
  if (!cs.done[s]) {
    const double al = cs.alpha[s];
    if (al == 0.0) {
      cs.done[s] = 1;  // breakdown (flagged by the product step)
    } else {
      beta = rzn / cs.rz[s];
      if (cs.hist_a && iter < cs.max_hist) {
        cs.hist_a[(int64_t)iter * S + s] = al;
        cs.hist_b[(int64_t)iter * S + s] = beta;
      }
      cs.iters[s] += 1;
      cs.rz[s] = rzn;
      cs.rr[s] = rrn;
      if (!isfinite(rrn)) {
        cs.flags[2] = 1;
        cs.done[s] = 1;
      } else if (rrn <= cs.tol2[s] * cs.bb[s]) {
        cs.done[s] = 1;
      }
    }
  }
  cs.beta[s] = beta;
}

hipError_t launch_cg_alpha(const CgState& cs, int nb, int S, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(S), dim3(kBlock), 0, st, cs, nb, S);
  return hipGetLastError();
}

template <typename VEC>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(int64_t n, int S, VEC* __restrict__ P,
                                                       const double* __restrict__ R,
                                                       const double* __restrict__ dinv, CgState cs) {
  const int nth = blockDim.x;
  const int64_t total = n * (int64_t)S;
  const int s_me = threadIdx.x % S;
  if (cs.done[s_me]) return;
  const double b = cs.beta[s_me];
  for (int64_t e = blockIdx.x * (int64_t)nth + threadIdx.x; e < total; e += (int64_t)gridDim.x * nth) {
    const int64_t i = e / S;
    const double z = dinv ? R[e] * dinv[i] : R[e];  // dinv == nullptr: R holds z = M^-1 r
    P[e] = (VEC)(z + b * (double)P[e]);
  }
}

// As k_cg_pupdate with z stored in float32 (the mixed path's block preconditioner:
// the search directions it forms are float32 anyway).
template <typename VEC>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate_z32(int64_t n, int S, VEC* __restrict__ P,
                                                           const float* __restrict__ Z, CgState cs) {
  const int nth = blockDim.x;
  const int64_t total = n * (int64_t)S;
  const int s_me = threadIdx.x % S;
  if (cs.done[s_me]) return;
  const double b = cs.beta[s_me];
  for (int64_t e = blockIdx.x * (int64_t)nth + threadIdx.x; e < total; e += (int64_t)gridDim.x * nth)
    P[e] = (VEC)((double)Z[e] + b * (double)P[e]);
}

static unsigned reduce_blocks(int64_t total, int nth) {
  int64_t b = (total + nth - 1) / nth;
  if (b > kReduceBlocks) b = kReduceBlocks;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Streaming CG kernels over n * S elements: enough workgroups to fill the chip,
// bounded by the partial-sum buffer.
static unsigned cg_blocks(int64_t total, int nth) {
  int64_t b = (total + 4 * (int64_t)nth - 1) / (4 * (int64_t)nth);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_cg_init(int64_t n, int S, const double* B, const double* dinv, double* X, double* R,
                          void* P, bool f32vec, const CgState& cs, double tol, hipStream_t st) {
  const int nth = cols_block(S);
  const unsigned nb = cg_blocks(n * S, nth);
  if (f32vec)
    hipLaunchKernelGGL(k_cg_init<float>, dim3(nb), dim3(nth), 0, st, n, S, B, dinv, X, R,
                       static_cast<float*>(P), cs, tol);
  else
    hipLaunchKernelGGL(k_cg_init<double>, dim3(nb), dim3(nth), 0, st, n, S, B, dinv, X, R,
                       static_cast<double*>(P), cs, tol);
  hipLaunchKernelGGL(k_cg_init_fin, dim3(S), dim3(kBlock), 0, st, cs, (int)nb, S, tol);
  return hipGetLastError();
}

hipError_t launch_cg_update(int64_t n, int S, double* X, double* R, const void* P, const void* Q, bool f32vec,
                            const double* dinv, const CgState& cs, int32_t iter, hipStream_t st) {
  const int nth = cols_block(S);
  const unsigned nb = cg_blocks(n * S, nth);
  const bool wx = X != nullptr;
  if (f32vec && wx)
    hipLaunchKernelGGL((k_cg_update<float, true>), dim3(nb), dim3(nth), 0, st, n, S, X, R,
                       static_cast<const float*>(P), static_cast<const double*>(Q), dinv, cs, iter);
  else if (f32vec)
    hipLaunchKernelGGL((k_cg_update<float, false>), dim3(nb), dim3(nth), 0, st, n, S, X, R,
                       static_cast<const float*>(P), static_cast<const double*>(Q), dinv, cs, iter);
  else if (wx)
    hipLaunchKernelGGL((k_cg_update<double, true>), dim3(nb), dim3(nth), 0, st, n, S, X, R,
                       static_cast<const double*>(P), static_cast<const double*>(Q), dinv, cs, iter);
  else
    hipLaunchKernelGGL((k_cg_update<double, false>), dim3(nb), dim3(nth), 0, st, n, S, X, R,
                       static_cast<const double*>(P), static_cast<const double*>(Q), dinv, cs, iter);
  hipLaunchKernelGGL(k_cg_beta, dim3(S), dim3(kBlock), 0, st, cs, (int)nb, S, iter);
  return hipGetLastError();
}

hipError_t launch_cg_init_fin(const CgState& cs, int nb, int S, double tol, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_init_fin, dim3(S), dim3(kBlock), 0, st, cs, nb, S, tol);
  return hipGetLastError();
}

hipError_t launch_cg_beta(const CgState& cs, int nb, int S, int32_t iter, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta, dim3(S), dim3(kBlock), 0, st, cs, nb, S, iter);
  return hipGetLastError();
}

hipError_t launch_cg_pupdate(int64_t n, int S, void* P, const double* R, const double* dinv, bool f32vec,
                             const CgState& cs, hipStream_t st) {
  const int nth = cols_block(S);
  int64_t blocks = (n * S + 4 * (int64_t)nth - 1) / (4 * (int64_t)nth);
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) blocks = 1;
  if (f32vec)
    hipLaunchKernelGGL(k_cg_pupdate<float>, dim3((unsigned)blocks), dim3(nth), 0, st, n, S,
                       static_cast<float*>(P), R, dinv, cs);
  else
    hipLaunchKernelGGL(k_cg_pupdate<double>, dim3((unsigned)blocks), dim3(nth), 0, st, n, S,
                       static_cast<double*>(P), R, dinv, cs);
  return hipGetLastError();
}

hipError_t launch_cg_pupdate_z32(int64_t n, int S, void* P, const float* Z, bool f32vec, const CgState& cs,
                                 hipStream_t st) {
  const int nth = cols_block(S);
  int64_t blocks = (n * S + 4 * (int64_t)nth - 1) / (4 * (int64_t)nth);
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) blocks = 1;
  if (f32vec)
    hipLaunchKernelGGL(k_cg_pupdate_z32<float>, dim3((unsigned)blocks), dim3(nth), 0, st, n, S,
                       static_cast<float*>(P), Z, cs);
  else
    hipLaunchKernelGGL(k_cg_pupdate_z32<double>, dim3((unsigned)blocks), dim3(nth), 0, st, n, S,
                       static_cast<double*>(P), Z, cs);
  return hipGetLastError();
}

// ---- small streaming kernels ----------------------------------------------------------
__global__ void k_axpy_sub(int64_t n, const double* __restrict__ b, const double* __restrict__ kx,
                           double* __restrict__ r) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - kx[i];
}
hipError_t launch_axpy_sub(int64_t n, const double* b, const double* kx, double* r, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_sub, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, b, kx, r);
  return hipGetLastError();
}

__global__ void k_add(int64_t n, double* __restrict__ x, const double* __restrict__ d) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += d[i];
}
hipError_t launch_add(int64_t n, double* x, const double* d, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, x, d);
  return hipGetLastError();
}

// out[0] = a^T b (b == nullptr: a^T a), deterministic two-level sum.
template <int MODE>  // 0: dot, 1: sum of logs
__global__ __launch_bounds__(kBlock) void k_reduce(int64_t n, const double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ out,
                                                   double* __restrict__ partial,
                                                   uint32_t* __restrict__ ticket) {
  __shared__ double sh[kBlock];
  __shared__ int am_last;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (MODE == 0) acc += a[i] * (b ? b[i] : a[i]);
    else acc += log(a[i]);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) am_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  reduce_partials(partial, gridDim.x, 1, sh, [&](int, double t) { out[0] = t; });
  if (threadIdx.x == 0) *ticket = 0u;
}

hipError_t launch_dot_partial(int64_t n, const double* a, const double* b, double* out, uint32_t* ticket,
                              hipStream_t st) {
  // out must have room for 1 + kReduceBlocks doubles (partials after the result).
  hipLaunchKernelGGL(k_reduce<0>, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, a, b, out,
                     out + 1, ticket);
  return hipGetLastError();
}

hipError_t launch_sum_log(int64_t n, const double* d, double* out, uint32_t* ticket, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce<1>, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, d, nullptr, out,
                     out + 1, ticket);
  return hipGetLastError();
}

__global__ void k_gather_rows(int64_t n, int S, const int32_t* __restrict__ perm,
                              const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t total = n * (int64_t)S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / S;
    const int s = (int)(e - p * S);
    const int64_t u = perm ? perm[p] : p;
    dst[e] = src[u * S + s];
  }
}
__global__ void k_scatter_rows(int64_t n, int S, const int32_t* __restrict__ perm,
                               const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t total = n * (int64_t)S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / S;
    const int s = (int)(e - p * S);
    const int64_t u = perm ? perm[p] : p;
    dst[u * S + s] = src[e];
  }
}
hipError_t launch_gather_rows(int64_t n, int S, const int32_t* perm, const double* src_user, double* dst_int,
                              hipStream_t st) {
  int64_t blocks = (n * S + kBlock - 1) / kBlock;
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, S, perm, src_user, dst_int);
  return hipGetLastError();
}
hipError_t launch_scatter_rows(int64_t n, int S, const int32_t* perm, const double* src_int, double* dst_user,
                               hipStream_t st) {
  int64_t blocks = (n * S + kBlock - 1) / kBlock;
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, S, perm, src_int, dst_user);
  return hipGetLastError();
}

// Probe right-hand sides D^{1/2} z_s (row-major [n * S]).
__global__ void k_probe_rhs(int64_t n, int S, const uint64_t* __restrict__ mask,
                            const double* __restrict__ diag, double* __restrict__ B) {
  const int64_t total = n * (int64_t)S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / S;
    const int s = (int)(e - p * S);
    const double sq = sqrt(diag[p]);
    B[e] = ((mask[p] >> s) & 1ull) ? -sq : sq;
  }
}
hipError_t launch_probe_rhs(int64_t n, int S, const uint64_t* mask, const double* diag, double* B,
                            hipStream_t st) {
  int64_t blocks = (n * S + kBlock - 1) / kBlock;
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_probe_rhs, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, S, mask, diag, B);
  return hipGetLastError();
}

__global__ void k_dinv(int64_t n, const double* __restrict__ diag, double* __restrict__ dinv,
                       int32_t* __restrict__ bad) {
  bool b = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = diag[i];
    if (!(d > 0.0) || !isfinite(d)) b = true;
    dinv[i] = 1.0 / d;
  }
  if (b) atomicOr(bad, 1);
}
hipError_t launch_dinv(int64_t n, const double* diag, double* dinv, int32_t* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_dinv, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, diag, dinv, bad);
  return hipGetLastError();
}

__global__ void k_check_finite(int64_t n, const double* __restrict__ v, int32_t* __restrict__ flag) {
  bool b = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(v[i])) b = true;
  if (b) atomicOr(flag, 1);
}
hipError_t launch_check_finite(int64_t n, const double* v, int32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_check_finite, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, v, flag);
  return hipGetLastError();
}

// Diagonal of a caller-supplied CSR (imported handles). Flags rows without a
// diagonal, column indices outside [0, n) or not strictly ascending, and row
// pointers that are not monotone from 0 to nnz; a flagged matrix is rejected
// before any product touches it.
template <typename V>
__global__ void k_extract_diag(int64_t n, int64_t nnz, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const V* __restrict__ val, double* __restrict__ diag, int32_t* __restrict__ bad) {
  bool b = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = rp[i], e = rp[i + 1];
    double d = 0.0;
    bool found = false;
    if (e < s || s < 0 || e > nnz || (i == 0 && s != 0) || (i == n - 1 && e != nnz)) {
      b = true;
      diag[i] = 0.0;
      continue;
    }
    for (int64_t k = s; k < e; ++k) {
      const int32_t c = col[k];
      if (c < 0 || c >= n || (k > s && c <= col[k - 1])) b = true;
      if (c == (int32_t)i) {
        d = (double)val[k];
        found = true;
      }
    }
    if (!found) b = true;
    diag[i] = d;
  }
  if (b) atomicOr(bad, 1);
}
hipError_t launch_extract_diag(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col, const void* val, int prec,
                               double* diag, int32_t* bad, hipStream_t st) {
  if (prec == GP2S_MIXED)
    hipLaunchKernelGGL(k_extract_diag<float>, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, nnz, rp, col,
                       static_cast<const float*>(val), diag, bad);
  else
    hipLaunchKernelGGL(k_extract_diag<double>, dim3(reduce_blocks(n, kBlock)), dim3(kBlock), 0, st, n, nnz, rp, col,
                       static_cast<const double*>(val), diag, bad);
  return hipGetLastError();
}

}  // namespace gp2s
