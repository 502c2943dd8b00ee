// Far-field bump kernel (Sec. 4.3, Eq. bump_kernel, core kernel 1):
//
//   K = K_loc + G G^T,  K_loc = W(||x_i - x_j|| / r) + sigma_n^2 I (sparse, radius-local,
//   no bump mask),  G[i][u] = g_u(x_i) = sum over the bumps p of group u of a_p bhat_p(x_i).
//
// The bump term couples points at any distance but has rank U, so it is never formed:
// the CG product is K_loc P (the sparse kernels) plus G (G^T P), the block-Jacobi blocks
// add G_b G_b^T, and the amplitude gradient reduces to dot products with the columns
// of G. Every sum below is float64 with a fixed reduction order.
#include "gp2s_internal.h"
#include "pair.h"

namespace gp2s {

// G[i * U + u] (rows in the order of x) and, when diag is given, diag[i] += sum_u G^2.
__global__ __launch_bounds__(kBlock) void k_ff_G(int64_t n, int dim, const double* __restrict__ x,
                                                 const double* __restrict__ centers,
                                                 const double* __restrict__ weights,
                                                 const int32_t* __restrict__ group, int P, int U, double bump_w2,
                                                 double* __restrict__ G, double* __restrict__ diag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double g[kMaxGroups];
  for (int u = 0; u < U; ++u) g[u] = 0.0;
  for (int p = 0; p < P; ++p) {
    double d2 = 0.0;
    for (int k = 0; k < dim; ++k) {
      const double d = x[i * dim + k] - centers[p * dim + k];
      d2 += d * d;
    }
    if (d2 < bump_w2) g[group[p]] += weights[p] * exp(1.0 - 1.0 / (1.0 - d2 / bump_w2));
  }
  double s2 = 0.0;
  for (int u = 0; u < U; ++u) {
    G[i * U + u] = g[u];
    s2 += g[u] * g[u];
  }
  if (diag) diag[i] += s2;
}

// C[u * S + s] = sum_i G[i * U + u] X[i * S + s]: per-workgroup partials over a fixed
// row range, then the last workgroup (ticket) sums them in workgroup order.
// Thread t accumulates column s = t % S over rows t / S, t / S + 256 / S, ...
template <typename VEC>
__global__ __launch_bounds__(kBlock) void k_ff_gtp(int64_t n, int S, int U, const double* __restrict__ G,
                                                   const VEC* __restrict__ X, double* __restrict__ partial,
                                                   uint32_t* __restrict__ ticket, double* __restrict__ C) {
  __shared__ double sh[kBlock];
  __shared__ int am_last;
  const int t = threadIdx.x;
  const int per = kBlock / S;  // threads per column
  const int s = t % S, lane_row = t / S;
  const bool active = lane_row < per;
  const int64_t rows_per_wg = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * rows_per_wg;
  const int64_t r1 = r0 + rows_per_wg < n ? r0 + rows_per_wg : n;
  for (int u = 0; u < U; ++u) {
    double acc = 0.0;
    if (active)
      for (int64_t i = r0 + lane_row; i < r1; i += per) acc += G[i * U + u] * (double)X[i * S + s];
    sh[t] = acc;
    __syncthreads();
    if (t < S) {
      double v = 0.0;
      for (int k = 0; k < per; ++k) v += sh[k * S + t];
      partial[((int64_t)u * S + t) * gridDim.x + blockIdx.x] = v;
    }
    __syncthreads();
  }
  __threadfence();
  __syncthreads();
  if (t == 0) am_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  for (int e = t; e < U * S; e += blockDim.x) {
    double v = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b) v += partial[(int64_t)e * gridDim.x + b];
    C[e] = v;
  }
  if (t == 0) *ticket = 0u;
}

// Y[i * S + s] += sum_u G[i * U + u] C[u * cu + s * cs] (C read with strides so that a
// block of test rows of G* can serve as C without a transposed copy).
__global__ __launch_bounds__(kBlock) void k_ff_add(int64_t n, int S, int U, const double* __restrict__ G,
                                                   const double* __restrict__ C, int64_t cu, int64_t cs,
                                                   double* __restrict__ Y) {
  const int64_t total = n * (int64_t)S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / S;
    const int s = (int)(e - i * S);
    double v = 0.0;
    for (int u = 0; u < U; ++u) v += G[i * U + u] * C[u * cu + s * cs];
    Y[e] += v;
  }
}

// Trace vectors of the diagonal preconditioner, W[i * S + s] = z_s[i] / sqrt(K_ii).
__global__ void k_ff_wjac(int64_t n, int S, const uint64_t* __restrict__ mask, const double* __restrict__ dinv,
                          double* __restrict__ W) {
  const int64_t total = n * (int64_t)S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / S;
    const int s = (int)(e - i * S);
    const double d = sqrt(dinv[i]);
    W[e] = ((mask[i] >> s) & 1ull) ? -d : d;
  }
}

// H[i * U + u] = (P g_u)_i = a_i (a^T g_u) - (1/2S) sum_s (q_si (w_s^T g_u) + w_si (q_s^T g_u)),
// the row sums of the symmetrised weight P = a a^T - (1/2S) sum_s (q_s w_s^T + w_s q_s^T)
// against the far-field columns; dLML/da_p = sum_i bhat_p(x_i) H[i * U + group(p)].
__global__ __launch_bounds__(kBlock) void k_ff_h(int64_t n, int S, int U, const double* __restrict__ a,
                                                 const double* __restrict__ Q, const double* __restrict__ W,
                                                 const double* __restrict__ ag, const double* __restrict__ wg,
                                                 const double* __restrict__ qg, double* __restrict__ H) {
  const int64_t total = n * (int64_t)U;
  const double inv2S = 0.5 / (double)S;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / U;
    const int u = (int)(e - i * U);
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += Q[i * S + s] * wg[u * S + s] + W[i * S + s] * qg[u * S + s];
    H[e] = a[i] * ag[u] - inv2S * t;
  }
}

// Column maxima of |B[i * S + s]| over i (one workgroup per column; max is order-free),
// then B[:, s] /= c_s (c_s = 0 leaves the column zero).
__global__ __launch_bounds__(kBlock) void k_ff_colscale(int64_t n, int S, double* __restrict__ B,
                                                        double* __restrict__ cs) {
  __shared__ double sh[kBlock];
  const int s = blockIdx.x;
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(B[i * S + s]));
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const double c = sh[0];
  if (threadIdx.x == 0) cs[s] = c;
  if (!(c > 0.0)) return;
  const double inv = 1.0 / c;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) B[i * S + s] *= inv;
}

// var[t0 + s] = prior_s - c_s^2 sum_i B[i * S + s] V[i * S + s] (B scaled by 1 / c_s, V
// its solution), prior = 1 + sum_u G*[t0 + s]^2; one workgroup per column, fixed order.
__global__ __launch_bounds__(kBlock) void k_ff_var(int64_t n, int S, int U, const double* __restrict__ B,
                                                   const double* __restrict__ V, const double* __restrict__ cs,
                                                   const double* __restrict__ Gt, int64_t t0,
                                                   double* __restrict__ var) {
  __shared__ double sh[kBlock];
  const int s = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += B[i * S + s] * V[i * S + s];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double prior = 1.0;
    for (int u = 0; u < U; ++u) prior += Gt[(t0 + s) * U + u] * Gt[(t0 + s) * U + u];
    var[t0 + s] = prior - cs[s] * cs[s] * sh[0];
  }
}

static unsigned ew_blocks(int64_t total) {
  int64_t b = (total + kBlock - 1) / kBlock;
  if (b > (1 << 16)) b = 1 << 16;
  return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_ff_G(int64_t n, int dim, const double* x, const double* centers, const double* weights,
                       const int32_t* group, int P, int U, double bump_w2, double* G, double* diag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ff_G, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, dim, x, centers,
                     weights, group, P, U, bump_w2, G, diag);
  return hipGetLastError();
}

unsigned ff_gtp_blocks(int64_t n) {
  int64_t b = (n + 4 * kBlock - 1) / (4 * kBlock);
  if (b > 1024) b = 1024;
  return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_ff_gtp(int64_t n, int S, int U, const double* G, const void* X, bool f32, double* partial,
                         uint32_t* ticket, double* C, hipStream_t st) {
  const unsigned g = ff_gtp_blocks(n);
  if (f32)
    hipLaunchKernelGGL(k_ff_gtp<float>, dim3(g), dim3(kBlock), 0, st, n, S, U, G, static_cast<const float*>(X),
                       partial, ticket, C);
  else
    hipLaunchKernelGGL(k_ff_gtp<double>, dim3(g), dim3(kBlock), 0, st, n, S, U, G, static_cast<const double*>(X),
                       partial, ticket, C);
  return hipGetLastError();
}

hipError_t launch_ff_add(int64_t n, int S, int U, const double* G, const double* C, int64_t cu, int64_t cs, double* Y,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ff_add, dim3(ew_blocks(n * S)), dim3(kBlock), 0, st, n, S, U, G, C, cu, cs, Y);
  return hipGetLastError();
}

hipError_t launch_ff_wjac(int64_t n, int S, const uint64_t* mask, const double* dinv, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_ff_wjac, dim3(ew_blocks(n * S)), dim3(kBlock), 0, st, n, S, mask, dinv, W);
  return hipGetLastError();
}

hipError_t launch_ff_h(int64_t n, int S, int U, const double* a, const double* Q, const double* W, const double* ag,
                       const double* wg, const double* qg, double* H, hipStream_t st) {
  hipLaunchKernelGGL(k_ff_h, dim3(ew_blocks(n * U)), dim3(kBlock), 0, st, n, S, U, a, Q, W, ag, wg, qg, H);
  return hipGetLastError();
}

hipError_t launch_ff_colscale(int64_t n, int S, double* B, double* cs, hipStream_t st) {
  hipLaunchKernelGGL(k_ff_colscale, dim3(S), dim3(kBlock), 0, st, n, S, B, cs);
  return hipGetLastError();
}

hipError_t launch_ff_var(int64_t n, int S, int U, const double* B, const double* V, const double* cs,
                         const double* Gt, int64_t t0, double* var, hipStream_t st) {
  hipLaunchKernelGGL(k_ff_var, dim3(S), dim3(kBlock), 0, st, n, S, U, B, V, cs, Gt, t0, var);
  return hipGetLastError();
}

}  // namespace gp2s
