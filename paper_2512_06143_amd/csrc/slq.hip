// Lanczos quadrature of z^T ln(Khat) z from the preconditioned-CG coefficients.
//
// The paper computes ln|K| on the host without naming the method ("LOGDET",
// Sec. 4.6, App. B.6). Here ln|K| = ln|M| + tr ln Khat, Khat = L^-1 K L^-T with
// M = L L^T the preconditioner (L = D^1/2, or the blockwise Cholesky factor), and
// tr ln Khat is estimated with Rademacher probes. Preconditioned CG on K q = L z is
// CG on Khat with initial residual z, i.e. Lanczos from z/||z||;
// its coefficients define the Lanczos tridiagonal T (m x m):
//   T_00 = 1/alpha_0,  T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1},
//   T_{k-1,k}^2 = beta_{k-1} / alpha_{k-1}^2,
// and z^T ln(Khat) z ~ ||z||^2 e_1^T ln(T) e_1 (Gauss quadrature).
//
// e_1^T ln(T) e_1 is evaluated without an eigendecomposition, from the identity
//   ln(lambda) = int_0^inf [1/(1+t) - 1/(lambda+t)] dt,  summed over T's spectrum:
//   e_1^T ln(T) e_1 = int_0^inf [1/(1+t) - e_1^T (T + tI)^-1 e_1] dt.
// With t = e^u the integrand decays exponentially in both directions and is analytic
// in the strip |Im u| < pi, so the trapezoidal rule in u converges geometrically
// (step 1/4: error ~ exp(-2 pi^2 / 0.25)). e_1^T (T + tI)^-1 e_1 = 1/d_0, where d comes
// from the bottom-up pivot recurrence d_{m-1} = T_{m-1,m-1} + t,
// d_k = T_kk + t - T_{k,k+1}^2 / d_{k+1}, which is stable because T + tI is positive
// definite. One workgroup per probe; lanes run independent quadrature nodes.
#include "gp2s_internal.h"

namespace gp2s {

constexpr double kSlqStep = 0.25;
constexpr int kSlqNodesPerThread = 4;

__global__ __launch_bounds__(kBlock) void k_slq(int S, const double* __restrict__ hist_a,
                                                const double* __restrict__ hist_b,
                                                const int32_t* __restrict__ iters,
                                                double* __restrict__ work, int64_t max_m,
                                                double* __restrict__ out) {
  const int s = blockIdx.x;
  const int m = iters[s];
  double* Td = work + (int64_t)s * 2 * max_m;
  double* E2 = Td + max_m;  // E2[k] = T_{k-1,k}^2 for k >= 1
  __shared__ double sh[kBlock];
  __shared__ double lam_hi_sh;
  if (m <= 0) {
    if (threadIdx.x == 0) out[s] = 0.0;
    return;
  }
  // Build T and a Gershgorin bound on its largest eigenvalue.
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    const double a = hist_a[(int64_t)k * S + s];
    double d = 1.0 / a;
    double e2 = 0.0;
    if (k > 0) {
      const double ap = hist_a[(int64_t)(k - 1) * S + s];
      const double bp = hist_b[(int64_t)(k - 1) * S + s];
      d += bp / ap;
      e2 = bp / (ap * ap);
    }
    Td[k] = d;
    E2[k] = e2;
  }
  __threadfence_block();
  __syncthreads();
  double gmax = 0.0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    double r = Td[k] + sqrt(E2[k]) + (k + 1 < m ? sqrt(E2[k + 1]) : 0.0);
    gmax = fmax(gmax, r);
  }
  sh[threadIdx.x] = gmax;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) lam_hi_sh = sh[0];
  __syncthreads();
  const double lam_hi = lam_hi_sh;
  // Integration range: beyond it the integrand is below ~1e-17 of its scale.
  const double u_hi = log(fmax(lam_hi, 1.0)) + 40.0;
  const double u_lo = log(fmin(lam_hi, 1.0)) - 69.1 - 40.0;  // condition numbers up to 1e30
  const int nodes = (int)((u_hi - u_lo) / kSlqStep) + 1;

  double acc = 0.0;
  for (int base = 0; base < nodes; base += blockDim.x * kSlqNodesPerThread) {
    double t[kSlqNodesPerThread], d[kSlqNodesPerThread];
    bool on[kSlqNodesPerThread];
#pragma unroll
    for (int q = 0; q < kSlqNodesPerThread; ++q) {
      const int node = base + q * blockDim.x + threadIdx.x;
      on[q] = node < nodes;
      t[q] = exp(u_lo + node * kSlqStep);
      d[q] = Td[m - 1] + t[q];
    }
    for (int k = m - 1; k >= 1; --k) {
      const double tk = Td[k - 1];
      const double e2 = E2[k];
#pragma unroll
      for (int q = 0; q < kSlqNodesPerThread; ++q) d[q] = tk + t[q] - e2 / d[q];
    }
#pragma unroll
    for (int q = 0; q < kSlqNodesPerThread; ++q)
      if (on[q]) acc += t[q] / (1.0 + t[q]) - t[q] / d[q];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[s] = sh[0] * kSlqStep;
}

// work must hold 2 * S * max(iters) doubles; the caller passes max_m.
hipError_t launch_slq_ws(int S, const double* hist_a, const double* hist_b, const int32_t* iters,
                         double* work, int64_t max_m, double* out, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slq, dim3(S), dim3(kBlock), 0, st, S, hist_a, hist_b, iters, work, max_m, out);
  return hipGetLastError();
}

}  // namespace gp2s
