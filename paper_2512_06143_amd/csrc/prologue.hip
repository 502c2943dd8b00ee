// Per-point prologue and spatial binning (counting sort into a cell list).
//
// The paper evaluates every covariance entry in dense blocks (Sec. 4.6, App. B.7).
// Here the support of the kernel is known before evaluation: W vanishes beyond r
// (Sec. 4.1) and the bump mask vanishes outside every bump (Sec. 4.3). Points are
// therefore sorted into bins of side >= r so that each row only tests the points of
// its 3^d neighbouring bins.
#include "gp2s_internal.h"
#include "pair.h"

namespace gp2s {

// Bounding box and finiteness of the points. part[b*6 + k] = min of coordinate k,
// part[b*6 + 3 + k] = max, over the points handled by workgroup b.
__global__ __launch_bounds__(kBlock) void k_bbox(const double* __restrict__ x, int64_t n, int dim,
                                                 double* __restrict__ part,
                                                 int32_t* __restrict__ nonfinite) {
  __shared__ double smin[3][kBlock];
  __shared__ double smax[3][kBlock];
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int k = 0; k < dim; ++k) {
      double v = x[i * dim + k];
      if (!isfinite(v)) bad = true;
      lo[k] = fmin(lo[k], v);
      hi[k] = fmax(hi[k], v);
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  for (int k = 0; k < 3; ++k) {
    smin[k][threadIdx.x] = lo[k];
    smax[k][threadIdx.x] = hi[k];
  }
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int k = 0; k < 3; ++k) {
        smin[k][threadIdx.x] = fmin(smin[k][threadIdx.x], smin[k][threadIdx.x + s]);
        smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      part[blockIdx.x * 6 + k] = smin[k][0];
      part[blockIdx.x * 6 + 3 + k] = smax[k][0];
    }
  }
}

hipError_t launch_bbox(const double* x, int64_t n, int dim, double* part, int32_t* nonfinite,
                       int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_bbox, dim3(nblocks), dim3(kBlock), 0, st, x, n, dim, part, nonfinite);
  return hipGetLastError();
}


// Bin index, bump mask g (float64) and support flag gamma of every point (user order).
// g_i = sum_k a_k exp(1 - 1/(1 - s_ik)), s_ik = ||x_i - c_k||^2 / w^2, for s_ik < 1
// (Sec. 4.3, Eq. bump with shape parameter 1; g a sum of P bumps). gamma_i marks a
// point strictly inside at least one bump; the pattern uses gamma, not g != 0.
__global__ __launch_bounds__(kBlock) void k_prologue(const double* __restrict__ x, int64_t n,
                                                     GridDev g, const double* __restrict__ centers,
                                                     const double* __restrict__ weights, int P,
                                                     double bump_w2, int32_t* __restrict__ bin_of,
                                                     int32_t* __restrict__ slot,
                                                     int32_t* __restrict__ bin_count,
                                                     double* __restrict__ g64_user,
                                                     uint8_t* __restrict__ gam, uint32_t* __restrict__ fkey,
                                                     int unit) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int dim = g.dim;
  double xi[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) xi[k] = x[i * dim + k];
  const int64_t b = bin_index(xi, g);
  fkey[i] = sub_cell_code(xi, g, dim);
  double gsum = 0.0;
  bool inside = false;
  bump_mask(xi, dim, centers, weights, P, bump_w2, gsum, inside);
  if (unit) {  // far-field kernel: the Wendland term carries no bump mask
    gsum = 1.0;
    inside = true;
  }
  bin_of[i] = (int32_t)b;
  slot[i] = atomicAdd(&bin_count[b], 1);
  g64_user[i] = inside ? gsum : 0.0;
  gam[i] = inside ? 1 : 0;
}

hipError_t launch_prologue(const double* x, int64_t n, const GridDev& g, const double* centers,
                           const double* weights, int P, double bump_w2, int32_t* bin_of,
                           int32_t* slot, int32_t* bin_count, double* g64_user, uint8_t* gam,
                           uint32_t* fkey, hipStream_t st, bool unit) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_prologue, dim3((unsigned)blocks), dim3(kBlock), 0, st, x, n, g, centers,
                     weights, P, bump_w2, bin_of, slot, bin_count, g64_user, gam, fkey, unit ? 1 : 0);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, const int32_t* __restrict__ bin_of,
                                                    const int32_t* __restrict__ slot,
                                                    const uint32_t* __restrict__ fkey,
                                                    const int64_t* __restrict__ bin_start,
                                                    int32_t* __restrict__ perm_tmp,
                                                    uint32_t* __restrict__ key_tmp) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t pos = bin_start[bin_of[i]] + slot[i];
  perm_tmp[pos] = (int32_t)i;
  key_tmp[pos] = fkey[i];
}

hipError_t launch_scatter(int64_t n, const int32_t* bin_of, const int32_t* slot, const uint32_t* fkey,
                          const int64_t* bin_start, int32_t* perm_tmp, uint32_t* key_tmp, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, bin_of, slot, fkey,
                     bin_start, perm_tmp, key_tmp);
  return hipGetLastError();
}

// The atomic slots give an arbitrary order inside a bin. Make it deterministic: the
// final position of a point is its bin start plus the number of points of the same
// bin that precede it in (sub-cell code, user index) order, i.e. a counting sort by
// bin followed by a rank sort inside each bin.
__global__ __launch_bounds__(kBlock) void k_binsort(int64_t n, const int32_t* __restrict__ perm_tmp,
                                                    const uint32_t* __restrict__ key_tmp,
                                                    const int32_t* __restrict__ bin_of,
                                                    const int64_t* __restrict__ bin_start,
                                                    int32_t* __restrict__ perm) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t me = perm_tmp[p];
  const uint32_t mk = key_tmp[p];
  const int32_t b = bin_of[me];
  const int64_t s = bin_start[b], e = bin_start[b + 1];
  int64_t rank = 0;
  for (int64_t q = s; q < e; ++q) {
    const uint32_t k = key_tmp[q];
    rank += (k < mk || (k == mk && perm_tmp[q] < me)) ? 1 : 0;
  }
  perm[s + rank] = me;
}

hipError_t launch_binsort(int64_t n, const int32_t* perm_tmp, const uint32_t* key_tmp, const int32_t* bin_of,
                          const int64_t* bin_start, int32_t* perm, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_binsort, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, perm_tmp, key_tmp, bin_of,
                     bin_start, perm);
  return hipGetLastError();
}

// Internal-order copies: float point + g (or -1 for points outside every bump) for
// the float32 path, the same in float64 for the float64 path, float64 coordinates
// for the gradient, g in float64, and the bin index.
__global__ __launch_bounds__(kBlock) void k_gather_points(
    int64_t n, int dim, const double* __restrict__ x, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ bin_of, const double* __restrict__ g64_user,
    const uint8_t* __restrict__ gam, float4* __restrict__ pts32, double4* __restrict__ pts64,
    double* __restrict__ x64, double* __restrict__ g64, int32_t* __restrict__ binid) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  int32_t u = perm[p];
  double c[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) {
    c[k] = x[(int64_t)u * dim + k];
    x64[p * dim + k] = c[k];
  }
  double gv = g64_user[u];
  bool in = gam[u] != 0;
  if (pts32) pts32[p] = make_float4((float)c[0], (float)c[1], (float)c[2], in ? (float)gv : pt_out_f32());
  if (pts64) pts64[p] = make_double4(c[0], c[1], c[2], in ? gv : pt_out_f64());
  g64[p] = gv;
  binid[p] = bin_of[u];
}

// New bump weights on an assembled handle: g and the point records' w of every
// internal point from its stored coordinates. The support flag depends only on the
// centres and the width, which stay fixed, so the pattern is unchanged.
__global__ __launch_bounds__(kBlock) void k_refresh_g(int64_t n, int dim, const double* __restrict__ x64,
                                                      const double* __restrict__ centers,
                                                      const double* __restrict__ weights, int P, double bump_w2,
                                                      float4* __restrict__ pts32, double4* __restrict__ pts64,
                                                      double* __restrict__ g64) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  double xi[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) xi[k] = x64[p * dim + k];
  double gs = 0.0;
  bool inside = false;
  bump_mask(xi, dim, centers, weights, P, bump_w2, gs, inside);
  g64[p] = inside ? gs : 0.0;
  if (pts32) pts32[p].w = inside ? (float)gs : pt_out_f32();
  if (pts64) pts64[p].w = inside ? gs : pt_out_f64();
}

hipError_t launch_refresh_g(int64_t n, int dim, const double* x64, const double* centers, const double* weights,
                            int P, double bump_w2, float4* pts32, double4* pts64, double* g64, hipStream_t st) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_refresh_g, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, dim, x64, centers, weights, P,
                     bump_w2, pts32, pts64, g64);
  return hipGetLastError();
}

hipError_t launch_gather_points(int64_t n, int dim, const double* x, const int32_t* perm,
                                const int32_t* bin_of, const double* g64_user, const uint8_t* gam,
                                float4* pts32, double4* pts64, double* x64, double* g64,
                                int32_t* binid, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_gather_points, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, dim, x, perm,
                     bin_of, g64_user, gam, pts32, pts64, x64, g64, binid);
  return hipGetLastError();
}

// Length-scale field of the general kernel (Eq. wendconv): lsq_i = l(x_i)^2 with
// ln l(x) = sum_q c_q bhat_q(x), bhat_q the unweighted bumps (same centres and width as g).
__global__ __launch_bounds__(kBlock) void k_ell(int64_t n, int dim, const double* __restrict__ x,
                                                const double* __restrict__ centers, const double* __restrict__ ls_w,
                                                int P, double bump_w2, double* __restrict__ lsq) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xi[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) xi[k] = x[i * dim + k];
  double h = 0.0;
  bool inside = false;
  bump_mask(xi, dim, centers, ls_w, P, bump_w2, h, inside);  // sum_q c_q bhat_q(x)
  lsq[i] = exp(2.0 * h);
}

hipError_t launch_ell(int64_t n, int dim, const double* x, const double* centers, const double* ls_w, int P,
                      double bump_w2, double* lsq, hipStream_t st) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ell, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, dim, x, centers, ls_w, P, bump_w2, lsq);
  return hipGetLastError();
}

// Rademacher probe signs from counter-based SplitMix64 (Steele, Lea and Flood, 2014):
// output k of the stream seeded with `seed` is mix(seed + (k + 1) * 0x9E3779B97F4A7C15);
// probe s at user point u uses k = s * 2^40 + u and is negative when bit 63 is set.
// mask[p] holds the sign bits of all probes for internal point p.
__device__ inline uint64_t splitmix_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_probe_masks(int64_t n, const int32_t* __restrict__ perm,
                                                        uint64_t seed, int S,
                                                        uint64_t* __restrict__ mask) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint64_t u = perm ? (uint64_t)perm[p] : (uint64_t)p;
  uint64_t m = 0;
  for (int s = 0; s < S; ++s) {
    uint64_t z = splitmix_at(seed, ((uint64_t)s << 40) + u);
    m |= (z >> 63) << s;
  }
  mask[p] = m;
}

hipError_t launch_probe_masks(int64_t n, const int32_t* perm, uint64_t seed, int S, uint64_t* mask,
                              hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_probe_masks, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, perm, seed, S,
                     mask);
  return hipGetLastError();
}

}  // namespace gp2s
