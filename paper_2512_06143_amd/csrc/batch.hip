// Batched instances: many independent GP instances of uneven size solved as one
// block-diagonal system in the same launches.
//
// Assembly kernels work per row (each row knows its instance). The CG kernels use an
// instance-aligned decomposition: every workgroup owns up to kBRows consecutive rows
// of a single instance, so column sums, step lengths, convergence flags and Lanczos
// coefficients are kept per (instance, column) with fixed-order reductions and no
// atomics. The arithmetic of every step is the single-instance one (see
// prologue.hip, assemble.hip, spmv.hip, pcg.hip, backward.hip).
#include "bj_apply.h"
#include "pair.h"
#include "spmm_rows.h"

namespace gp2s {

__device__ inline int find_inst(const int64_t* rs, int M, int64_t u) {
  int lo = 0, hi = M;  // rs[lo] <= u < rs[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rs[mid] <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- prologue, binning, gathers ------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bbbox(const double* __restrict__ x3, BatchGeom g,
                                                  double* __restrict__ part, int32_t* __restrict__ nonfinite) {
  __shared__ double sh[6][kBlock];
  const int i = blockIdx.x;
  const int64_t r0 = g.row_start[i], r1 = g.row_start[i + 1];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t u = r0 + threadIdx.x; u < r1; u += blockDim.x) {
    for (int k = 0; k < 3; ++k) {
      const double v = x3[u * 3 + k];
      if (!isfinite(v)) bad = true;
      lo[k] = fmin(lo[k], v);
      hi[k] = fmax(hi[k], v);
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  for (int k = 0; k < 3; ++k) {
    sh[k][threadIdx.x] = lo[k];
    sh[3 + k][threadIdx.x] = hi[k];
  }
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = fmin(sh[k][threadIdx.x], sh[k][threadIdx.x + o]);
        sh[3 + k][threadIdx.x] = fmax(sh[3 + k][threadIdx.x], sh[3 + k][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[i * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_bbbox(const double* x3, const BatchGeom& g, double* part, int32_t* nonfinite, hipStream_t st) {
  hipLaunchKernelGGL(k_bbbox, dim3(g.M), dim3(kBlock), 0, st, x3, g, part, nonfinite);
  return hipGetLastError();
}

__device__ inline int32_t bcoord(double v, double o, double inv_h, int32_t nb) {
  const double f = floor((v - o) * inv_h);
  return (int32_t)fmax(0.0, fmin(f, (double)(nb - 1)));
}

__global__ __launch_bounds__(kBlock) void k_bprologue(const double* __restrict__ x3, BatchGeom g,
                                                      const double* __restrict__ centers3,
                                                      const double* __restrict__ weights,
                                                      int32_t* __restrict__ bin_of, int32_t* __restrict__ slot,
                                                      int32_t* __restrict__ bin_count,
                                                      double* __restrict__ g64_user, uint8_t* __restrict__ gam,
                                                      uint32_t* __restrict__ fkey) {
  const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= g.n) return;
  const int i = find_inst(g.row_start, g.M, u);
  const BInst& I = g.inst[i];
  const double xi[3] = {x3[u * 3], x3[u * 3 + 1], x3[u * 3 + 2]};
  int64_t b = 0;
  for (int k = 2; k >= 0; --k) b = b * I.grid.nb[k] + bcoord(xi[k], I.grid.origin[k], I.grid.inv_h[k], I.grid.nb[k]);
  fkey[u] = sub_cell_code(xi, I.grid, I.dim);
  double gs = 0.0;
  bool inside = false;
  for (int p = 0; p < I.P; ++p) {
    const double* c = centers3 + (int64_t)(I.cent0 + p) * 3;
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double d = xi[k] - c[k];
      d2 += d * d;
    }
    if (d2 < I.bump_w2) {
      inside = true;
      gs += weights[I.cent0 + p] * exp(1.0 - 1.0 / (1.0 - d2 / I.bump_w2));
    }
  }
  b += I.bin0;
  bin_of[u] = (int32_t)b;
  slot[u] = atomicAdd(&bin_count[b], 1);
  g64_user[u] = inside ? gs : 0.0;
  gam[u] = inside ? 1 : 0;
}

hipError_t launch_bprologue(const double* x3, const BatchGeom& g, const double* centers3, const double* weights,
                            int32_t* bin_of, int32_t* slot, int32_t* bin_count, double* g64_user, uint8_t* gam,
                            uint32_t* fkey, hipStream_t st) {
  const int64_t blocks = (g.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_bprologue, dim3((unsigned)blocks), dim3(kBlock), 0, st, x3, g, centers3, weights, bin_of,
                     slot, bin_count, g64_user, gam, fkey);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_bgather(const double* __restrict__ x3, BatchGeom g,
                                                    const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ bin_of,
                                                    const double* __restrict__ g64_user,
                                                    const uint8_t* __restrict__ gam, float4* __restrict__ pts32,
                                                    double4* __restrict__ pts64, double* __restrict__ x64,
                                                    double* __restrict__ g64, int32_t* __restrict__ binid,
                                                    int32_t* __restrict__ inst_of_row) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= g.n) return;
  const int64_t u = perm[p];
  const double c0 = x3[u * 3], c1 = x3[u * 3 + 1], c2 = x3[u * 3 + 2];
  x64[p * 3] = c0;
  x64[p * 3 + 1] = c1;
  x64[p * 3 + 2] = c2;
  const double gv = g64_user[u];
  const bool in = gam[u] != 0;
  if (pts32) pts32[p] = make_float4((float)c0, (float)c1, (float)c2, in ? (float)gv : pt_out_f32());
  if (pts64) pts64[p] = make_double4(c0, c1, c2, in ? gv : pt_out_f64());
  g64[p] = gv;
  binid[p] = bin_of[u];
  inst_of_row[p] = find_inst(g.row_start, g.M, u);
}

hipError_t launch_bgather(const double* x3, const BatchGeom& g, const int32_t* perm, const int32_t* bin_of,
                          const double* g64_user, const uint8_t* gam, float4* pts32, double4* pts64, double* x64,
                          double* g64, int32_t* binid, int32_t* inst_of_row, hipStream_t st) {
  const int64_t blocks = (g.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_bgather, dim3((unsigned)blocks), dim3(kBlock), 0, st, x3, g, perm, bin_of, g64_user, gam,
                     pts32, pts64, x64, g64, binid, inst_of_row);
  return hipGetLastError();
}

// ---- assembly ----------------------------------------------------------------------------------
__device__ inline float bsq32(const float4& a, const float4& b) {
  const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}
__device__ inline double bsq64(const double4& a, const double4& b) {
  const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return __fma_rn(dz, dz, __fma_rn(dy, dy, __dmul_rn(dx, dx)));
}
__device__ inline double bentry64(const double4& pi, const double4& pj, double r2, double inv_r2, int kern) {
  const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
  const double d2 = dx * dx + dy * dy + dz * dz;
  const double t = fmax((r2 - d2) * inv_r2, 0.0);
  const double rho = sqrt(d2 * inv_r2);
  const double om = t / (1.0 + rho);
  return pi.w * pj.w * wendland_w<double>(kern, rho, om);
}
// Float32-stored value: float64 evaluation, one rounding (see entry_f32).
__device__ inline float bentry32(const float4& pi, const float4& pj, double r2, double inv_r2, int kern) {
  return (float)bentry64(make_double4(pi.x, pi.y, pi.z, pi.w), make_double4(pj.x, pj.y, pj.z, pj.w), r2, inv_r2, kern);
}

__device__ inline uint32_t blane_prefix(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One wavefront per row, as in the single-instance assembly; the instance's grid, radius
// and noise come from its table entry, and neighbour runs reach +-m bins.
template <bool FILL, bool F32>
__global__ __launch_bounds__(kBlock) void k_bassemble(BAsm a, int64_t nblocks_padded, int32_t* __restrict__ row_cnt,
                                                      const int64_t* __restrict__ row_ptr,
                                                      int32_t* __restrict__ col, void* __restrict__ val,
                                                      double* __restrict__ diag, int32_t* __restrict__ overflow) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t per = nblocks_padded / 8;
  const int64_t lb = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t row = lb * (kBlock / kWave) + threadIdx.x / kWave;
  if (row >= a.g.n) return;
  const BInst& I = a.g.inst[a.g.inst_of_row[row]];
  float4 pi32;
  double4 pi64;
  bool in_i;
  if (F32) {
    pi32 = a.pts32[row];
    in_i = pt_in(pi32.w);
  } else {
    pi64 = a.pts64[row];
    in_i = pt_in(pi64.w);
  }
  const float r2f = (float)I.r2;
  const int64_t base = FILL ? row_ptr[row] : 0;
  const int64_t end = FILL ? min(row_ptr[row + 1], a.cap) : 0;
  if (FILL && lane == 0 && row_ptr[row + 1] > a.cap) atomicOr(overflow, 1);
  if (!in_i) {
    if (lane == 0) {
      if (FILL) {
        if (base < end) {
          col[base] = (int32_t)row;
          if (F32) {
            const float v = (float)I.noise;
            static_cast<float*>(val)[base] = v;
            diag[row] = (double)v;
          } else {
            static_cast<double*>(val)[base] = I.noise;
            diag[row] = I.noise;
          }
        }
      } else {
        row_cnt[row] = 1;
      }
    }
    return;
  }
  const int32_t lbin = (int32_t)(a.binid[row] - I.bin0);
  const int nbx = I.grid.nb[0], nby = I.grid.nb[1], nbz = I.grid.nb[2];
  const int bx = lbin % nbx, t = lbin / nbx, by = t % nby, bz = t / nby;
  const int m = I.m;
  const int x0 = max(bx - m, 0), x1 = min(bx + m, nbx - 1);
  const double gi64 = a.g64[row];
  int64_t cnt = 0;
  for (int dz = -m; dz <= m; ++dz) {
    const int zz = bz + dz;
    if (zz < 0 || zz >= nbz) continue;
    for (int dy = -m; dy <= m; ++dy) {
      const int yy = by + dy;
      if (yy < 0 || yy >= nby) continue;
      const int64_t rb = I.bin0 + ((int64_t)zz * nby + yy) * nbx;
      const int64_t s = a.bin_start[rb + x0], e = a.bin_start[rb + x1 + 1];
      for (int64_t c = s; c < e; c += kWave) {
        const int64_t j = c + lane;
        const bool ok = j < e;
        bool pass;
        float4 pj32;
        double4 pj64;
        if (F32) {
          pj32 = ok ? a.pts32[j] : make_float4(0.f, 0.f, 0.f, pt_out_f32());
          pass = ok && (j == row || (pt_in(pj32.w) && bsq32(pi32, pj32) < r2f));
        } else {
          pj64 = ok ? a.pts64[j] : make_double4(0., 0., 0., pt_out_f64());
          pass = ok && (j == row || (pt_in(pj64.w) && bsq64(pi64, pj64) < I.r2));
        }
        const uint64_t mk = __ballot(pass);
        const int64_t pos = base + cnt + blane_prefix(mk);
        if (FILL && pass && pos < end) {
          col[pos] = (int32_t)j;
          if (F32) {
            const float v = (j == row) ? (float)(gi64 * gi64 + I.noise) : bentry32(pi32, pj32, I.r2, I.inv_r2, I.kern);
            static_cast<float*>(val)[pos] = v;
            if (j == row) diag[row] = (double)v;
          } else {
            const double v = (j == row) ? gi64 * gi64 + I.noise : bentry64(pi64, pj64, I.r2, I.inv_r2, I.kern);
            static_cast<double*>(val)[pos] = v;
            if (j == row) diag[row] = v;
          }
        }
        cnt += __popcll(mk);
      }
    }
  }
  if (!FILL && lane == 0) row_cnt[row] = (int32_t)cnt;
}

template <bool FILL>
static hipError_t bassemble(const BAsm& a, int prec, int32_t* row_cnt, const int64_t* row_ptr, int32_t* col,
                            void* val, double* diag, int32_t* overflow, hipStream_t st) {
  const int64_t nb = (a.g.n + (kBlock / kWave) - 1) / (kBlock / kWave);
  const int64_t padded = (nb + 7) / 8 * 8;
  if (prec == GP2S_MIXED)
    hipLaunchKernelGGL((k_bassemble<FILL, true>), dim3((unsigned)padded), dim3(kBlock), 0, st, a, padded, row_cnt,
                       row_ptr, col, val, diag, overflow);
  else
    hipLaunchKernelGGL((k_bassemble<FILL, false>), dim3((unsigned)padded), dim3(kBlock), 0, st, a, padded, row_cnt,
                       row_ptr, col, val, diag, overflow);
  return hipGetLastError();
}
hipError_t launch_bassemble_count(const BAsm& a, int prec, int32_t* row_cnt, hipStream_t st) {
  return bassemble<false>(a, prec, row_cnt, nullptr, nullptr, nullptr, nullptr, nullptr, st);
}
hipError_t launch_bassemble_fill(const BAsm& a, int prec, const int64_t* row_ptr, int32_t* col, void* val,
                                 double* diag, int32_t* overflow, hipStream_t st) {
  return bassemble<true>(a, prec, nullptr, row_ptr, col, val, diag, overflow, st);
}

// Probe signs indexed by the instance-local user row (so each instance's probes are
// those of a single-instance run with the same seed).
__device__ inline uint64_t bsplitmix(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ __launch_bounds__(kBlock) void k_bprobe_masks(BatchGeom g, const int32_t* __restrict__ perm, uint64_t seed,
                                                         int S, uint64_t* __restrict__ mask) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= g.n) return;
  const int i = g.inst_of_row[p];
  const uint64_t u = (uint64_t)(perm[p] - g.row_start[i]);
  uint64_t mk = 0;
  for (int s = 0; s < S; ++s) mk |= (bsplitmix(seed, ((uint64_t)s << 40) + u) >> 63) << s;
  mask[p] = mk;
}
hipError_t launch_bprobe_masks(const BatchGeom& g, const int32_t* perm, uint64_t seed, int S, uint64_t* mask,
                               hipStream_t st) {
  const int64_t blocks = (g.n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_bprobe_masks, dim3((unsigned)blocks), dim3(kBlock), 0, st, g, perm, seed, S, mask);
  return hipGetLastError();
}

// ---- instance-aligned CG ------------------------------------------------------------------------
struct BRows {
  int inst;
  int64_t blk, lo, hi;
};
// Row block of this workgroup: the identity for set-up kernels (blk_map null), the
// compacted list of open instances' blocks inside the CG loop.
__device__ inline BRows brows(const BatchGeom& g) {
  BRows r;
  r.blk = g.blk_map ? (int64_t)g.blk_map[blockIdx.x] : (int64_t)blockIdx.x;
  r.inst = g.blk_inst[r.blk];
  const BInst& I = g.inst[r.inst];
  r.lo = I.row0 + (r.blk - I.blk0) * kBRows;
  r.hi = min(r.lo + (int64_t)kBRows, I.row0 + I.rows);
  return r;
}

// True when some column of instance i is still iterating (uniform over the workgroup).
__device__ inline bool inst_open(const CgState& cs, int i, int S) {
  return __syncthreads_or((int)threadIdx.x < S && !cs.done[i * S + threadIdx.x]) != 0;
}

// Q = K P for one instance-aligned workgroup; `L` lanes per row (a power of two >= S),
// 64 / L rows per wave side by side. Entries are exchanged inside a row's lane segment
// with shuffles. P may be float32; products accumulate and are stored in float64.
// Per-column p^T q partials go to partial[block * S + column].
template <int L, typename V, typename PT>
__global__ __launch_bounds__(kBlock) void k_bspmm(BatchGeom g, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const V* __restrict__ val, int S,
                                                  const PT* __restrict__ X, double* __restrict__ Y, CgState cs) {
  constexpr int U = L < 8 ? L : 8;
  const BRows br = brows(g);
  if (!inst_open(cs, br.inst, S)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int seg = lane / L, sl = lane % L;
  const int rows_per_pass = (kBlock / kWave) * (kWave / L);
  const int slot = wid * (kWave / L) + seg;
  const bool active = sl < S;
  const PT* __restrict__ Xl = X + (active ? sl : 0);
  double dot = 0.0;
  for (int64_t row = br.lo + slot; row < br.hi; row += rows_per_pass) {
    const int64_t s = rp[row], e = rp[row + 1];
    double acc = 0.0;
    for (int64_t k0 = s; k0 < e; k0 += L) {
      const int64_t k = k0 + sl;
      const int32_t off = k < e ? col[k] * S : 0;
      const V vj = k < e ? val[k] : (V)0;
      const int cnt = (int)min((int64_t)L, e - k0);
      // U gathers in flight per step; lanes past the row end hold (offset 0, value 0)
      for (int l = 0; l < cnt; l += U) {
        V vv[U];
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          vv[u] = __shfl(vj, l + u, L);
          xv[u] = (double)Xl[__shfl(off, l + u, L)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (double)vv[u] * xv[u];
      }
    }
    if (active) {
      Y[row * S + sl] = acc;
      dot += acc * (double)X[row * S + sl];
    }
  }
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = dot;
  __syncthreads();
  if ((int)threadIdx.x < S) {
    double t = 0.0;
    for (int q = 0; q < kBlock / L; ++q) t += sh[q * L + threadIdx.x];
    cs.partial[(int64_t)threadIdx.x * g.nblk + br.blk] = t;
  }
}

// Entry-parallel variant (spmm_rows.h) for S in {8, 16, 32, 64}: G lanes per row.
template <int G, int S, typename V, typename PT>
__global__ __launch_bounds__(kBlock) void k_bspmm_e(BatchGeom g, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col, const V* __restrict__ val,
                                                    const PT* __restrict__ X, double* __restrict__ Y, CgState cs) {
  constexpr int CW = S < 16 ? S : 16;
  constexpr int NP = S / CW;
  constexpr int OW = CW / G;
  const BRows br = brows(g);
  if (!inst_open(cs, br.inst, S)) return;
  const int lane = threadIdx.x % G;
  double dot[NP * OW];
#pragma unroll
  for (int j = 0; j < NP * OW; ++j) dot[j] = 0.0;
  for (int64_t row = br.lo + threadIdx.x / G; row < br.hi; row += kBlock / G) {
    const int64_t s = rp[row], e = rp[row + 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      double q[OW];
      row_cols_product<G, CW>(col, val, s, e, lane, X, S, p * CW, q);
      const int64_t o = row * S + p * CW + lane * OW;
#pragma unroll
      for (int j = 0; j < OW; ++j) {
        Y[o + j] = q[j];
        dot[p * OW + j] += q[j] * (double)X[o + j];
      }
    }
  }
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
    cs.partial[(int64_t)threadIdx.x * g.nblk + br.blk] = t;
  }
}

// Slice-per-lane variant (spmm_rows.h) for S in {8, 16, 32, 64}: one wave per row.
template <int S, typename V, typename PT>
__global__ __launch_bounds__(kBlock) void k_bspmm_s(BatchGeom g, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col, const V* __restrict__ val,
                                                    const PT* __restrict__ X, double* __restrict__ Y, CgState cs) {
  constexpr int VW = 16 / sizeof(PT);
  constexpr int LE = S / VW;
  const BRows br = brows(g);
  if (!inst_open(cs, br.inst, S)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int cq = lane % LE;
  double dot[VW];
#pragma unroll
  for (int c = 0; c < VW; ++c) dot[c] = 0.0;
  for (int64_t row = br.lo + wid; row < br.hi; row += kBlock / kWave) {
    double acc[VW];
    row_slices_product<S>(col, val, rp[row], rp[row + 1], lane, X, acc);
    if (lane < LE) {
      const int64_t o = row * S + cq * VW;
#pragma unroll
      for (int c = 0; c < VW; ++c) {
        Y[o + c] = acc[c];
        dot[c] += acc[c] * (double)X[o + c];
      }
    }
  }
  __shared__ double sh[kBlock / kWave][S];
  if (lane < LE)
#pragma unroll
    for (int c = 0; c < VW; ++c) sh[wid][cq * VW + c] = dot[c];
  __syncthreads();
  if ((int)threadIdx.x < S) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += sh[w][threadIdx.x];
    cs.partial[(int64_t)threadIdx.x * g.nblk + br.blk] = t;
  }
}

// single right-hand side per instance: G lanes per row
template <int G, typename V>
__global__ __launch_bounds__(kBlock) void k_bspmv(BatchGeom g, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const V* __restrict__ val,
                                                  const double* __restrict__ x, double* __restrict__ y, CgState cs) {
  const BRows br = brows(g);
  if (!inst_open(cs, br.inst, 1)) return;
  const int lane = threadIdx.x & (G - 1);
  const int grp = threadIdx.x / G;
  double dot = 0.0;
  for (int64_t row = br.lo + grp; row < br.hi; row += kBlock / G) {
    const int64_t s = rp[row], e = rp[row + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t k = s + lane;
    for (; k + 3 * G < e; k += 4 * G) {
      const int32_t c0 = col[k], c1 = col[k + G], c2 = col[k + 2 * G], c3 = col[k + 3 * G];
      const double v0 = (double)val[k], v1 = (double)val[k + G], v2 = (double)val[k + 2 * G],
                   v3 = (double)val[k + 3 * G];
      const double x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
      a0 += v0 * x0;
      a1 += v1 * x1;
      a2 += v2 * x2;
      a3 += v3 * x3;
    }
    for (; k < e; k += G) a0 += (double)val[k] * x[col[k]];
    double acc = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
    if (lane == 0) {
      y[row] = acc;
      dot += acc * x[row];
    }
  }
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = dot;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cs.partial[br.blk] = sh[0];
}

// Per-workgroup partials are stored column-major, partial[(which * S + s) * nblk + block],
// so one column's partials over an instance's workgroups are contiguous. Returns their sum.
__device__ inline double binst_sum(const BatchGeom& g, const double* partial, int i, int which, int S, int s,
                                   double* sh) {
  const BInst& I = g.inst[i];
  const double* __restrict__ part = partial + ((int64_t)which * S + s) * g.nblk;
  double v = 0.0;
  for (int64_t b = I.blk0 + threadIdx.x; b < I.blk0 + I.nblk; b += blockDim.x)
    v += part[b];
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

__global__ __launch_bounds__(kBlock) void k_bcg_alpha(BatchGeom g, CgState cs, int S) {
  __shared__ double sh[kBlock];
  const int c = blockIdx.x, i = c / S, s = c % S;
  if (cs.done[c]) {
    if (threadIdx.x == 0) cs.alpha[c] = 0.0;
    return;
  }
  const double pq = binst_sum(g, cs.partial, i, 0, S, s, sh);
  if (threadIdx.x == 0) {
    double a = 0.0;
    if (!(pq > 0.0) || !isfinite(pq)) {
      cs.flags[0] = 1;
      cs.flags[3] = c;
    } else {
      a = cs.rz[c] / pq;
    }
    cs.alpha[c] = a;
  }
}

template <int G, typename V>
static void bspmv_g(const BatchGeom& g, const int64_t* rp, const int32_t* col, const V* val, const double* P, double* Q,
                    const CgState& cs, hipStream_t st) {
  hipLaunchKernelGGL((k_bspmv<G, V>), dim3((unsigned)g.grid), dim3(kBlock), 0, st, g, rp, col, val, P, Q, cs);
}
template <int L, typename V, typename PT>
static void bspmm_l(const BatchGeom& g, const int64_t* rp, const int32_t* col, const V* val, int S, const PT* P,
                    double* Q, const CgState& cs, hipStream_t st) {
  hipLaunchKernelGGL((k_bspmm<L, V, PT>), dim3((unsigned)g.grid), dim3(kBlock), 0, st, g, rp, col, val, S, P, Q, cs);
}
template <typename V, typename PT>
static void bspmm_any(int lanes, const BatchGeom& g, const int64_t* rp, const int32_t* col, const V* val, int S,
                      const PT* P, double* Q, const CgState& cs, hipStream_t st) {
  switch (lanes) {
    case 2: bspmm_l<2>(g, rp, col, val, S, P, Q, cs, st); break;
    case 4: bspmm_l<4>(g, rp, col, val, S, P, Q, cs, st); break;
    case 8: bspmm_l<8>(g, rp, col, val, S, P, Q, cs, st); break;
    case 16: bspmm_l<16>(g, rp, col, val, S, P, Q, cs, st); break;
    case 32: bspmm_l<32>(g, rp, col, val, S, P, Q, cs, st); break;
    default: bspmm_l<64>(g, rp, col, val, S, P, Q, cs, st); break;
  }
}
template <typename V>
static void bspmv_any(int G, const BatchGeom& g, const int64_t* rp, const int32_t* col, const V* val, const double* P,
                      double* Q, const CgState& cs, hipStream_t st) {
  switch (G) {
    case 4: bspmv_g<4>(g, rp, col, val, P, Q, cs, st); break;
    case 8: bspmv_g<8>(g, rp, col, val, P, Q, cs, st); break;
    case 16: bspmv_g<16>(g, rp, col, val, P, Q, cs, st); break;
    case 32: bspmv_g<32>(g, rp, col, val, P, Q, cs, st); break;
    default: bspmv_g<64>(g, rp, col, val, P, Q, cs, st); break;
  }
}

template <typename V, typename PT>
static void bspmm_slices(const BatchGeom& g, const int64_t* rp, const int32_t* col, const V* val, int S,
                         const PT* P, double* Q, const CgState& cs, hipStream_t st) {
  dim3 grid((unsigned)g.grid), block(kBlock);
  switch (S) {
    case 8: hipLaunchKernelGGL((k_bspmm_s<8, V, PT>), grid, block, 0, st, g, rp, col, val, P, Q, cs); break;
    case 16: hipLaunchKernelGGL((k_bspmm_s<16, V, PT>), grid, block, 0, st, g, rp, col, val, P, Q, cs); break;
    case 32: hipLaunchKernelGGL((k_bspmm_s<32, V, PT>), grid, block, 0, st, g, rp, col, val, P, Q, cs); break;
    default: hipLaunchKernelGGL((k_bspmm_s<64, V, PT>), grid, block, 0, st, g, rp, col, val, P, Q, cs); break;
  }
}

// Entry-parallel block product with G lanes per row; false if S has no instance.
template <typename V, typename PT>
static bool bspmm_entry(int G, const BatchGeom& g, const int64_t* rp, const int32_t* col, const V* val, int S,
                        const PT* P, double* Q, const CgState& cs, hipStream_t st) {
  dim3 grid((unsigned)g.grid), block(kBlock);
#define GP2S_BSPMM_E(GG, SS)                                                                            \
  if (G == GG && S == SS) {                                                                            \
    hipLaunchKernelGGL((k_bspmm_e<GG, SS, V, PT>), grid, block, 0, st, g, rp, col, val, P, Q, cs);     \
    return true;                                                                                       \
  }
  GP2S_BSPMM_E(4, 8) GP2S_BSPMM_E(8, 8)
  GP2S_BSPMM_E(4, 16) GP2S_BSPMM_E(8, 16) GP2S_BSPMM_E(16, 16)
  GP2S_BSPMM_E(4, 32) GP2S_BSPMM_E(8, 32) GP2S_BSPMM_E(16, 32)
  GP2S_BSPMM_E(4, 64) GP2S_BSPMM_E(8, 64) GP2S_BSPMM_E(16, 64)
#undef GP2S_BSPMM_E
  return false;
}

// `lanes`: lanes per row -- the SpMV lane group for S = 1; for S > 1 the lanes per row
// of the lane-per-column product (>= S), 1 for the slice-per-lane product, or -G for
// the entry-parallel product with G lanes per row. Both are chosen by the autotuner.
hipError_t launch_bcg_matvec(int prec, const BatchGeom& g, const int64_t* rp, const int32_t* col, const void* val,
                             int S, int lanes, const void* P, void* Q, bool f32vec, const CgState& cs,
                             hipStream_t st) {
  if (S == 1) {
    if (prec == GP2S_MIXED)
      bspmv_any(lanes, g, rp, col, static_cast<const float*>(val), static_cast<const double*>(P),
                static_cast<double*>(Q), cs, st);
    else
      bspmv_any(lanes, g, rp, col, static_cast<const double*>(val), static_cast<const double*>(P),
                static_cast<double*>(Q), cs, st);
  } else if (lanes == 1 && (S == 8 || S == 16 || S == 32 || S == 64) && (f32vec || prec != GP2S_MIXED) &&
             (reinterpret_cast<uintptr_t>(P) & 15) == 0) {
    if (f32vec)
      bspmm_slices(g, rp, col, static_cast<const float*>(val), S, static_cast<const float*>(P),
                   static_cast<double*>(Q), cs, st);
    else
      bspmm_slices(g, rp, col, static_cast<const double*>(val), S, static_cast<const double*>(P),
                   static_cast<double*>(Q), cs, st);
  } else if (lanes < 0 && entry_product_ok(S, -lanes) && (f32vec || prec != GP2S_MIXED) &&
             (reinterpret_cast<uintptr_t>(P) & 15) == 0) {
    if (f32vec)
      bspmm_entry(-lanes, g, rp, col, static_cast<const float*>(val), S, static_cast<const float*>(P),
                  static_cast<double*>(Q), cs, st);
    else
      bspmm_entry(-lanes, g, rp, col, static_cast<const double*>(val), S, static_cast<const double*>(P),
                  static_cast<double*>(Q), cs, st);
  } else if (f32vec) {
    bspmm_any(lanes, g, rp, col, static_cast<const float*>(val), S, static_cast<const float*>(P),
              static_cast<double*>(Q), cs, st);
  } else if (prec == GP2S_MIXED) {
    bspmm_any(lanes, g, rp, col, static_cast<const float*>(val), S, static_cast<const double*>(P),
              static_cast<double*>(Q), cs, st);
  } else {
    bspmm_any(lanes, g, rp, col, static_cast<const double*>(val), S, static_cast<const double*>(P),
              static_cast<double*>(Q), cs, st);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bcg_alpha, dim3((unsigned)(g.M * S)), dim3(kBlock), 0, st, g, cs, S);
  return hipGetLastError();
}

// Per-column sums of one workgroup (thread t owns column t % S; S divides kBlock).
__device__ inline void bcols_partial(double* sh, int S, double v, double* partial, int64_t nblk, int64_t blk,
                                     int which) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kBlock / 2; o >= S; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if ((int)threadIdx.x < S) partial[((int64_t)which * S + threadIdx.x) * nblk + blk] = sh[threadIdx.x];
  __syncthreads();
}

template <typename VEC>
__global__ __launch_bounds__(kBlock) void k_bcg_init(BatchGeom g, int S, const double* __restrict__ B,
                                                     const double* __restrict__ dinv, double* __restrict__ X,
                                                     double* __restrict__ R, VEC* __restrict__ P, CgState cs) {
  __shared__ double sh[kBlock];
  const BRows br = brows(g);
  double rz = 0.0, bb = 0.0;
  for (int64_t e = br.lo * S + threadIdx.x; e < br.hi * S; e += kBlock) {
    const int64_t i = e / S;
    const double b = B[e];
    const double z = b * dinv[i];
    X[e] = 0.0;
    R[e] = b;
    P[e] = (VEC)z;
    rz += b * z;
    bb += b * b;
  }
  bcols_partial(sh, S, rz, cs.partial, g.nblk, br.blk, 0);
  bcols_partial(sh, S, bb, cs.partial, g.nblk, br.blk, 1);
}

__global__ __launch_bounds__(kBlock) void k_bcg_init_fin(BatchGeom g, CgState cs, int S, double tol) {
  __shared__ double sh[kBlock];
  const int c = blockIdx.x, i = c / S, s = c % S;
  const double rz = binst_sum(g, cs.partial, i, 0, S, s, sh);
  const double bb = binst_sum(g, cs.partial, i, 1, S, s, sh);
  if (threadIdx.x == 0) {
    cs.rz[c] = rz;
    cs.bb[c] = bb;
    cs.rr[c] = bb;
    cs.tol2[c] = tol * tol;
    cs.iters[c] = 0;
    cs.alpha[c] = 0.0;
    cs.beta[c] = 0.0;
    cs.done[c] = (bb == 0.0) ? 1 : 0;
    if (!isfinite(rz) || !isfinite(bb)) cs.flags[2] = 1;
  }
}

hipError_t launch_bcg_init(const BatchGeom& g, int S, const double* B, const double* dinv, double* X, double* R,
                           void* P, bool f32vec, const CgState& cs, double tol, hipStream_t st) {
  if (f32vec)
    hipLaunchKernelGGL(k_bcg_init<float>, dim3((unsigned)g.nblk), dim3(kBlock), 0, st, g, S, B, dinv, X, R,
                       static_cast<float*>(P), cs);
  else
    hipLaunchKernelGGL(k_bcg_init<double>, dim3((unsigned)g.nblk), dim3(kBlock), 0, st, g, S, B, dinv, X, R,
                       static_cast<double*>(P), cs);
  hipLaunchKernelGGL(k_bcg_init_fin, dim3((unsigned)(g.M * S)), dim3(kBlock), 0, st, g, cs, S, tol);
  return hipGetLastError();
}

template <typename VEC>
__global__ __launch_bounds__(kBlock) void k_bcg_update(BatchGeom g, int S, double* __restrict__ X,
                                                       double* __restrict__ R, const VEC* __restrict__ P,
                                                       const double* __restrict__ Q, const double* __restrict__ dinv,
                                                       CgState cs) {
  __shared__ double sh[kBlock];
  const BRows br = brows(g);
  if (!inst_open(cs, br.inst, S)) return;
  const int s_me = threadIdx.x % S;
  const double a = cs.alpha[br.inst * S + s_me];
  double rz = 0.0, rr = 0.0;
  for (int64_t e = br.lo * S + threadIdx.x; e < br.hi * S; e += kBlock) {
    const int64_t i = e / S;
    double r = R[e];
    if (a != 0.0) {
      X[e] += a * (double)P[e];
      r -= a * Q[e];
      R[e] = r;
    }
    rz += r * (r * dinv[i]);
    rr += r * r;
  }
  bcols_partial(sh, S, rz, cs.partial, g.nblk, br.blk, 0);
  bcols_partial(sh, S, rr, cs.partial, g.nblk, br.blk, 1);
}

__global__ __launch_bounds__(kBlock) void k_bcg_beta(BatchGeom g, CgState cs, int S, const int32_t* __restrict__ iter_dev) {
  __shared__ double sh[kBlock];
  const int c = blockIdx.x, i = c / S, s = c % S;
  if (cs.done[c]) {
    if (threadIdx.x == 0) cs.beta[c] = 0.0;
    return;
  }
  const double rzn = binst_sum(g, cs.partial, i, 0, S, s, sh);
  const double rrn = binst_sum(g, cs.partial, i, 1, S, s, sh);
  if (threadIdx.x != 0) return;
  const int32_t iter = *iter_dev;
  const int SM = g.M * S;
  double beta = 0.0;
  const double al = cs.alpha[c];
  if (al == 0.0) {
    cs.done[c] = 1;
  } else {
    beta = rzn / cs.rz[c];
    if (cs.hist_a && iter < cs.max_hist) {
      cs.hist_a[(int64_t)iter * SM + c] = al;
      cs.hist_b[(int64_t)iter * SM + c] = beta;
    }
    cs.iters[c] += 1;
    cs.rz[c] = rzn;
    cs.rr[c] = rrn;
    if (!isfinite(rrn)) {
      cs.flags[2] = 1;
      cs.done[c] = 1;
    } else if (rrn <= cs.tol2[c] * cs.bb[c]) {
      cs.done[c] = 1;
    }
  }
  cs.beta[c] = beta;
}

hipError_t launch_bcg_update(const BatchGeom& g, int S, double* X, double* R, const void* P, const void* Q, bool f32vec,
                             const double* dinv, const CgState& cs, const int32_t* iter_dev, hipStream_t st) {
  if (f32vec)
    hipLaunchKernelGGL(k_bcg_update<float>, dim3((unsigned)g.grid), dim3(kBlock), 0, st, g, S, X, R,
                       static_cast<const float*>(P), static_cast<const double*>(Q), dinv, cs);
  else
    hipLaunchKernelGGL(k_bcg_update<double>, dim3((unsigned)g.grid), dim3(kBlock), 0, st, g, S, X, R,
                       static_cast<const double*>(P), static_cast<const double*>(Q), dinv, cs);
  hipLaunchKernelGGL(k_bcg_beta, dim3((unsigned)(g.M * S)), dim3(kBlock), 0, st, g, cs, S, iter_dev);
  return hipGetLastError();
}

template <typename VEC>
__global__ __launch_bounds__(kBlock) void k_bcg_pupdate(BatchGeom g, int S, VEC* __restrict__ P,
                                                        const double* __restrict__ R, const double* __restrict__ dinv,
                                                        CgState cs, int32_t* __restrict__ iter_dev) {
  // The iteration counter advances once per iteration, after every reader of it.
  if (blockIdx.x == 0 && threadIdx.x == 0) *iter_dev += 1;
  const BRows br = brows(g);
  const int c = br.inst * S + (int)(threadIdx.x % S);
  if (cs.done[c]) return;
  const double b = cs.beta[c];
  for (int64_t e = br.lo * S + threadIdx.x; e < br.hi * S; e += kBlock) {
    const double z = dinv ? R[e] * dinv[e / S] : R[e];  // no dinv: R holds z = M^-1 r
    P[e] = (VEC)(z + b * (double)P[e]);
  }
}

hipError_t launch_bcg_pupdate(const BatchGeom& g, int S, void* P, const double* R, const double* dinv, bool f32vec,
                              const CgState& cs, int32_t* iter_dev, hipStream_t st) {
  if (f32vec)
    hipLaunchKernelGGL(k_bcg_pupdate<float>, dim3((unsigned)g.grid), dim3(kBlock), 0, st, g, S,
                       static_cast<float*>(P), R, dinv, cs, iter_dev);
  else
    hipLaunchKernelGGL(k_bcg_pupdate<double>, dim3((unsigned)g.grid), dim3(kBlock), 0, st, g, S,
                       static_cast<double*>(P), R, dinv, cs, iter_dev);
  return hipGetLastError();
}

// ---- block-Jacobi preconditioner ----------------------------------------------------------------
static_assert(kBRows == kBJ, "the batch's row blocks are the preconditioner's blocks");
// The batch's row blocks (64 rows of one instance, instance-aligned) are the
// preconditioner's blocks, factored by launch_bj_factor with the batch's block list. One
// CG update per workgroup and block: INIT r = b, x = 0; otherwise x += alpha p, r -=
// alpha q with the instance's alpha per column; then z = M^-1 r on the matrix cores and
// the per-column partials of r^T z (which 0) and r^T r (which 1) in the batch's layout.
template <typename VEC, bool INIT, typename MT>
__global__ __launch_bounds__(kBJThreads) void k_bbj_update(BatchGeom g, int S, const double* __restrict__ B,
                                                           double* __restrict__ X, double* __restrict__ R,
                                                           const VEC* __restrict__ P, const double* __restrict__ Q,
                                                           const MT* __restrict__ Mfrag, double* __restrict__ Z,
                                                           CgState cs) {
  __shared__ double Rs[kBJ * kBJ];  // residual block [row][column], column stride 64
  __shared__ double red[kBJThreads / kWave][kBJ];
  const BRows br = brows(g);
  if (!INIT && !inst_open(cs, br.inst, S)) return;
  const int t = threadIdx.x;
  const int nth = (kBJThreads / S) * S;
  const int s_me = t % S;
  const double a = (INIT || t >= nth) ? 0.0 : cs.alpha[br.inst * S + s_me];
  const int64_t r0 = br.lo;
  const int m = (int)(br.hi - br.lo);
  double rr = 0.0;
  double rz[kBJ / 16] = {0.0, 0.0, 0.0, 0.0};
  if (t < nth && m > 0) {
    // Four elements per thread and pass with unconditional loads (past the block's last
    // row, its last element is read instead; a finished column still reads p, q, x), so
    // their loads are all in flight before the first use.
    constexpr int kU = 4;
    const int elast = m * S - 1;
    for (int e0 = t; e0 < kBJ * S; e0 += kU * nth) {
      double rv[kU], qv[kU], xv[kU];
      VEC pv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nth;
        const int64_t gi = r0 * S + (e < elast ? e : elast);
        if (INIT) {
          rv[u] = B[gi];
        } else {
          rv[u] = R[gi];
          qv[u] = Q[gi];
          pv[u] = P[gi];
          xv[u] = X[gi];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nth;
        if (e < kBJ * S) {
          const int i = e / S;
          double r = i < m ? rv[u] : 0.0;
          if (i < m) {
            const int64_t gi = r0 * S + e;
            if (INIT) {
              R[gi] = r;
              X[gi] = 0.0;
            } else if (a != 0.0) {
              X[gi] = xv[u] + a * (double)pv[u];
              r -= a * qv[u];
              R[gi] = r;
            }
            rr += r * r;
          }
          Rs[i * kBJ + s_me] = r;
        }
      }
    }
  }
  __syncthreads();
  bj_apply_block<kBJ>(Rs, Mfrag + br.blk * (int64_t)(kBJ * kBJ), m, S, r0, Z, rz);
  __syncthreads();
  const double rzt = bj_rz_total<kBJThreads / kWave>(rz, red, S);
  if (t < S) cs.partial[(int64_t)t * g.nblk + br.blk] = rzt;
  Rs[t] = rr;  // thread t holds column t % S (threads >= nth hold zero)
  __syncthreads();
  if (t < S) {
    double v = 0.0;
    for (int k = t; k < kBJThreads; k += S) v += Rs[k];
    cs.partial[((int64_t)S + t) * g.nblk + br.blk] = v;
  }
}

hipError_t launch_bbj_init(const BatchGeom& g, int S, const double* B, double* X, double* R, void* P, bool f32vec,
                           const double* Mfrag, double* Z, const CgState& cs, double tol, hipStream_t st,
                           const float* M32) {
  if (M32)
    hipLaunchKernelGGL((k_bbj_update<double, true, float>), dim3((unsigned)g.nblk), dim3(kBJThreads), 0, st, g, S, B,
                       X, R, nullptr, nullptr, M32, Z, cs);
  else
    hipLaunchKernelGGL((k_bbj_update<double, true, double>), dim3((unsigned)g.nblk), dim3(kBJThreads), 0, st, g, S,
                       B, X, R, nullptr, nullptr, Mfrag, Z, cs);
  hipLaunchKernelGGL(k_bcg_init_fin, dim3((unsigned)(g.M * S)), dim3(kBlock), 0, st, g, cs, S, tol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_copy_dir(g.n, S, Z, P, f32vec, st);
}

hipError_t launch_bbj_update(const BatchGeom& g, int S, double* X, double* R, const void* P, const void* Q,
                             bool f32vec, const double* Mfrag, double* Z, const CgState& cs, const int32_t* iter_dev,
                             hipStream_t st, const float* M32) {
  const dim3 grid((unsigned)g.grid), block(kBJThreads);
  const double* Qd = static_cast<const double*>(Q);
  if (f32vec && M32)
    hipLaunchKernelGGL((k_bbj_update<float, false, float>), grid, block, 0, st, g, S, nullptr, X, R,
                       static_cast<const float*>(P), Qd, M32, Z, cs);
  else if (f32vec)
    hipLaunchKernelGGL((k_bbj_update<float, false, double>), grid, block, 0, st, g, S, nullptr, X, R,
                       static_cast<const float*>(P), Qd, Mfrag, Z, cs);
  else if (M32)
    hipLaunchKernelGGL((k_bbj_update<double, false, float>), grid, block, 0, st, g, S, nullptr, X, R,
                       static_cast<const double*>(P), Qd, M32, Z, cs);
  else
    hipLaunchKernelGGL((k_bbj_update<double, false, double>), grid, block, 0, st, g, S, nullptr, X, R,
                       static_cast<const double*>(P), Qd, Mfrag, Z, cs);
  hipLaunchKernelGGL(k_bcg_beta, dim3((unsigned)(g.M * S)), dim3(kBlock), 0, st, g, cs, S, iter_dev);
  return hipGetLastError();
}

// ---- per-instance reductions ---------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_bseg_reduce(BatchGeom g, const double* __restrict__ a,
                                                        const double* __restrict__ b, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  const BInst& I = g.inst[blockIdx.x];
  double v = 0.0;
  for (int64_t r = I.row0 + threadIdx.x; r < I.row0 + I.rows; r += kBlock)
    v += MODE == 0 ? a[r] * (b ? b[r] : a[r]) : log(a[r]);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}
hipError_t launch_bseg_reduce(const BatchGeom& g, int mode, const double* a, const double* b, double* out,
                              hipStream_t st) {
  if (mode == 0)
    hipLaunchKernelGGL(k_bseg_reduce<0>, dim3(g.M), dim3(kBlock), 0, st, g, a, b, out);
  else
    hipLaunchKernelGGL(k_bseg_reduce<1>, dim3(g.M), dim3(kBlock), 0, st, g, a, b, out);
  return hipGetLastError();
}

// ---- gradient ----------------------------------------------------------------------------------------
__device__ inline double bb64(double v, int l) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, l);
  p.y = __builtin_amdgcn_readlane(p.y, l);
  return __builtin_bit_cast(double, p);
}
__device__ inline uint64_t bbu64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline double bwsum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <bool F32>
__global__ __launch_bounds__(kBlock) void k_bbackward_rows(BBackward b, double* __restrict__ Rrow,
                                                           double* __restrict__ Trow, double* __restrict__ Urow) {
  const int lane = threadIdx.x & (kWave - 1);
  const XcdRows rr = xcd_rows(b.g.n, threadIdx.x / kWave, kBlock / kWave);
  const int S = b.S;
  const bool active = lane < S;
  for (int64_t row = rr.first; row < rr.end; row += rr.step) {
    const BInst& I = b.g.inst[b.g.inst_of_row[row]];
    const double inv_r = 1.0 / I.radius;
    float4 pi32;
    double4 pi64;
    if (F32) pi32 = b.pts32[row];
    else pi64 = b.pts64[row];
    const double ai = b.a[row];
    const uint64_t mi = b.mask[row];
    const double dsi = sqrt(b.dinv[row]);
    const double qi = active ? b.Q[row * S + lane] : 0.0;
    const double wi = active ? (b.W ? b.W[row * S + lane] : (((mi >> lane) & 1ull) ? -dsi : dsi)) : 0.0;
    double accR = 0.0, accT = 0.0, aR = 0.0, aT = 0.0;
    const int64_t s0 = b.rp[row], e0 = b.rp[row + 1];
    for (int64_t k0 = s0; k0 < e0; k0 += kWave) {
      const int64_t k = k0 + lane;
      const bool valid = k < e0;
      const int32_t j = valid ? b.col[k] : (int32_t)row;
      double gW = 0.0, gWp = 0.0;
      if (valid) {
        double W, dW, gj;
        if (F32) {
          // float64 evaluation from the float32 coordinates (the trace term cancels heavily)
          const float4 pj = b.pts32[j];
          const double dx = (double)pi32.x - (double)pj.x, dy = (double)pi32.y - (double)pj.y,
                       dz = (double)pi32.z - (double)pj.z;
          const double d2 = dx * dx + dy * dy + dz * dz;
          const double t = fmax((I.r2 - d2) * I.inv_r2, 0.0);
          const double rho = sqrt(d2 * I.inv_r2);
          const double om = t / (1.0 + rho);
          wendland_w_dr<double>(I.kern, rho, om, inv_r, W, dW);
          gj = b.g64[j];
        } else {
          const double4 pj = b.pts64[j];
          const double dx = pi64.x - pj.x, dy = pi64.y - pj.y, dz = pi64.z - pj.z;
          const double d2 = dx * dx + dy * dy + dz * dz;
          const double t = fmax((I.r2 - d2) * I.inv_r2, 0.0);
          const double rho = sqrt(d2 * I.inv_r2);
          const double om = t / (1.0 + rho);
          wendland_w_dr<double>(I.kern, rho, om, inv_r, W, dW);
          gj = pt_g(pj.w);
        }
        gW = gj * W;
        gWp = gj * dW;
        const double aj = b.a[j];
        aR += gW * aj;
        aT += gWp * aj;
      }
      const uint64_t mj = valid ? b.mask[j] : 0ull;
      const double dsj = valid ? sqrt(b.dinv[j]) : 0.0;
      const int cnt = (int)((e0 - k0) < kWave ? (e0 - k0) : kWave);
      for (int l = 0; l < cnt; ++l) {
        const int32_t jj = __builtin_amdgcn_readlane(j, l);
        const double gw = bb64(gW, l), gwp = bb64(gWp, l), ds = bb64(dsj, l);
        const uint64_t mm = bbu64(mj, l);
        if (active) {
          const double qj = b.Q[(int64_t)jj * S + lane];
          const double wj = b.W ? b.W[(int64_t)jj * S + lane] : (((mm >> lane) & 1ull) ? -ds : ds);
          const double c = qi * wj + qj * wi;
          accR += gw * c;
          accT += gwp * c;
        }
      }
    }
    const double sR = bwsum(aR), sT = bwsum(aT), pR = bwsum(accR), pT = bwsum(accT), U = bwsum(qi * wi);
    if (lane == 0) {
      const double inv2S = 0.5 / (double)S;
      Rrow[row] = ai * sR - inv2S * pR;
      Trow[row] = ai * sT - inv2S * pT;
      Urow[row] = U;
    }
  }
}

hipError_t launch_bbackward_rows(const BBackward& b, int prec, double* Rrow, double* Trow, double* Urow,
                                 hipStream_t st) {
  int64_t blocks = (b.g.n + (kBlock / kWave) - 1) / (kBlock / kWave);
  if (blocks > (1 << 16)) blocks = 1 << 16;
  blocks = round_up8(blocks < 1 ? 1 : blocks);
  if (prec == GP2S_MIXED)
    hipLaunchKernelGGL(k_bbackward_rows<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, b, Rrow, Trow, Urow);
  else
    hipLaunchKernelGGL(k_bbackward_rows<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, b, Rrow, Trow, Urow);
  return hipGetLastError();
}

// One workgroup per instance: dLML/dr, dLML/da_k, dLML/dsigma^2 from the row sums.
__global__ __launch_bounds__(kBlock) void k_bgrad_reduce(BatchGeom g, int S, const double* __restrict__ x64,
                                                         const double* __restrict__ g64, const double* __restrict__ a,
                                                         const double* __restrict__ Rrow,
                                                         const double* __restrict__ Trow,
                                                         const double* __restrict__ Urow,
                                                         const double* __restrict__ centers3,
                                                         const int32_t* __restrict__ goff, double* __restrict__ grad) {
  __shared__ double sh[kBlock];
  const int i = blockIdx.x;
  const BInst& I = g.inst[i];
  auto block_sum = [&](double v) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    const double t = sh[0];
    __syncthreads();
    return t;
  };
  double cr = 0.0, cs2 = 0.0;
  for (int64_t r = I.row0 + threadIdx.x; r < I.row0 + I.rows; r += kBlock) {
    cr += 0.5 * g64[r] * Trow[r];
    cs2 += 0.5 * (a[r] * a[r] - Urow[r] / (double)S);
  }
  double t = block_sum(cr);
  if (threadIdx.x == 0) grad[goff[i]] = t;
  t = block_sum(cs2);
  if (threadIdx.x == 0) grad[goff[i] + I.P + 1] = t;
  for (int k = 0; k < I.P; ++k) {
    const double* c = centers3 + (int64_t)(I.cent0 + k) * 3;
    double acc = 0.0;
    for (int64_t r = I.row0 + threadIdx.x; r < I.row0 + I.rows; r += kBlock) {
      double d2 = 0.0;
      for (int q = 0; q < 3; ++q) {
        const double d = x64[r * 3 + q] - c[q];
        d2 += d * d;
      }
      if (d2 < I.bump_w2) acc += exp(1.0 - 1.0 / (1.0 - d2 / I.bump_w2)) * Rrow[r];
    }
    t = block_sum(acc);
    if (threadIdx.x == 0) grad[goff[i] + 1 + k] = t;
  }
}

hipError_t launch_bgrad_reduce(const BatchGeom& g, int S, const double* x64, const double* g64, const double* a,
                               const double* Rrow, const double* Trow, const double* Urow, const double* centers3,
                               const int32_t* goff, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_bgrad_reduce, dim3(g.M), dim3(kBlock), 0, st, g, S, x64, g64, a, Rrow, Trow, Urow, centers3,
                     goff, grad);
  return hipGetLastError();
}

}  // namespace gp2s
