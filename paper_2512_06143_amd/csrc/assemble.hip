// Covariance assembly: pair culling, kernel evaluation and stream compaction into CSR.
//
// K_ij = g_i g_j W(||x_i - x_j|| / r) + sigma_n^2 [i == j], W a Wendland member for
// rho < 1: the C^2 (1 - rho)^4 (4 rho + 1) or Eq. wendland's C^6 (Sec. 4.1 product
// construction; Sec. 4.3 bump mask g). The paper computes dense block pairs and keeps the non-zeros
// (Sec. 4.6, App. B.7); here only candidates from the 3^d neighbouring bins are
// tested, and a pair is stored when ||x_i - x_j|| < r and both points lie inside
// some bump (the diagonal always).
//
// One wavefront owns 16 consecutive rows of the binned order, so the rows of one cell lie
// together. For each cell among them, lanes take 64 consecutive candidates of the cell's
// neighbour-bin runs at a time (bins adjacent along x are contiguous in the sorted order;
// the runs are concatenated in ascending order) and test them against each of the
// wave's rows of that cell in turn: a candidate is loaded once per wave rather than once
// per row. The wave ballot plus the lane's popcount prefix (mbcnt) give every survivor
// its slot, so each row is written as one contiguous, ascending run, the same for any
// number of rows per wave. The count pass and the fill pass execute the same candidate
// sequence and the same test.
//
// Float32 path: the support test uses float32 distances. Entry values are evaluated in
// float64 from the float32 coordinates and g (t = 1 - rho^2 from the exact squared
// distance, 1 - rho = t / (1 + rho), the polynomial) and rounded once to float32, so
// the stored matrix differs from K by at most half an ulp per entry.
//
// General kernel (Eq. wendconv, axis radii, length-scale field l): the same sweep with
// the per-axis scaled distance tested against m_ij = (l_i^2 + l_j^2) / 2 (cells are
// sized by the radii times the bound of l), and the prefactor (l_i l_j / m_ij)^{d/2}.
#include <type_traits>

#include "gp2s_internal.h"
#include "pair.h"

namespace gp2s {

// Rows per wave. A wave takes kAsmRows consecutive rows of the binned order, so the rows
// of one cell lie together; the cell's candidate list is walked once per wave, and every
// candidate is tested against all of the wave's rows in that cell.
constexpr int kAsmRows = 16;

template <int DIM, bool FILL, bool F32>
__global__ __launch_bounds__(kBlock) void k_assemble(AssembleArgs a, int64_t nblocks_padded,
                                                     int32_t* __restrict__ row_cnt,
                                                     const int64_t* __restrict__ row_ptr,
                                                     int32_t* __restrict__ col, void* __restrict__ val,
                                                     double* __restrict__ diag) {
  using PtT = typename std::conditional<F32, float4, double4>::type;
  constexpr int NW = kBlock / kWave;
  // the wave's rows: point, g, length-scale weight l^2 and (fill pass) the row's CSR range;
  // read back with a wave-uniform address (one broadcast LDS read per row and step)
  __shared__ PtT s_pt[NW][kAsmRows];
  __shared__ double s_g[NW][kAsmRows];
  __shared__ double s_l[NW][kAsmRows];
  __shared__ int64_t s_base[NW][FILL ? kAsmRows : 1];
  __shared__ int64_t s_end[NW][FILL ? kAsmRows : 1];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int64_t lb = xcd_block(nblocks_padded);
  const int64_t g0 = (lb * NW + w) * (int64_t)kAsmRows;
  if (g0 >= a.n) return;  // uniform per wave
  const int nr = (int)((a.n - g0) < kAsmRows ? (a.n - g0) : kAsmRows);
  const bool gen = a.kg.general != 0;

  // lane r < nr holds row g0 + r
  const int64_t myrow = g0 + lane;
  const bool have = lane < nr;
  int32_t mybin = -1;
  bool in_mine = false;
  if (have) {
    PtT p;
    if constexpr (F32) {
      p = a.pts32[myrow];
    } else {
      p = a.pts64[myrow];
    }
    s_pt[w][lane] = p;
    in_mine = pt_in(p.w);
    mybin = a.binid[myrow];
    s_g[w][lane] = a.g64[myrow];
    s_l[w][lane] = a.kg.lsq ? a.kg.lsq[myrow] : 1.0;
    if (FILL) {
      s_base[w][lane] = row_ptr[myrow];
      s_end[w][lane] = row_ptr[myrow + 1];
    }
  }
  __builtin_amdgcn_wave_barrier();
  int32_t cnt = 0;  // lane r: entries of row g0 + r found so far
  if (have && !in_mine) {
    // outside every bump: g = 0, only the noise on the diagonal is stored
    if (FILL) {
      const int64_t base = s_base[w][lane];
      col[base] = (int32_t)myrow;
      if constexpr (F32) {
        const float v = (float)a.noise;
        static_cast<float*>(val)[base] = v;
        diag[myrow] = (double)v;
      } else {
        static_cast<double*>(val)[base] = a.noise;
        diag[myrow] = a.noise;
      }
    }
    cnt = 1;
  }
  const int nbx = a.grid.nb[0], nby = a.grid.nb[1], nbz = a.grid.nb[2];
  constexpr int NR = DIM == 3 ? 9 : 3;
  int r = 0;
  while (r < nr) {  // runs of rows in one cell (uniform)
    const int32_t bin = __builtin_amdgcn_readlane(mybin, r);
    const uint64_t same = __ballot(have && mybin == bin);  // lanes r .. r2 - 1 (rows are bin-sorted)
    const int r2 = r + __popcll(same);
    const uint64_t act = __ballot(lane >= r && lane < r2 && in_mine);
    r = r2;
    if (!act) continue;
    // The 3^(d-1) runs of neighbouring bins (bins adjacent along x are contiguous in the
    // sorted order), in ascending order, concatenated into one candidate list: run q starts
    // at rs[q] and takes candidate indices pre[q] .. pre[q + 1] - 1.
    int bx, by, bz;
    decode_bin<DIM>(bin, a.grid, bx, by, bz);
    const int x0 = bx > 0 ? bx - 1 : 0;
    const int x1 = bx + 1 < nbx ? bx + 1 : nbx - 1;
    int64_t rs[NR];
    int32_t pre[NR + 1];
    pre[0] = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int dz = DIM == 3 ? q / 3 - 1 : 0, dy = q % 3 - 1;
      const int zz = bz + dz, yy = by + dy;
      int64_t s0 = 0, e0 = 0;
      if (zz >= 0 && zz < nbz && yy >= 0 && yy < nby) {
        const int64_t rb = ((int64_t)zz * nby + yy) * nbx;
        s0 = a.bin_start[rb + x0];
        e0 = a.bin_start[rb + x1 + 1];
      }
      rs[q] = s0;
      pre[q + 1] = pre[q] + (int32_t)(e0 - s0);
    }
    const int32_t C = pre[NR];
    for (int32_t c0 = 0; c0 < C; c0 += kWave) {
      // this lane's candidate of the step
      const int32_t idx = c0 + lane;
      int64_t j = rs[0] + idx;
#pragma unroll
      for (int q = 1; q < NR; ++q)
        if (idx >= pre[q]) j = rs[q] + (idx - pre[q]);  // empty runs are overridden by the next
      const bool ok = idx < C;
      PtT pj;
      if constexpr (F32) {
        pj = ok ? a.pts32[j] : make_float4(0.f, 0.f, 0.f, pt_out_f32());
      } else {
        pj = ok ? a.pts64[j] : make_double4(0., 0., 0., pt_out_f64());
      }
      const double lj = (a.kg.lsq && ok) ? a.kg.lsq[j] : 1.0;
      const bool cand = ok && pt_in(pj.w);
      // every row of the run inside a bump, in order
      for (uint64_t rem = act; rem; rem &= rem - 1) {
        const int rr = __builtin_ctzll(rem);
        const int64_t row = g0 + rr;
        const PtT pi = s_pt[w][rr];
        const double li = s_l[w][rr];
        bool pass;
        if constexpr (F32) {
          pass = ok && (j == row || (cand && (gen ? gen_pass_f32<DIM>(pi, pj, a.kg, li, lj)
                                                : sqdist_f32<DIM>(pi, pj) < a.r2f)));
        } else {
          pass = ok && (j == row || (cand && (gen ? gen_pass_f64<DIM>(pi, pj, a.kg, li, lj)
                                                : sqdist_f64<DIM>(pi, pj) < a.r2)));
        }
        const uint64_t m = __ballot(pass);
        if (FILL && m) {
          const int64_t pos = s_base[w][rr] + __builtin_amdgcn_readlane(cnt, rr) + lane_prefix(m);
          if (pass && pos < s_end[w][rr]) {  // never past the row counted by the first pass
            col[pos] = (int32_t)j;
            const double gi64 = s_g[w][rr];
            if constexpr (F32) {
              const float v = (j == row) ? (float)(gi64 * gi64 + a.noise)
                              : gen ? gen_entry_f32<DIM>(pi, pj, a.kg, li, lj, a.kern)
                                    : entry_f32(pi, pj, a.r2, a.inv_r2, a.kern);
              static_cast<float*>(val)[pos] = v;
              if (j == row) diag[row] = (double)v;
            } else {
              const double v = (j == row) ? gi64 * gi64 + a.noise
                               : gen ? gen_entry_f64<DIM>(pi, pj, a.kg, li, lj, a.kern)
                                     : entry_f64(pi, pj, a.r2, a.inv_r2, a.kern);
              static_cast<double*>(val)[pos] = v;
              if (j == row) diag[row] = v;
            }
          }
        }
        if (lane == rr) cnt += __popcll(m);
      }
    }
  }
  if (!FILL && have) row_cnt[myrow] = cnt;
}

template <bool FILL>
static hipError_t launch_assemble_t(const AssembleArgs& a, int prec, int32_t* row_cnt,
                                    const int64_t* row_ptr, int32_t* col, void* val, double* diag,
                                    hipStream_t st) {
  const int64_t rows_per_block = (int64_t)(kBlock / kWave) * kAsmRows;
  int64_t nblocks = (a.n + rows_per_block - 1) / rows_per_block;
  int64_t padded = (nblocks + 7) / 8 * 8;
  dim3 grid((unsigned)padded), block(kBlock);
  const bool f32 = prec == GP2S_MIXED;
  if (a.grid.dim == 2) {
    if (f32)
      hipLaunchKernelGGL((k_assemble<2, FILL, true>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val, diag);
    else
      hipLaunchKernelGGL((k_assemble<2, FILL, false>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val, diag);
  } else {
    if (f32)
      hipLaunchKernelGGL((k_assemble<3, FILL, true>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val, diag);
    else
      hipLaunchKernelGGL((k_assemble<3, FILL, false>), grid, block, 0, st, a, padded, row_cnt, row_ptr, col, val, diag);
  }
  return hipGetLastError();
}

hipError_t launch_assemble_count(const AssembleArgs& a, int prec, int32_t* row_cnt, hipStream_t st) {
  return launch_assemble_t<false>(a, prec, row_cnt, nullptr, nullptr, nullptr, nullptr, st);
}

hipError_t launch_assemble_fill(const AssembleArgs& a, int prec, const int64_t* row_ptr,
                                int32_t* col, void* val, double* diag, hipStream_t st) {
  return launch_assemble_t<true>(a, prec, nullptr, row_ptr, col, val, diag, st);
}

}  // namespace gp2s
