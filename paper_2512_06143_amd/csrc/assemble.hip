// Covariance assembly: pair culling, kernel evaluation and stream compaction into CSR.
//
// K_ij = g_i g_j W(||x_i - x_j|| / r) + sigma_n^2 [i == j], W a Wendland member for
// rho < 1: the C^2 (1 - rho)^4 (4 rho + 1) or Eq. wendland's C^6 (Sec. 4.1 product
// construction; Sec. 4.3 bump mask g). The paper computes dense block pairs and keeps the non-zeros
// (Sec. 4.6, App. B.7); here only candidates from the 3^d neighbouring bins are
// tested, and a pair is stored when ||x_i - x_j|| < r and both points lie inside
// some bump (the diagonal always).
//
// One wavefront owns one row. Lanes take consecutive candidates of the row's neighbour-
// bin runs (bins adjacent along x are contiguous in the sorted order; the runs are
// concatenated in ascending order), test them, and the
// wave ballot plus the lane's popcount prefix (mbcnt) give every survivor its slot,
// so each row is written as one contiguous, ascending, coalesced run. The count
// pass and the fill pass execute the same candidate sequence and the same test.
//
// Float32 path: the support test uses float32 distances. Entry values are evaluated in
// float64 from the float32 coordinates and g (t = 1 - rho^2 from the exact squared
// distance, 1 - rho = t / (1 + rho), the polynomial) and rounded once to float32, so
// the stored matrix differs from K by at most half an ulp per entry.
//
// General kernel (Eq. wendconv, axis radii, length-scale field l): the same sweep with
// the per-axis scaled distance tested against m_ij = (l_i^2 + l_j^2) / 2 (cells are
// sized by the radii times the bound of l), and the prefactor (l_i l_j / m_ij)^{d/2}.
#include "gp2s_internal.h"
#include "pair.h"

namespace gp2s {

template <int DIM, bool FILL, bool F32>
__global__ __launch_bounds__(kBlock) void k_assemble(AssembleArgs a, int64_t nblocks_padded,
                                                     int32_t* __restrict__ row_cnt,
                                                     const int64_t* __restrict__ row_ptr,
                                                     int32_t* __restrict__ col, void* __restrict__ val,
                                                     double* __restrict__ diag) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lb = xcd_block(nblocks_padded);
  const int64_t row = lb * (kBlock / kWave) + threadIdx.x / kWave;
  if (row >= a.n) return;  // uniform per wave

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
  const int64_t base = FILL ? row_ptr[row] : 0;
  const int64_t end = FILL ? row_ptr[row + 1] : 0;
  if (!in_i) {
    // Outside every bump: g_i = 0, only the noise on the diagonal is stored.
    if (lane == 0) {
      if (FILL) {
        col[base] = (int32_t)row;
        double d = a.noise;
        if (F32) {
          float v = (float)d;
          static_cast<float*>(val)[base] = v;
          diag[row] = (double)v;
        } else {
          static_cast<double*>(val)[base] = d;
          diag[row] = d;
        }
      } else {
        row_cnt[row] = 1;
      }
    }
    return;
  }
  int bx, by, bz;
  decode_bin<DIM>(a.binid[row], a.grid, bx, by, bz);
  const int nbx = a.grid.nb[0], nby = a.grid.nb[1], nbz = a.grid.nb[2];
  const int x0 = bx > 0 ? bx - 1 : 0;
  const int x1 = bx + 1 < nbx ? bx + 1 : nbx - 1;
  // The 3^(d-1) runs of neighbouring bins (bins adjacent along x are contiguous in the
  // sorted order), in ascending order, concatenated into one candidate list: run r starts
  // at rs[r] and takes candidate indices pre[r] .. pre[r + 1] - 1. Lanes then take 64
  // consecutive candidates of the list, across run boundaries, so short runs do not leave
  // most lanes of a step idle.
  constexpr int NR = DIM == 3 ? 9 : 3;
  int64_t rs[NR];
  int32_t pre[NR + 1];
  pre[0] = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int dz = DIM == 3 ? r / 3 - 1 : 0, dy = r % 3 - 1;
    const int zz = bz + dz, yy = by + dy;
    int64_t s0 = 0, e0 = 0;
    if (zz >= 0 && zz < nbz && yy >= 0 && yy < nby) {
      const int64_t rb = ((int64_t)zz * nby + yy) * nbx;
      s0 = a.bin_start[rb + x0];
      e0 = a.bin_start[rb + x1 + 1];
    }
    rs[r] = s0;
    pre[r + 1] = pre[r] + (int32_t)(e0 - s0);
  }
  const int32_t C = pre[NR];
  int64_t cnt = 0;
  const double gi64 = a.g64[row];
  const bool gen = a.kg.general != 0;
  const double li = a.kg.lsq ? a.kg.lsq[row] : 1.0;

  // Candidates are taken 64 at a time from the concatenated runs. In the count pass and
  // the float32-stored fill the next step's candidate is loaded before the current one is
  // tested, so that its latency overlaps the test (rows in crowded cells take many steps);
  // the float64-stored fill loads in place (its registers would cost occupancy).
  constexpr bool kAhead = !FILL || F32;
  auto cand = [&](int32_t idx, int64_t& j, bool& ok, float4& p32, double4& p64, double& l) {
    j = rs[0] + idx;
#pragma unroll
    for (int r = 1; r < NR; ++r)
      if (idx >= pre[r]) j = rs[r] + (idx - pre[r]);  // empty runs are overridden by the next
    ok = idx < C;
    if (F32) p32 = ok ? a.pts32[j] : make_float4(0.f, 0.f, 0.f, pt_out_f32());
    else p64 = ok ? a.pts64[j] : make_double4(0., 0., 0., pt_out_f64());
    l = (a.kg.lsq && ok) ? a.kg.lsq[j] : 1.0;
  };
  int64_t jn = 0;
  bool okn = false;
  float4 pn32 = make_float4(0.f, 0.f, 0.f, pt_out_f32());
  double4 pn64 = make_double4(0., 0., 0., pt_out_f64());
  double ln = 1.0;
  if (kAhead) cand(lane, jn, okn, pn32, pn64, ln);
  for (int32_t c0 = 0; c0 < C; c0 += kWave) {
    int64_t j = jn;
    bool ok = okn;
    float4 pj32 = pn32;
    double4 pj64 = pn64;
    double lj = ln;
    if (!kAhead) cand(c0 + lane, j, ok, pj32, pj64, lj);
    else if (c0 + kWave < C) cand(c0 + kWave + lane, jn, okn, pn32, pn64, ln);
    bool pass;
    if (F32) {
      pass = ok && (j == row || (pt_in(pj32.w) && (gen ? gen_pass_f32<DIM>(pi32, pj32, a.kg, li, lj)
                                                        : sqdist_f32<DIM>(pi32, pj32) < a.r2f)));
    } else {
      pass = ok && (j == row || (pt_in(pj64.w) && (gen ? gen_pass_f64<DIM>(pi64, pj64, a.kg, li, lj)
                                                       : sqdist_f64<DIM>(pi64, pj64) < a.r2)));
    }
    const uint64_t m = __ballot(pass);
    const int64_t pos = base + cnt + lane_prefix(m);
    if (FILL && pass && pos < end) {  // never past the row counted by the first pass
      col[pos] = (int32_t)j;
      if (F32) {
        float v = (j == row) ? (float)(gi64 * gi64 + a.noise)
                  : gen ? gen_entry_f32<DIM>(pi32, pj32, a.kg, li, lj, a.kern)
                        : entry_f32(pi32, pj32, a.r2, a.inv_r2, a.kern);
        static_cast<float*>(val)[pos] = v;
        if (j == row) diag[row] = (double)v;
      } else {
        double v = (j == row) ? gi64 * gi64 + a.noise
                   : gen ? gen_entry_f64<DIM>(pi64, pj64, a.kg, li, lj, a.kern)
                         : entry_f64(pi64, pj64, a.r2, a.inv_r2, a.kern);
        static_cast<double*>(val)[pos] = v;
        if (j == row) diag[row] = v;
      }
    }
    cnt += __popcll(m);
  }
  if (!FILL && lane == 0) row_cnt[row] = (int32_t)cnt;
}

template <bool FILL>
static hipError_t launch_assemble_t(const AssembleArgs& a, int prec, int32_t* row_cnt,
                                    const int64_t* row_ptr, int32_t* col, void* val, double* diag,
                                    hipStream_t st) {
  const int rows_per_block = kBlock / kWave;
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
