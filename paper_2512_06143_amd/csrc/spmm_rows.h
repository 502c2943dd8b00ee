// Entry-parallel product of stored CSR rows with a row-major block of S vectors.
//
// The lane-per-column products (one lane per right-hand side, stored entries
// broadcast across the wave) spend about five vector instructions per stored entry on
// broadcasts, address arithmetic and conversions. Here the G lanes of a row group
// split the row's stored entries instead: each lane gathers the 16-byte-aligned slice
// X[col, c0 .. c0 + CW) of every G-th entry with 16-byte loads and accumulates CW
// columns in float64, which costs one conversion and one fused multiply-add per
// column and entry. A recursive-halving exchange across the group then leaves every
// lane with CW / G consecutive columns of the result, so no lane holds a sum the others
// have to wait for.
#pragma once

#include "gp2s_internal.h"

namespace gp2s {

template <int CW>
__device__ inline void load_cols(const float* __restrict__ p, float (&v)[CW]) {
  static_assert(CW % 4 == 0, "float slices are read as float4");
#pragma unroll
  for (int q = 0; q < CW / 4; ++q) {
    const float4 t = reinterpret_cast<const float4*>(p)[q];
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
}
template <int CW>
__device__ inline void load_cols(const double* __restrict__ p, double (&v)[CW]) {
  static_assert(CW % 2 == 0, "double slices are read as double2");
#pragma unroll
  for (int q = 0; q < CW / 2; ++q) {
    const double2 t = reinterpret_cast<const double2*>(p)[q];
    v[2 * q] = t.x;
    v[2 * q + 1] = t.y;
  }
}

// As load_cols, through a generic pointer that may address LDS or global memory.
template <int CW>
__device__ inline void load_cols_generic(const float* p, float (&v)[CW]) {
#pragma unroll
  for (int q = 0; q < CW / 4; ++q) {
    const float4 t = reinterpret_cast<const float4*>(p)[q];
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
}
template <int CW>
__device__ inline void load_cols_generic(const double* p, double (&v)[CW]) {
#pragma unroll
  for (int q = 0; q < CW / 2; ++q) {
    const double2 t = reinterpret_cast<const double2*>(p)[q];
    v[2 * q] = t.x;
    v[2 * q + 1] = t.y;
  }
}

// Columns c0 .. c0 + CW of row [s, e) times X (row stride S). `lane` in [0, G) is the
// lane's index inside its row group; every lane of the group must call this together
// (the exchange uses width-G shuffles). On return out[j] holds column
// c0 + lane * (CW / G) + j.
template <int G, int CW, typename V, typename PT>
__device__ inline void row_cols_product(const int32_t* __restrict__ col, const V* __restrict__ val, int64_t s,
                                        int64_t e, int lane, const PT* __restrict__ X, int S, int c0,
                                        double (&out)[CW / G]) {
  static_assert(G >= 2 && G <= CW && (G & (G - 1)) == 0, "G must be a power of two <= CW");
  double acc[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) acc[j] = 0.0;
  int64_t k = s + lane;
  for (; k + G < e; k += 2 * G) {  // two entries per lane in flight
    const int32_t ca = col[k], cb = col[k + G];
    const double va = (double)val[k], vb = (double)val[k + G];
    PT xa[CW], xb[CW];
    load_cols<CW>(X + (int64_t)ca * S + c0, xa);
    load_cols<CW>(X + (int64_t)cb * S + c0, xb);
#pragma unroll
    for (int j = 0; j < CW; ++j) acc[j] += va * (double)xa[j];
#pragma unroll
    for (int j = 0; j < CW; ++j) acc[j] += vb * (double)xb[j];
  }
  if (k < e) {
    const int32_t ca = col[k];
    const double va = (double)val[k];
    PT xa[CW];
    load_cols<CW>(X + (int64_t)ca * S + c0, xa);
#pragma unroll
    for (int j = 0; j < CW; ++j) acc[j] += va * (double)xa[j];
  }
  // Recursive halving: at offset o the lane whose bit o is set keeps the upper half of
  // its live columns, its partner the lower half; each adds what the other sends.
#pragma unroll
  for (int o = G / 2, len = CW; o >= 1; o >>= 1, len >>= 1) {
    const bool upper = (lane & o) != 0;
#pragma unroll
    for (int j = 0; j < len / 2; ++j) {
      const double send = upper ? acc[j] : acc[j + len / 2];
      const double keep = upper ? acc[j + len / 2] : acc[j];
      acc[j] = keep + __shfl_xor(send, o, G);
    }
  }
#pragma unroll
  for (int j = 0; j < CW / G; ++j) out[j] = acc[j];
}

// Slice-per-lane product of one stored row with all S columns of X, for a whole wave:
// a lane owns the VW = 16 / sizeof(PT) consecutive columns (lane % LE) * VW, LE = S / VW
// lanes cover one row of X, and the wave's EPS = 64 / LE lane groups take EPS stored
// entries per step. Every group reads a contiguous S-wide row of X with 16-byte loads,
// so one load instruction moves EPS whole rows of X. Entries are loaded 64 at a time
// (one per lane) and handed to their groups with shuffles; lanes past the row end hold
// (offset 0, value 0). Returns, in every lane, the row's products for its VW columns.
template <int S, typename V, typename PT>
__device__ inline void row_slices_product(const int32_t* __restrict__ col, const V* __restrict__ val, int64_t s,
                                          int64_t e, int lane, const PT* __restrict__ X,
                                          double (&acc)[16 / sizeof(PT)]) {
  constexpr int VW = 16 / sizeof(PT);
  constexpr int LE = S / VW;
  constexpr int EPS = kWave / LE;
  constexpr int U = LE < 4 ? LE : 4;  // steps in flight; LE is a multiple of U
  const int q = lane / LE, cq = lane % LE;
#pragma unroll
  for (int c = 0; c < VW; ++c) acc[c] = 0.0;
  for (int64_t k0 = s; k0 < e; k0 += kWave) {
    const int64_t k = k0 + lane;
    const int32_t off = k < e ? col[k] * S : 0;
    const V vj = k < e ? val[k] : (V)0;
    const int cnt = (int)min((int64_t)kWave, e - k0);
    const int steps = (cnt + EPS - 1) / EPS;  // <= LE
    for (int j = 0; j < steps; j += U) {
      V v[U];
      PT x[U][VW];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = (j + u) * EPS + q;
        v[u] = __shfl(vj, src);
        load_cols<VW>(X + __shfl(off, src) + cq * VW, x[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < VW; ++c) acc[c] += (double)v[u] * (double)x[u][c];
    }
  }
#pragma unroll
  for (int m = LE; m < kWave; m <<= 1)
#pragma unroll
    for (int c = 0; c < VW; ++c) acc[c] += __shfl_xor(acc[c], m);
}

// As row_slices_product, for a row of an LDS-staged tile: rows of X in the tile's staged
// column intervals are read from `lds` (row-major, S values per row), all others from X.
// iv_lo / iv_len / iv_base describe the tile's intervals (base -1: not staged).
template <int S, typename V, typename PT>
__device__ inline void row_tiled_product(const int32_t* __restrict__ col, const V* __restrict__ val, int64_t s,
                                         int64_t e, int lane, const PT* __restrict__ X, const PT* lds, int niv,
                                         const int32_t* iv_lo, const int32_t* iv_len, const int32_t* iv_base,
                                         double (&acc)[16 / sizeof(PT)]) {
  constexpr int VW = 16 / sizeof(PT);
  constexpr int LE = S / VW;
  constexpr int EPS = kWave / LE;
  constexpr int U = LE < 4 ? LE : 4;
  const int q = lane / LE, cq = lane % LE;
#pragma unroll
  for (int c = 0; c < VW; ++c) acc[c] = 0.0;
  for (int64_t k0 = s; k0 < e; k0 += kWave) {
    const int64_t k = k0 + lane;
    int32_t off = 0, loc = -1;
    V vj = (V)0;
    if (k < e) {
      const int32_t c = col[k];
      off = c * S;
      vj = val[k];
      for (int t = 0; t < niv; ++t) {
        const int32_t d = c - iv_lo[t];
        if (d >= 0 && d < iv_len[t] && iv_base[t] >= 0) loc = (iv_base[t] + d) * S;
      }
    }
    const int cnt = (int)min((int64_t)kWave, e - k0);
    const int steps = (cnt + EPS - 1) / EPS;
    for (int j = 0; j < steps; j += U) {
      V v[U];
      PT x[U][VW];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = (j + u) * EPS + q;
        v[u] = __shfl(vj, src);
        const int32_t l = __shfl(loc, src);
        const int32_t o = __shfl(off, src);
        // one generic (flat) load whose address lies in LDS or in global memory, so
        // that the U loads of a step stay in flight together
        const PT* p = l >= 0 ? lds + l + cq * VW : X + o + cq * VW;
        load_cols_generic<VW>(p, x[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < VW; ++c) acc[c] += (double)v[u] * (double)x[u][c];
    }
  }
#pragma unroll
  for (int m = LE; m < kWave; m <<= 1)
#pragma unroll
    for (int c = 0; c < VW; ++c) acc[c] += __shfl_xor(acc[c], m);
}

// Sums v over the lanes of a wave that share `lane % G` (they own the same columns);
// afterwards lanes 0 .. G-1 hold the wave's totals.
template <int G>
__device__ inline double wave_sum_strided(double v) {
#pragma unroll
  for (int o = G; o < kWave; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace gp2s
