// Row-grouped copy of a CSR matrix for the multi-column block product.
//
// Consecutive rows of the bin order are spatial neighbours, so their column lists
// overlap heavily (at 63 stored entries per row, 4 consecutive rows reference 42% as
// many distinct columns as they have entries, 8 rows 25%). Grouping kGrp rows and
// storing, for each group, the sorted union of their columns with one value per row
// (zero where a row has no entry) lets the block product gather each row of X once per
// group instead of once per entry. The group layout:
//   gptr [ngroups + 1]      start of group g's union entries,
//   gcol [entries]          the union columns, ascending,
//   gval [entries * kGrp]   gval[k * kGrp + r] = K[kGrp g + r][gcol[k]] (0 if absent),
//   map  [nnz]              CSR entry -> its slot k * kGrp + r in gval (refills of the values).
// The union is a kGrp-way merge of ascending lists, one wave per group: lanes 0..kGrp-1
// hold the heads of their rows and the wave minimum is the next union column.
#include "gp2s_internal.h"

namespace gp2s {

static_assert(kGrp >= 1 && kGrp <= 8, "the merge holds one row per lane among lanes 0..7");

__device__ inline int32_t wave_min8(int32_t v) {
  // minimum over lanes 0..7 (kGrp <= 8; lanes past kGrp hold INT32_MAX); every lane of
  // the wave takes part in the shuffles
  v = min(v, __shfl_xor(v, 4, kWave));
  v = min(v, __shfl_xor(v, 2, kWave));
  v = min(v, __shfl_xor(v, 1, kWave));
  return __shfl(v, 0, kWave);
}

template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_grp_merge(int64_t n, const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col, int64_t ngroups,
                                                      int32_t* __restrict__ cnt, const int64_t* __restrict__ gptr,
                                                      int32_t* __restrict__ gcol, int32_t* __restrict__ map) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t g = blockIdx.x * (int64_t)(kBlock / kWave) + threadIdx.x / kWave;
  if (g >= ngroups) return;  // uniform per wave
  const int64_t row = g * kGrp + lane;
  const bool mine = lane < kGrp && row < n;
  int64_t p = mine ? rp[row] : 0;
  const int64_t e = mine ? rp[row + 1] : 0;
  int64_t k = FILL ? gptr[g] : 0;
  int64_t count = 0;
  for (;;) {
    const int32_t head = p < e ? col[p] : INT32_MAX;
    const int32_t m = wave_min8(head);
    if (m == INT32_MAX) break;
    if (FILL) {
      if (lane == 0) gcol[k] = m;
      if (head == m) map[p] = (int32_t)(k * kGrp + lane);
      ++k;
    }
    if (head == m) ++p;
    ++count;
  }
  if (!FILL && lane == 0) cnt[g] = (int32_t)count;
}

template <typename V>
__global__ void k_grp_values(int64_t nnz, const V* __restrict__ val, const int32_t* __restrict__ map,
                             V* __restrict__ gval) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
    gval[map[k]] = val[k];
}

hipError_t launch_grp_count(int64_t n, const int64_t* rp, const int32_t* col, int64_t ngroups, int32_t* cnt,
                            hipStream_t st) {
  const int64_t blocks = (ngroups + kBlock / kWave - 1) / (kBlock / kWave);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grp_merge<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, rp, col, ngroups, cnt,
                     nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_grp_fill(int64_t n, const int64_t* rp, const int32_t* col, int64_t ngroups, const int64_t* gptr,
                           int32_t* gcol, int32_t* map, hipStream_t st) {
  const int64_t blocks = (ngroups + kBlock / kWave - 1) / (kBlock / kWave);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grp_merge<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, n, rp, col, ngroups, nullptr,
                     gptr, gcol, map);
  return hipGetLastError();
}

hipError_t launch_grp_values(int64_t nnz, const void* val, int prec, const int32_t* map, void* gval, hipStream_t st) {
  int64_t blocks = (nnz + kBlock - 1) / kBlock;
  if (blocks > (1 << 16)) blocks = 1 << 16;
  if (blocks < 1) return hipSuccess;
  if (prec == GP2S_MIXED)
    hipLaunchKernelGGL(k_grp_values<float>, dim3((unsigned)blocks), dim3(kBlock), 0, st, nnz,
                       static_cast<const float*>(val), map, static_cast<float*>(gval));
  else
    hipLaunchKernelGGL(k_grp_values<double>, dim3((unsigned)blocks), dim3(kBlock), 0, st, nnz,
                       static_cast<const double*>(val), map, static_cast<double*>(gval));
  return hipGetLastError();
}

}  // namespace gp2s
