// Exclusive prefix sums (row counts -> CSR row pointers, bin counts -> bin starts).
// Three passes: per-tile sums, a single-workgroup scan of the tile sums, and a
// per-tile scan that adds the tile offset. Deterministic (integer arithmetic).
#include "gp2s_internal.h"

namespace gp2s {

constexpr int kScanItems = 16;                     // elements per thread
constexpr int kScanTile = kBlock * kScanItems;     // elements per workgroup

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  // Wave-level inclusive scan with shuffles, then across the 4 waves of the block.
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int64_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      int64_t t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[kBlock / kWave] = acc;
  }
  __syncthreads();
  int64_t excl = x - v + sh[wid];
  if (total) *total = sh[kBlock / kWave];
  __syncthreads();
  return excl;
}

__global__ __launch_bounds__(kBlock) void k_tile_sums(const int32_t* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ tile_sum) {
  __shared__ int64_t sh[kBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t acc = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) acc += in[i];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = sh[0];
}

// Single workgroup: exclusive scan of the tile sums in place; grand total at [ntiles].
__global__ __launch_bounds__(kBlock) void k_scan_tiles(int64_t* __restrict__ tile_sum, int64_t ntiles) {
  __shared__ int64_t sh[kBlock / kWave + 1];
  int64_t carry = 0;
  for (int64_t base = 0; base < ntiles; base += kBlock) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < ntiles ? tile_sum[i] : 0;
    int64_t total;
    int64_t e = block_exclusive_scan(v, sh, &total);
    if (i < ntiles) tile_sum[i] = carry + e;
    carry += total;
  }
  if (threadIdx.x == 0) tile_sum[ntiles] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                       const int64_t* __restrict__ tile_off,
                                                       int64_t* __restrict__ out) {
  __shared__ int64_t sh[kBlock / kWave + 1];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  // Each thread owns kScanItems consecutive elements.
  int64_t first = base + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = first + k;
    v[k] = i < n ? in[i] : 0;
    acc += v[k];
  }
  int64_t excl = block_exclusive_scan(acc, sh, nullptr) + tile_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = first + k;
    if (i < n) out[i] = excl;
    excl += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    // grand total
    out[n] = tile_off[gridDim.x];
  }
}

size_t scan_workspace_bytes(int64_t n) {
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  return (size_t)(ntiles + 1) * sizeof(int64_t);
}

hipError_t launch_exscan_i32_i64(const int32_t* in, int64_t* out, int64_t n, void* ws, hipStream_t st) {
  int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles == 0) {
    return hipMemsetAsync(out, 0, sizeof(int64_t), st);
  }
  int64_t* tiles = static_cast<int64_t*>(ws);
  hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)ntiles), dim3(kBlock), 0, st, in, n, tiles);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kBlock), 0, st, tiles, ntiles);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kBlock), 0, st, in, n, tiles, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_i64_to_i32(const int64_t* __restrict__ in,
                                                       int32_t* __restrict__ out, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int32_t)in[i];
}

hipError_t launch_i64_to_i32(const int64_t* in, int32_t* out, int64_t n, hipStream_t st) {
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_i64_to_i32, dim3((unsigned)blocks), dim3(kBlock), 0, st, in, out, n);
  return hipGetLastError();
}

}  // namespace gp2s
