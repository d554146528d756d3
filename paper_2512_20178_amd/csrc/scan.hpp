// Device-wide exclusive scan by reduce-then-scan (three launches, no
// atomics, no spin waits): per-tile sums -> one-workgroup scan of the tile
// sums -> per-tile scan with the tile's offset.  Inputs and outputs are
// functors so that a scan can read computed values (e.g. popcounts) and
// write compacted results directly.
#pragma once

#include "common.hpp"

namespace shiro {

constexpr int kScanItems = 16;                    // default elements per thread

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) {
    T y = __shfl_up(x, s, kWave);
    if (lane >= s) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over the 256-thread workgroup.
// lds must hold kWavesPerBlock elements.  *total receives the block sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds, T* total) {
  T inc = wave_inclusive_scan(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == kWave - 1) lds[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) {
    T t = lds[i];
    off += (i < w) ? t : T(0);
    tot += t;
  }
  __syncthreads();
  if (total) *total = tot;
  return off + inc - v;
}

template <int ITEMS, class In>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(In in, int64_t n, int64_t* tile_sums) {
  __shared__ int64_t lds[kWavesPerBlock];
  const int64_t base = (int64_t)blockIdx.x * (kBlock * ITEMS) + (int64_t)threadIdx.x * ITEMS;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (base + i < n) s += in(base + i);
  int64_t tot;
  block_exclusive_scan<int64_t>(s, lds, &tot);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the tile sums in place.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(int64_t* sums, int64_t ntiles,
                                                       int64_t* d_total);

template <int ITEMS, class In, class Out>
__global__ __launch_bounds__(kBlock) void k_scan_down(In in, int64_t n, const int64_t* tile_off,
                                                      Out out) {
  __shared__ int64_t lds[kWavesPerBlock];
  const int64_t base = (int64_t)blockIdx.x * (kBlock * ITEMS) + (int64_t)threadIdx.x * ITEMS;
  int64_t v[ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    v[i] = (base + i < n) ? in(base + i) : 0;
    s += v[i];
  }
  int64_t ex = block_exclusive_scan<int64_t>(s, lds, nullptr) + tile_off[blockIdx.x];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (base + i < n) out(base + i, ex, v[i]);
    ex += v[i];
  }
}

__global__ void k_set_i64(int64_t* p, int64_t v);

inline int64_t scan_tiles_of(int64_t n, int items = kScanItems) { return ceil_div(n, (int64_t)kBlock * items); }

// Host driver.  scratch must hold scan_tiles_of(n, ITEMS) int64.
template <int ITEMS = kScanItems, class In, class Out>
int scan_generic(In in, int64_t n, Out out, int64_t* d_total, void* scratch, hipStream_t s) {
  if (n <= 0) {
    if (d_total) {
      k_set_i64<<<1, 1, 0, s>>>(d_total, 0);
      SHIRO_LAUNCH_CHECK();
    }
    return SHIRO_OK;
  }
  const int64_t ntiles = scan_tiles_of(n, ITEMS);
  int64_t* sums = reinterpret_cast<int64_t*>(scratch);
  k_scan_reduce<ITEMS, In><<<dim3((unsigned)ntiles), kBlock, 0, s>>>(in, n, sums);
  SHIRO_LAUNCH_CHECK();
  k_scan_tiles<<<1, kBlock, 0, s>>>(sums, ntiles, d_total);
  SHIRO_LAUNCH_CHECK();
  k_scan_down<ITEMS, In, Out><<<dim3((unsigned)ntiles), kBlock, 0, s>>>(in, n, sums, out);
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

}  // namespace shiro
