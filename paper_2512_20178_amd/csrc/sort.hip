// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8 bits per pass,
// without atomics.
//
// A workgroup owns a tile of 4096 consecutive keys, split into 64 sub-tiles
// of 64 keys (one key per lane).  Inside a sub-tile, eight ballots give every
// lane the mask of lanes holding the same digit; the lane's rank is the
// popcount of that mask below it and the lowest lane of each digit group
// records the group size.  Sub-tile counts are prefix-summed per digit in
// LDS, tile totals go to a digit-major histogram whose exclusive scan gives
// each (digit, tile) its output offset.  Order inside a digit is tile, then
// sub-tile, then lane: the input order, hence stable and deterministic.
#include "plan.hpp"
#include "scan.hpp"

namespace shiro {

namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSubTile = kWave;                                   // 64 keys
constexpr int kSubTilesPerWave = 16;
constexpr int kSubTiles = kSubTilesPerWave * kWavesPerBlock;      // 64
constexpr int kSortTile = kSubTile * kSubTiles;                   // 4096 keys

static_assert(kSortTile < 65536, "sub-tile counts are 16-bit");

// Same-digit lane mask of this lane inside the wave (invalid lanes excluded).
__device__ __forceinline__ uint64_t digit_peers(uint32_t digit, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool set = (digit >> b) & 1u;
    const uint64_t bal = __ballot(set);
    m &= set ? bal : ~bal;
  }
  return m;
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Rank keys of the tile; fills cnt[st][d] with the exclusive per-digit
// offsets of each sub-tile inside the tile and tot[d] with tile totals.
// keys/ranks are this thread's kSubTilesPerWave keys.
__device__ __forceinline__ void rank_tile(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                          uint16_t (*cnt)[kRadix], uint32_t* tot,
                                          uint32_t (&key)[kSubTilesPerWave],
                                          uint16_t (&rank)[kSubTilesPerWave], int64_t tile_base) {
  for (int i = threadIdx.x; i < kSubTiles * kRadix; i += kBlock) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < kSubTilesPerWave; ++j) {
    const int st = w * kSubTilesPerWave + j;
    const int64_t idx = tile_base + (int64_t)st * kSubTile + lane;
    const bool valid = idx < n;
    key[j] = valid ? keys[idx] : 0u;
    const uint32_t d = (key[j] >> shift) & (kRadix - 1);
    const uint64_t peers = digit_peers(d, valid);
    rank[j] = (uint16_t)__popcll(peers & lanes_below());
    if (valid && rank[j] == 0) cnt[st][d] = (uint16_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: exclusive scan over sub-tiles (thread d owns digit d)
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
    for (int st = 0; st < kSubTiles; ++st) {
      const uint32_t c = cnt[st][d];
      cnt[st][d] = (uint16_t)run;
      run += c;
    }
    tot[d] = run;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_sort_count(const uint32_t* __restrict__ keys, int64_t n,
                                                       int shift, int32_t* __restrict__ hist,
                                                       int64_t ntiles) {
  __shared__ uint16_t cnt[kSubTiles][kRadix];
  __shared__ uint32_t tot[kRadix];
  uint32_t key[kSubTilesPerWave];
  uint16_t rank[kSubTilesPerWave];
  rank_tile(keys, n, shift, cnt, tot, key, rank, (int64_t)blockIdx.x * kSortTile);
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = (int32_t)tot[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_sort_scatter(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t n, int shift,
    const int64_t* __restrict__ hist_off, int64_t ntiles, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
  __shared__ uint16_t cnt[kSubTiles][kRadix];
  __shared__ uint32_t tot[kRadix];
  __shared__ int64_t base[kRadix];
  uint32_t key[kSubTilesPerWave];
  uint16_t rank[kSubTilesPerWave];
  const int64_t tile_base = (int64_t)blockIdx.x * kSortTile;
  rank_tile(keys, n, shift, cnt, tot, key, rank, tile_base);
  base[threadIdx.x] = hist_off[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < kSubTilesPerWave; ++j) {
    const int st = w * kSubTilesPerWave + j;
    const int64_t idx = tile_base + (int64_t)st * kSubTile + lane;
    if (idx < n) {
      const uint32_t d = (key[j] >> shift) & (kRadix - 1);
      const int64_t pos = base[d] + cnt[st][d] + rank[j];
      keys_out[pos] = key[j];
      vals_out[pos] = vals[idx];
    }
  }
}

__global__ void k_copy_u32(const uint32_t* __restrict__ a, uint32_t* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

}  // namespace

int64_t sort_scratch_bytes(int64_t n) {
  const int64_t ntiles = ceil_div(n > 0 ? n : 1, kSortTile);
  const int64_t nh = ntiles * kRadix;
  return 2 * n * 4 + 256      // ping-pong keys/values
         + nh * 4 + 256       // histogram
         + nh * 8 + 256       // scanned histogram
         + scan_scratch_bytes(nh);
}

int radix_sort_pairs(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                     uint32_t* vals_out, int64_t n, int key_bits, void* scratch, hipStream_t s) {
  if (n <= 0) return SHIRO_OK;
  const int64_t ntiles = ceil_div(n, kSortTile);
  const int64_t nh = ntiles * kRadix;
  char* p = reinterpret_cast<char*>(scratch);
  auto take = [&](int64_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  uint32_t* tk = reinterpret_cast<uint32_t*>(take(n * 4));
  uint32_t* tv = reinterpret_cast<uint32_t*>(take(n * 4));
  int32_t* hist = reinterpret_cast<int32_t*>(take(nh * 4));
  int64_t* hoff = reinterpret_cast<int64_t*>(take(nh * 8));
  void* scan_tmp = take(scan_scratch_bytes(nh));

  int passes = (key_bits + kRadixBits - 1) / kRadixBits;
  const unsigned g = (unsigned)ceil_div(n, kBlock) < 65536u ? (unsigned)ceil_div(n, kBlock) : 65536u;
  if (passes == 0) {
    k_copy_u32<<<g, kBlock, 0, s>>>(keys_in, keys_out, n);
    k_copy_u32<<<g, kBlock, 0, s>>>(vals_in, vals_out, n);
    SHIRO_LAUNCH_CHECK();
    return SHIRO_OK;
  }
  // Choose the ping-pong order so that the last pass writes keys_out/vals_out.
  const uint32_t* ck = keys_in;
  const uint32_t* cv = vals_in;
  for (int pass = 0; pass < passes; ++pass) {
    const bool last = pass == passes - 1;
    const bool to_out = ((passes - 1 - pass) % 2) == 0;
    uint32_t* ok = to_out ? keys_out : tk;
    uint32_t* ov = to_out ? vals_out : tv;
    (void)last;
    const int shift = pass * kRadixBits;
    k_sort_count<<<(unsigned)ntiles, kBlock, 0, s>>>(ck, n, shift, hist, ntiles);
    SHIRO_LAUNCH_CHECK();
    SHIRO_TRY(exclusive_scan_i32_to_i64(hist, nh, hoff, nullptr, scan_tmp, s));
    k_sort_scatter<<<(unsigned)ntiles, kBlock, 0, s>>>(ck, cv, n, shift, hoff, ntiles, ok, ov);
    SHIRO_LAUNCH_CHECK();
    ck = ok;
    cv = ov;
  }
  return SHIRO_OK;
}

}  // namespace shiro
