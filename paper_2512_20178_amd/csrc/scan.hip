// Device-wide exclusive scans used by selection, sorting and segment lists.
#include "plan.hpp"
#include "scan.hpp"

namespace shiro {

__global__ __launch_bounds__(kBlock) void k_scan_tiles(int64_t* sums, int64_t ntiles,
                                                       int64_t* d_total) {
  __shared__ int64_t lds[kWavesPerBlock];
  int64_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += kBlock) {
    const int64_t i = b + threadIdx.x;
    const int64_t v = i < ntiles ? sums[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan<int64_t>(v, lds, &tot);
    if (i < ntiles) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && d_total) *d_total = carry;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

namespace {
struct InI32 {
  const int32_t* p;
  __device__ int64_t operator()(int64_t i) const { return p[i]; }
};
struct InI64 {
  const int64_t* p;
  __device__ int64_t operator()(int64_t i) const { return p[i]; }
};
struct OutI64 {
  int64_t* p;
  __device__ void operator()(int64_t i, int64_t prefix, int64_t) const { p[i] = prefix; }
};
}  // namespace

int64_t scan_scratch_bytes(int64_t n) { return scan_tiles_of(n > 0 ? n : 1, 1) * 8 + 256; }

int exclusive_scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, int64_t* d_total,
                              void* scratch, hipStream_t s) {
  return scan_generic(InI32{in}, n, OutI64{out}, d_total, scratch, s);
}

int exclusive_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* d_total,
                       void* scratch, hipStream_t s) {
  return scan_generic(InI64{in}, n, OutI64{out}, d_total, scratch, s);
}

}  // namespace shiro
