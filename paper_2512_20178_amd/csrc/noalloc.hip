// Allocation-free form of the batched product (shiro_spmm_noalloc): the
// carry slots of rows cut by chunk boundaries live in a fixed device array
// of this file instead of a buffer the plan allocates, so the call makes no
// device allocation of any kind once the plan is prepared.
#include <mutex>

#include "plan.hpp"

// Fixed work area: 32 MiB of carry slots (2 slots of N floats per merge-path
// chunk).  That covers every per-rank panel of 2^17 rows and ~4M nonzeros
// at N up to 256 with the tuned chunk sizes; larger patterns are rejected.
// Host code never uses this name as an address: it stands for the host-side
// shadow of the array; the device address comes from hipGetSymbolAddress.
static constexpr int64_t kScratchFloats = int64_t(8) << 20;
static __device__ __align__(256) float scratch[kScratchFloats];

namespace shiro {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

// Device address of the array on the current device, looked up once per
// device (each device holds its own copy of the array).
int scratch_on_current_device(int* dev_out, float** out) {
  int dev = -1;
  SHIRO_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(SHIRO_ERR_UNSUPPORTED, "spmm_noalloc: device index outside [0, 64)");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(SHIRO_ERR_HIP, std::string("spmm_noalloc: hipGetSymbolAddress failed: ") +
                                          hipGetErrorString(e));
    g_ptr[dev] = static_cast<float*>(p);
  }
  *dev_out = dev;
  *out = g_ptr[dev];
  return SHIRO_OK;
}

}  // namespace
}  // namespace shiro

using namespace shiro;

extern "C" {

SHIRO_API int shiro_spmm_noalloc(shiro_plan plan, const float* d_vals, const void* d_Bpacked, int64_t ldp,
                                 int32_t N, shiro_dtype in_dt, void* d_Y, int64_t ldy, shiro_dtype out_dt,
                                 shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_noalloc: plan is NULL");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "spmm_noalloc: call shiro_select_rows first");
  if ((in_dt != SHIRO_F32 && in_dt != SHIRO_BF16) || (out_dt != SHIRO_F32 && out_dt != SHIRO_BF16))
    return set_error(SHIRO_ERR_UNSUPPORTED, "spmm_noalloc: unknown dtype");
  if (in_dt == SHIRO_F32 && out_dt == SHIRO_BF16)
    return set_error(SHIRO_ERR_UNSUPPORTED, "spmm_noalloc: F32 input with BF16 output is not supported");
  if (N < 0 || ldp < N || ldy < N)
    return set_error(SHIRO_ERR_INVALID_ARG, "spmm_noalloc: need N >= 0, ldp >= N, ldy >= N");
  if (N > 0 && plan->rows > 0 && !d_Y) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_noalloc: d_Y is NULL");
  if (N > 0 && plan->nnz > 0 && (!d_Bpacked || !d_vals))
    return set_error(SHIRO_ERR_INVALID_ARG, "spmm_noalloc: NULL input");
  int dev = -1;
  float* area = nullptr;
  SHIRO_TRY(scratch_on_current_device(&dev, &area));
  if (dev != plan->device)
    return set_error(SHIRO_ERR_INVALID_ARG, "spmm_noalloc: the current device is not the plan's device");
  return launch_spmm_fixed(plan, tuning_for(plan, SHIRO_KERNEL_SPMM, N, in_dt), d_vals, d_Bpacked, ldp, N,
                           in_dt, d_Y, ldy, out_dt, area, kScratchFloats, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
