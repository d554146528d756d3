// Shared helpers of the gfx950 library: error plumbing, wave64 primitives,
// 16-byte vector loads/stores for float32 and bfloat16 rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/shiro.h"

namespace shiro {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kBlock = 256;   // threads per workgroup (4 wavefronts)
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------------------
// host-side status handling
// ---------------------------------------------------------------------------
int set_error(int code, const std::string& msg);

#define SHIRO_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::shiro::set_error(e_ == hipErrorOutOfMemory ? SHIRO_ERR_OOM : SHIRO_ERR_HIP, \
                                std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SHIRO_TRY(call)     \
  do {                      \
    int s_ = (call);        \
    if (s_ != SHIRO_OK) return s_; \
  } while (0)

#define SHIRO_LAUNCH_CHECK() SHIRO_HIP(hipGetLastError())

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Wave index inside the workgroup, known uniform (lets the compiler keep
// values derived from it in scalar registers).
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

template <typename T>
__device__ __forceinline__ T uniform(T v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Native clang vectors (what the AMDGPU backend maps to dwordx4 accesses).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// bfloat16 is carried as its 16-bit pattern.
typedef uint16_t bf16_t;

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) {
  return __uint_as_float(bits16 << 16);
}
// Round to nearest even (gfx950 v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
  __bf16 b = (__bf16)x;
  return __builtin_bit_cast(uint16_t, b);
}

// ---------------------------------------------------------------------------
// cross-lane sums without the LDS crossbar (DPP row ops, permlane swaps)
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}

// Sum of x over each aligned group of LANES lanes.  The sum is exact in the
// group's last lane (lane LANES-1 of the group); other lanes hold partial
// sums.  Every step adds two disjoint partial sums, so the result does not
// depend on anything but the inputs.
template <int LANES>
__device__ __forceinline__ float group_sum(float x) {
  static_assert(LANES == 8 || LANES == 16 || LANES == 32 || LANES == 64, "lanes");
  x = dpp_add<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
  x = dpp_add<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
  x = dpp_add<0x141, 0xF>(x);  // row_half_mirror: 8-lane sums
  if constexpr (LANES >= 16) x = dpp_add<0x140, 0xF>(x);  // row_mirror: 16-lane sums
  if constexpr (LANES >= 32) x = dpp_add<0x142, 0xA>(x);  // row_bcast15 into rows 1, 3
  if constexpr (LANES >= 64) x = dpp_add<0x143, 0xC>(x);  // row_bcast31 into rows 2, 3
  return x;
}

// Lane-wise sum over the 64/LANES groups of a wavefront (lane l gets
// sum over g of x[l mod LANES + g LANES]), in a fixed pairing order.
template <int LANES>
__device__ __forceinline__ float groups_sum(float x) {
  if constexpr (LANES <= 8) {
    // pair lanes i and i+8 inside each row of 16 (rotate by 8)
    x = x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false));
  }
  if constexpr (LANES <= 16) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(x), __float_as_int(x), false, false);
    x = __int_as_float(r[0]) + __int_as_float(r[1]);
  }
  if constexpr (LANES <= 32) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(x), __float_as_int(x), false, false);
    x = __int_as_float(r[0]) + __int_as_float(r[1]);
  }
  return x;
}

// Element traits: VEC elements of T per lane, converted to float.
template <typename T>
struct Elem;

template <>
struct Elem<float> {
  static constexpr int kVec16 = 4;  // elements per 16 bytes
  template <int VEC>
  __device__ __forceinline__ static void load(const float* p, float (&o)[VEC]) {
    if constexpr (VEC % 4 == 0) {
#pragma unroll
      for (int q = 0; q < VEC / 4; ++q) {
        f32x4 v = *reinterpret_cast<const f32x4*>(p + 4 * q);
        o[4 * q] = v.x; o[4 * q + 1] = v.y; o[4 * q + 2] = v.z; o[4 * q + 3] = v.w;
      }
    } else if constexpr (VEC == 2) {
      f32x2 v = *reinterpret_cast<const f32x2*>(p);
      o[0] = v.x; o[1] = v.y;
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) o[e] = p[e];
    }
  }
  template <int VEC>
  __device__ __forceinline__ static void load_nt(const float* p, float (&o)[VEC]) {
    if constexpr (VEC == 4) {
      f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
      o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    } else {
      load<VEC>(p, o);
    }
  }
  template <int VEC>
  __device__ __forceinline__ static void store_nt(float* p, const float (&v)[VEC]) {
    if constexpr (VEC == 4) {
      f32x4 w = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(p));
    } else {
      store<VEC>(p, v);
    }
  }
  template <int VEC>
  __device__ __forceinline__ static void store(float* p, const float (&v)[VEC]) {
    if constexpr (VEC % 4 == 0) {
#pragma unroll
      for (int q = 0; q < VEC / 4; ++q) {
        f32x4 w = {v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
        *reinterpret_cast<f32x4*>(p + 4 * q) = w;
      }
    } else if constexpr (VEC == 2) {
      f32x2 w = {v[0], v[1]};
      *reinterpret_cast<f32x2*>(p) = w;
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) p[e] = v[e];
    }
  }
};

template <>
struct Elem<bf16_t> {
  static constexpr int kVec16 = 8;
  template <int VEC>
  __device__ __forceinline__ static void load(const bf16_t* p, float (&o)[VEC]) {
    if constexpr (VEC == 8) {
      u32x4 v = *reinterpret_cast<const u32x4*>(p);
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[2 * e] = __uint_as_float(w[e] << 16);
        o[2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
      }
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) o[e] = bf16_to_f32(p[e]);
    }
  }
  template <int VEC>
  __device__ __forceinline__ static void load_nt(const bf16_t* p, float (&o)[VEC]) {
    if constexpr (VEC == 8) {
      u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[2 * e] = __uint_as_float(w[e] << 16);
        o[2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
      }
    } else {
      load<VEC>(p, o);
    }
  }
  template <int VEC>
  __device__ __forceinline__ static void store_nt(bf16_t* p, const float (&v)[VEC]) {
    if constexpr (VEC == 8) {
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        w[e] = (uint32_t)f32_to_bf16(v[2 * e]) | ((uint32_t)f32_to_bf16(v[2 * e + 1]) << 16);
      u32x4 o = {w[0], w[1], w[2], w[3]};
      __builtin_nontemporal_store(o, reinterpret_cast<u32x4*>(p));
    } else {
      store<VEC>(p, v);
    }
  }
  template <int VEC>
  __device__ __forceinline__ static void store(bf16_t* p, const float (&v)[VEC]) {
    if constexpr (VEC == 8) {
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        w[e] = (uint32_t)f32_to_bf16(v[2 * e]) | ((uint32_t)f32_to_bf16(v[2 * e + 1]) << 16);
      u32x4 o = {w[0], w[1], w[2], w[3]};
      *reinterpret_cast<u32x4*>(p) = o;
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) p[e] = f32_to_bf16(v[e]);
    }
  }
};

// Raw 16-byte (or narrower) copy of VEC elements of T, bit-exact.
template <typename T, int VEC>
struct RawVec {
  static constexpr int kBytes = VEC * (int)sizeof(T);
  __device__ __forceinline__ static void copy(const T* __restrict__ src, T* __restrict__ dst) {
    if constexpr (kBytes == 16) {
      *reinterpret_cast<u32x4*>(dst) = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src));
    } else if constexpr (kBytes == 8) {
      *reinterpret_cast<u32x2*>(dst) = *reinterpret_cast<const u32x2*>(src);
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) dst[e] = src[e];
    }
  }
};

}  // namespace shiro
