// Device helpers shared by the fast refinement kernels: storage-type loads and stores
// (FP32, or bfloat16 widened to FP32), streaming (nontemporal) accesses, DPP lane
// shifts and the XCD-aware workgroup renumbering.
#ifndef ICR_SWEEP_IO_H
#define ICR_SWEEP_IO_H

#include "icr_internal.h"

namespace icr {
namespace sweep {

template <typename TS> struct Io;
template <> struct Io<float> {
  static __device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
  static __device__ __forceinline__ float2 ld2(const float* p) { return *reinterpret_cast<const float2*>(p); }
  static __device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
  static __device__ __forceinline__ void st1(float* p, float v) { *p = v; }
  static __device__ __forceinline__ void st2(float* p, float a, float b) {
    *reinterpret_cast<float2*>(p) = make_float2(a, b);
  }
};
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  return static_cast<uint32_t>(f32_to_bf16(a)) | (static_cast<uint32_t>(f32_to_bf16(b)) << 16);
}
template <> struct Io<bf16_t> {
  static __device__ __forceinline__ float4 ld4(const bf16_t* p) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  }
  static __device__ __forceinline__ float2 ld2(const bf16_t* p) {
    const uint32_t u = *reinterpret_cast<const uint32_t*>(p);
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
  }
  static __device__ __forceinline__ void st4(bf16_t* p, float4 v) {
    *reinterpret_cast<uint2*>(p) = make_uint2(pack_bf16(v.x, v.y), pack_bf16(v.z, v.w));
  }
  static __device__ __forceinline__ void st1(bf16_t* p, float v) { *p = f32_to_bf16(v); }
  static __device__ __forceinline__ void st2(bf16_t* p, float a, float b) {
    *reinterpret_cast<uint32_t*>(p) = pack_bf16(a, b);
  }
};

// Workgroups are handed to the 8 XCDs round-robin (workgroup w runs on XCD w % 8),
// and each XCD has its own L2. Renumber so that XCD k works through a contiguous
// range of logical tiles: neighbouring tiles, which read each other's halo, then
// share an L2 and run at about the same time.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int w, int n) {
  const int per = n / kXcds;
  return w < per * kXcds ? (w % kXcds) * per + w / kXcds : w;
}

// Streams that are read or written exactly once bypass cache retention.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
template <typename TS>
__device__ __forceinline__ float4 ld4_stream(const TS* p);
template <>
__device__ __forceinline__ float4 ld4_stream<float>(const float* p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
template <>
__device__ __forceinline__ float4 ld4_stream<bf16_t>(const bf16_t* p) {
  const nt_u2 u = __builtin_nontemporal_load(reinterpret_cast<const nt_u2*>(p));
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                     __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
}
template <typename TS>
__device__ __forceinline__ void st4_stream(TS* p, float4 v);
template <>
__device__ __forceinline__ void st4_stream<float>(float* p, float4 v) {
  const nt_f4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<nt_f4*>(p));
}
template <>
__device__ __forceinline__ void st4_stream<bf16_t>(bf16_t* p, float4 v) {
  const nt_u2 w = {pack_bf16(v.x, v.y), pack_bf16(v.z, v.w)};
  __builtin_nontemporal_store(w, reinterpret_cast<nt_u2*>(p));
}

// Cross-lane moves over the whole wavefront (DPP wave shifts); lane 0 (from_left) and
// lane 63 (from_right) read 0. A tile row of lanes may be any divisor of 64: the lanes
// at the ends of a row are halo lanes, so what crosses a row boundary is never used.
__device__ __forceinline__ float dpp_from_left(float v) {   // lane i <- lane i-1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_from_right(float v) {  // lane i <- lane i+1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

// Kernel arguments are fetched from memory by scalar loads that the compiler places
// after the kernel's first branches, so a kernel could wait for two or three dependent
// fetch rounds before its first vector load. Naming the arguments here, at the top of
// a kernel, makes them resident in scalar registers at once: one fetch round.
template <typename T>
__device__ __forceinline__ void pin_scalar(const T& v) {
  asm volatile("" ::"s"(v));
}
template <typename... T>
__device__ __forceinline__ void fetch_args(const T&... v) {
  (pin_scalar(v), ...);
}

}  // namespace sweep
}  // namespace icr

#endif  // ICR_SWEEP_IO_H
