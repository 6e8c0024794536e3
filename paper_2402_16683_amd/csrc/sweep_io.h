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

// Level slices that start off a vector boundary: a level-0 size n0^d that is not a
// multiple of 4 shifts every later level's slice of a xi-shaped buffer (and every sample
// of a batch) by 1-3 elements. These storage tags keep the layout and the element size but
// read and write element by element instead of in vectors (still contiguous over a
// wavefront), so such plans run the same kernels with the same arithmetic.
struct f32u {
  float v;
};
struct bf16u {
  bf16_t v;
};
template <typename TS> struct IsF32Storage { static constexpr bool value = false; };
template <> struct IsF32Storage<float> { static constexpr bool value = true; };
template <> struct IsF32Storage<f32u> { static constexpr bool value = true; };

template <> struct Io<f32u> {
  static __device__ __forceinline__ float4 ld4(const f32u* p) { return make_float4(p[0].v, p[1].v, p[2].v, p[3].v); }
  static __device__ __forceinline__ float2 ld2(const f32u* p) { return make_float2(p[0].v, p[1].v); }
  static __device__ __forceinline__ void st4(f32u* p, float4 v) {
    p[0].v = v.x; p[1].v = v.y; p[2].v = v.z; p[3].v = v.w;
  }
  static __device__ __forceinline__ void st1(f32u* p, float v) { p->v = v; }
  static __device__ __forceinline__ void st2(f32u* p, float a, float b) { p[0].v = a; p[1].v = b; }
};
__device__ __forceinline__ float widen_bf16(bf16_t u) { return __uint_as_float(static_cast<uint32_t>(u) << 16); }
template <> struct Io<bf16u> {
  static __device__ __forceinline__ float4 ld4(const bf16u* p) {
    return make_float4(widen_bf16(p[0].v), widen_bf16(p[1].v), widen_bf16(p[2].v), widen_bf16(p[3].v));
  }
  static __device__ __forceinline__ float2 ld2(const bf16u* p) { return make_float2(widen_bf16(p[0].v), widen_bf16(p[1].v)); }
  static __device__ __forceinline__ void st4(bf16u* p, float4 v) {
    p[0].v = f32_to_bf16(v.x); p[1].v = f32_to_bf16(v.y); p[2].v = f32_to_bf16(v.z); p[3].v = f32_to_bf16(v.w);
  }
  static __device__ __forceinline__ void st1(bf16u* p, float v) { p->v = f32_to_bf16(v); }
  static __device__ __forceinline__ void st2(bf16u* p, float a, float b) {
    p[0].v = f32_to_bf16(a); p[1].v = f32_to_bf16(b);
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
template <>
__device__ __forceinline__ float4 ld4_stream<f32u>(const f32u* p) {
  return make_float4(__builtin_nontemporal_load(&p[0].v), __builtin_nontemporal_load(&p[1].v),
                     __builtin_nontemporal_load(&p[2].v), __builtin_nontemporal_load(&p[3].v));
}
template <>
__device__ __forceinline__ float4 ld4_stream<bf16u>(const bf16u* p) {
  return make_float4(widen_bf16(__builtin_nontemporal_load(&p[0].v)), widen_bf16(__builtin_nontemporal_load(&p[1].v)),
                     widen_bf16(__builtin_nontemporal_load(&p[2].v)), widen_bf16(__builtin_nontemporal_load(&p[3].v)));
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
template <>
__device__ __forceinline__ void st4_stream<f32u>(f32u* p, float4 v) {
  __builtin_nontemporal_store(v.x, &p[0].v);
  __builtin_nontemporal_store(v.y, &p[1].v);
  __builtin_nontemporal_store(v.z, &p[2].v);
  __builtin_nontemporal_store(v.w, &p[3].v);
}
template <>
__device__ __forceinline__ void st4_stream<bf16u>(bf16u* p, float4 v) {
  __builtin_nontemporal_store(f32_to_bf16(v.x), &p[0].v);
  __builtin_nontemporal_store(f32_to_bf16(v.y), &p[1].v);
  __builtin_nontemporal_store(f32_to_bf16(v.z), &p[2].v);
  __builtin_nontemporal_store(f32_to_bf16(v.w), &p[3].v);
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
