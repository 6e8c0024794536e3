// Internal declarations shared by the ICR library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "icr.h"

namespace icr {

constexpr int kMaxLevels = ICR_MAX_DEPTH + 1;

constexpr int pow3(int d) { return d == 0 ? 1 : 3 * pow3(d - 1); }

// bfloat16 storage: the upper 16 bits of an IEEE float.
using bf16_t = uint16_t;

// ---------------------------------------------------------------------------
// Storage <-> arithmetic conversions
// ---------------------------------------------------------------------------
template <typename TS> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };
template <> struct Acc<bf16_t> { using type = float; };

__device__ __forceinline__ double load_acc(const double* p) { return *p; }
__device__ __forceinline__ float load_acc(const float* p) { return *p; }
__device__ __forceinline__ float load_acc(const bf16_t* p) {
  return __uint_as_float(static_cast<uint32_t>(*p) << 16);
}
__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

__device__ __forceinline__ void store_acc(double* p, double v) { *p = v; }
__device__ __forceinline__ void store_acc(float* p, float v) { *p = v; }
__device__ __forceinline__ bf16_t f32_to_bf16(float v) {
  // round to nearest even (gfx950 converts in hardware)
  return __builtin_bit_cast(bf16_t, static_cast<__bf16>(v));
}
__device__ __forceinline__ void store_acc(bf16_t* p, float v) { *p = f32_to_bf16(v); }

// dst[0 .. n) = src[0 .. n) widened to the arithmetic type, by `threads` threads with
// kU loads per thread in flight (a load-then-store loop would wait for every load in
// turn); reads use clamped in-bounds indices, only the stores are predicated.
template <int kU = 8, typename TA, typename TS>
__device__ __forceinline__ void copy_widen(TA* dst, const TS* src, int64_t n, int t, int threads) {
  for (int64_t base = t; base < n; base += int64_t(kU) * threads) {
    TA v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + int64_t(u) * threads;
      v[u] = load_acc(src + (i < n ? i : n - 1));
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = base + int64_t(u) * threads;
      if (i < n) dst[i] = v[u];
    }
  }
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct LevelMats {
  double* r64 = nullptr;  // [nsets][2^d][3^d]
  double* s64 = nullptr;  // [nsets][2^d][2^d], lower triangular
  void* r_c = nullptr;    // arithmetic type; stationary: [2^d][3^d]; charted: [2^d*3^d][nsets]
  void* s_c = nullptr;    // arithmetic type; stationary: [2^d][2^d]; charted: [2^d*2^d][nsets]
  int64_t nsets = 0;      // 1; per interior coarse pixel (2-D chart); per radial shell (cylinder)
  // plans built for hyperparameter gradients: d/d length of R and sqrtD, same layouts
  double* dr64 = nullptr;
  double* ds64 = nullptr;
  void* dr_c = nullptr;
  void* ds_c = nullptr;
  // Stationary levels: host copies of the FP32 matrices, passed to the fast kernels by
  // value, and the reflection-sector form of R (see sector_kernel in build_f64.hip).
  double* sector64 = nullptr;  // device scratch: [3^d] coefficients, [3^d] off-pattern, [3^d] on-pattern
  float h_r[8 * 27];
  float h_s[8 * 8];
  float h_sector[27];
  double sector_asym = 1.0;    // max off-pattern / max on-pattern entry of Q R P^-1
  bool sector_ok = false;      // R is reflection-symmetric to FP32 precision
  // Shell-charted 3-D levels: per set the reflection-sector coefficients of the second
  // and third axes with the first kept dense, and sqrtD (see shell_sector_kernel).
  float* shell_tab = nullptr;   // device, FP32 [nsets][kShellStride]
  double* shell_chk = nullptr;  // device, [nsets][2]: max off-pattern, max on-pattern |M|
  double shell_asym = 1.0;      // max over sets of off-pattern / on-pattern
  bool shell_ok = false;        // every set is symmetric in the two axes to FP32 precision
  // Plans built for hyperparameter gradients: the same fast-kernel forms of dR / dsqrtD
  // (d / d length), used by the gradient contraction.
  double* dsector64 = nullptr;
  float h_dsector[27];
  float h_ds[8 * 8];
  bool dsector_ok = false;
  float* dshell_tab = nullptr;
  double* dshell_chk = nullptr;
  bool dshell_ok = false;
};

// Floats per set of a shell table: C[9][2][3], sqrtD lower (36), padding to 16 bytes.
constexpr int kShellStride = 96;

// R is applied in the reflection-sector basis only when its asymmetric part is below
// FP32 rounding of R itself.
constexpr double kSectorTolerance = 1e-7;


}  // namespace icr

struct icr_plan {
  icr_config cfg;
  int ndim = 0;
  int depth = 0;
  int precision = 0;
  int charted = 0;   // matrices per pixel or per shell instead of one set per level
  int shell = 0;     // charted with one set per interior coarse index along the first axis
                     // (both log-radial charts: their distances do not depend on the angle)
  int device = 0;
  int shapes[icr::kMaxLevels][3];  // level shapes, axes beyond ndim are 1 (stored leading)
  int64_t offsets[icr::kMaxLevels + 1];
  int64_t n_xi = 0, n_out = 0, n0 = 0;
  int elem_bytes = 0;
  double origins[icr::kMaxLevels][3];
  double spacings[icr::kMaxLevels][3];
  double* l00_64 = nullptr;  // [n0][n0] lower Cholesky factor of K_00
  void* l00_c = nullptr;     // arithmetic type, row-major lower
  void* u00_c = nullptr;     // arithmetic type, row-major upper (= L00^T)
  double* dl00_64 = nullptr; // [n0][n0] d L00 / d length (plans built for hyperparameter gradients)
  int hypergrad = 0;         // built with ICR_FLAG_HYPERGRAD
  icr::LevelMats lev[ICR_MAX_DEPTH];
  int32_t clamped[icr::kMaxLevels];
  void* pool = nullptr;      // the one device allocation the plan owns
  int64_t pool_bytes = 0;
};

namespace icr {
// Shell levels keep an FP32 table with one row per set for the fast kernels: in 3-D the
// sector form of the two symmetric axes, in 2-D the dense R and sqrtD.
inline bool shell_tables(const icr_plan* p) { return p->shell && p->ndim >= 2; }
}  // namespace icr

namespace icr {

// error reporting (thread-local message)
void set_error(const std::string& msg);
void clear_error();

// ---------------------------------------------------------------------------
// Kernel launchers (each returns hipSuccess or the launch error)
// ---------------------------------------------------------------------------

// FP64 build
hipError_t launch_build_k00(const icr_plan* p, double* a, hipStream_t st);
hipError_t launch_cholesky_level0(const icr_plan* p, double* a, int32_t* counts, int32_t* status,
                                  hipStream_t st);
hipError_t launch_level0_convert(const icr_plan* p, hipStream_t st);
hipError_t launch_build_level(const icr_plan* p, int level, int32_t* counts, int32_t* status,
                              hipStream_t st);
hipError_t launch_level_convert(const icr_plan* p, int level, hipStream_t st);
hipError_t launch_level0_length_derivative(const icr_plan* p, double* scratch, hipStream_t st);
// MGVI vector operations (mgvi.hip): y = w^(1/2 or 1) * v; a -= c
hipError_t launch_weight(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* v, int64_t v_bs,
                         void* y, int64_t y_bs, int64_t n, bool half, hipStream_t st);
hipError_t launch_sub(const icr_plan* p, int64_t batch, void* a, const void* c, int64_t n, hipStream_t st);
// Hyperparameter gradients (hypergrad.hip)
int64_t hypergrad_partials(const icr_plan* p);
hipError_t launch_hyper_grad(const icr_plan* p, int64_t batch, const void* xi, const void* s,
                             const void* s_levels, const void* s_bar, const void* sbar_levels,
                             double* grad, double* partials, hipStream_t st);
hipError_t launch_sector(const icr_plan* p, int level, hipStream_t st);
hipError_t launch_shell_sector(const icr_plan* p, int level, hipStream_t st);

// level 0 apply: out = L00 in (forward) / U00 in (+ add) (adjoint); w optional
struct Level0Args {
  const void* in; int64_t in_bs;
  void* out; int64_t out_bs;
  const void* w; int64_t w_bs;    // forward only: out *= w
  const void* add; int64_t add_bs;  // adjoint only: out += add
  int64_t batch;
  const int32_t* halt = nullptr;  // device flag: when set (non-zero) the kernel does nothing
};
hipError_t launch_level0_fwd(const icr_plan* p, const Level0Args& a, hipStream_t st);
hipError_t launch_level0_adj(const icr_plan* p, const Level0Args& a, hipStream_t st);

// one refinement level
struct RefineFwdArgs {
  const void* s_in; int64_t s_in_bs;   // coarse field, level l
  const void* xi; int64_t xi_bs;       // excitations of level l+1
  void* s_out; int64_t s_out_bs;       // fine field, level l+1
  const void* w; int64_t w_bs;         // optional: s_out *= w (arithmetic type)
  int64_t batch;
  // gradient contraction (try_refine3_dot_sector): instead of storing the fine field,
  // sum <dot, fine field> per workgroup into partial[b * partial_bs + workgroup]
  const void* dot = nullptr; int64_t dot_bs = 0;
  double* partial = nullptr; int64_t partial_bs = 0;
  double* partial_sig = nullptr;       // and <dot, value sqrtD xi>, same layout
  const int32_t* halt = nullptr;       // device flag: when set (non-zero) the kernel does nothing
};
struct RefineAdjArgs {
  const void* y; int64_t y_bs;          // fine cotangent, level l+1
  void* xi_bar; int64_t xi_bar_bs;      // excitation cotangent, level l+1
  void* s_bar; int64_t s_bar_bs;        // coarse cotangent, level l
  const void* add; int64_t add_bs;      // optional: xi_bar += add (storage type)
  int64_t batch;
  const int32_t* halt = nullptr;        // device flag: when set (non-zero) the kernel does nothing
};
// The metric's last level both ways in one launch (M v = L^T (w * L v) + v at the finest
// level): the coarse field s_l, the level's v (excitations of the forward, values added
// to the excitation cotangent), w (arithmetic type) in; v's excitation cotangent plus v
// and the coarse cotangent s_bar_l out.
struct RefineMetricArgs {
  const void* s_in; int64_t s_in_bs;    // coarse field, level l
  const void* v; int64_t v_bs;          // level l+1 part of v
  const void* w; int64_t w_bs;          // weights of level l+1 (arithmetic type)
  void* out; int64_t out_bs;            // level l+1 part of M v
  void* s_bar; int64_t s_bar_bs;        // coarse cotangent, level l
  int64_t batch;
  const int32_t* halt = nullptr;        // device flag: when set (non-zero) the kernel does nothing
  // optional: per-workgroup partial sums of <s, w * s> over the level (s the forward's
  // fine field) at dot[b * dot_bs + workgroup], FP64, each in a fixed order
  double* dot = nullptr; int64_t dot_bs = 0;
};
hipError_t launch_refine_fwd(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st);
hipError_t launch_refine_adj(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st);
// The 3-D fast forward with the derivative matrices of the level and a dot-product
// epilogue (a.dot, a.partial, a.partial_sig); reports the workgroups per sample
// (partial sums written to each) in *wgs. False when the level or the buffers do not qualify or more than max_wgs
// workgroups per sample would be needed.
bool try_refine3_dot_sector(const icr_plan* p, int level, const RefineFwdArgs& a, int64_t max_wgs,
                            hipStream_t st, hipError_t* err, int64_t* wgs);
hipError_t launch_refine_fwd_generic(const icr_plan* p, int level, const RefineFwdArgs& a,
                                     hipStream_t st);
// Specialised kernels: return false (launching nothing) when the level or the buffers
// do not qualify; otherwise launch and report the launch status in *err.
bool try_refine3_fwd_sector(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st,
                            hipError_t* err);
bool try_refine3_adj_sector(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st,
                            hipError_t* err);
bool try_refine2_fwd(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st, hipError_t* err);
bool try_refine2_adj(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st, hipError_t* err);
// Whether the fused kernel takes this level and these buffers (else the caller runs the
// two sweeps), and its launch.
bool refine2_metric_ok(const icr_plan* p, int level, const RefineMetricArgs& a);
int64_t refine2_metric_partials(const icr_plan* p, int level, int64_t batch);  // workgroups per sample
hipError_t launch_refine2_metric(const icr_plan* p, int level, const RefineMetricArgs& a, hipStream_t st);
hipError_t launch_refine_adj_generic(const icr_plan* p, int level, const RefineAdjArgs& a,
                                     hipStream_t st);

// The first K refinement levels (and level 0 when its factor is small) of a sweep in one
// launch (fused.hip). fused_levels returns K (0: no fusion) and whether level 0 is included.
int fused_levels(const icr_plan* p, bool* level0);
hipError_t launch_fused_fwd(const icr_plan* p, int K, bool level0, int64_t batch, const void* xi, void* ws,
                            int64_t ws_bs, void* out, int64_t out_bs, const void* w, int64_t w_bs,
                            const int32_t* halt, hipStream_t st);
hipError_t launch_fused_adj(const icr_plan* p, int K, bool level0, int64_t batch, const void* y, int64_t y_bs,
                            void* xi_bar, void* ws, int64_t ws_bs, const void* add, const int32_t* halt,
                            hipStream_t st);

// A kernel whose launch carries a halt flag returns at once while the flag is set: the
// early-stopping CG enqueues all of its iterations and stops them on the device.
__device__ __forceinline__ bool halted(const int32_t* halt) {
  return halt != nullptr && *halt != 0;
}

// conjugate gradients on the metric (cg.hip); `metric` applies L^T W L + 1, its kernels
// doing nothing while `halt` (NULL: never) is set. absdelta > 0 stops a sample once one
// step lowers its CG energy by less than absdelta; iterations_done (optional, device
// [batch]) receives the steps each sample took.
// When `dot` is not NULL and the metric's finest level runs in the fused kernel with at
// most dot_cap wavefronts per sample, that kernel also writes its partial sums of
// <L v, w * L v> (dot[b * dot_cap + k], k < *ndot) and *ndot is their count; else *ndot = 0.
using MetricFn = hipError_t (*)(const icr_plan*, int64_t, const void*, int64_t, const void*, void*, void*,
                                const int32_t*, hipStream_t, double* dot, int dot_cap, int* ndot);
int64_t cg_workspace_bytes(const icr_plan* p, int64_t batch);
hipError_t launch_cg(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* bvec,
                     void* x, int32_t iterations, double absdelta, int32_t* iterations_done, double* norms,
                     void* workspace, hipStream_t st, MetricFn metric);

}  // namespace icr
