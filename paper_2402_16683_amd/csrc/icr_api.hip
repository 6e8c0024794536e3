// C ABI of the ICR library: configuration checks, the plan (level sizes, offsets,
// device matrices), and the level-by-level drivers of the forward sweep, its
// adjoint and the metric. Declarations and contracts are in include/icr.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "host_checks.h"
#include "icr_internal.h"

namespace icr {
namespace {
thread_local std::string g_error;
}
void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }
}  // namespace icr

namespace {

using icr::kMaxLevels;

icr_status fail(icr_status s, const std::string& msg) {
  icr::set_error(msg);
  return s;
}

#define ICR_HIP_TRY(expr)                                                                     \
  do {                                                                                        \
    const hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(ICR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int elem_bytes_of(int precision) {
  return precision == ICR_F64 ? 8 : precision == ICR_F32 ? 4 : 2;
}
int acc_bytes_of(int precision) { return precision == ICR_F64 ? 8 : 4; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

icr_status check_config(const icr_config* c) {
  if (!c) return fail(ICR_ERR_INVALID_ARG, "cfg is NULL");
  if (c->ndim < 1 || c->ndim > 3) return fail(ICR_ERR_INVALID_ARG, "ndim must be 1, 2 or 3");
  if (c->depth < 0 || c->depth > ICR_MAX_DEPTH)
    return fail(ICR_ERR_INVALID_ARG, "depth must be in [0, " + std::to_string(ICR_MAX_DEPTH) + "]");
  if (c->kernel < ICR_MATERN12 || c->kernel > ICR_SQEXP) return fail(ICR_ERR_INVALID_ARG, "unknown kernel");
  if (c->chart != ICR_CHART_REGULAR && c->chart != ICR_CHART_LOGRADIAL_2D &&
      c->chart != ICR_CHART_LOGRADIAL_CYL_3D)
    return fail(ICR_ERR_INVALID_ARG, "unknown chart");
  if (c->chart == ICR_CHART_LOGRADIAL_2D) {
    if (c->ndim != 2) return fail(ICR_ERR_INVALID_ARG, "the log-radial chart needs ndim == 2");
    if (!finite_pos(c->chart_params[0]) || !std::isfinite(c->chart_params[1]) ||
        !std::isfinite(c->chart_params[2]))
      return fail(ICR_ERR_INVALID_ARG, "log-radial chart needs r0 > 0 and finite growth/angle");
  }
  if (c->chart == ICR_CHART_LOGRADIAL_CYL_3D) {
    if (c->ndim != 3) return fail(ICR_ERR_INVALID_ARG, "the log-radial cylinder chart needs ndim == 3");
    if (!finite_pos(c->chart_params[0]) || !std::isfinite(c->chart_params[1]) ||
        !std::isfinite(c->chart_params[2]) || !finite_pos(c->chart_params[3]))
      return fail(ICR_ERR_INVALID_ARG,
                  "log-radial cylinder chart needs r0 > 0, finite growth/angle and height scale > 0");
  }
  if (c->precision < ICR_F64 || c->precision > ICR_BF16_F32ACC)
    return fail(ICR_ERR_INVALID_ARG, "unknown precision");
  if (c->flags & ~(ICR_FLAG_NO_CLAMP | ICR_FLAG_HYPERGRAD)) return fail(ICR_ERR_INVALID_ARG, "unknown flag bits");
  if (c->reserved != 0) return fail(ICR_ERR_INVALID_ARG, "reserved must be 0");
  if (!finite_pos(c->scale) || !finite_pos(c->length))
    return fail(ICR_ERR_INVALID_ARG, "scale and length must be finite and > 0");
  int64_t n0 = 1;
  for (int a = 0; a < c->ndim; ++a) {
    if (!finite_pos(c->distances0[a])) return fail(ICR_ERR_INVALID_ARG, "distances0 must be finite and > 0");
    if (c->shape0[a] < 1 || c->shape0[a] > 65536) return fail(ICR_ERR_INVALID_ARG, "shape0 out of range");
    n0 *= c->shape0[a];
  }
  if (n0 > 4096)
    return fail(ICR_ERR_UNSUPPORTED, "level 0 has more than 4096 pixels (dense Cholesky limit)");
  // every refined level needs an interior; sizes must stay addressable
  for (int a = 0; a < c->ndim; ++a) {
    int64_t n = c->shape0[a];
    for (int l = 0; l < c->depth; ++l) {
      if (n < 3) return fail(ICR_ERR_INVALID_ARG, "a refined level has fewer than 3 pixels along an axis");
      n = 2 * (n - 2);
      if (n > (int64_t(1) << 24)) return fail(ICR_ERR_INVALID_ARG, "level size exceeds 2^24 pixels per axis");
    }
  }
  return ICR_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

bool aligned(const void* p, int el) { return (reinterpret_cast<uintptr_t>(p) % el) == 0; }

void* at(const void* base, int64_t elems, int el) {
  return static_cast<char*>(const_cast<void*>(base)) + elems * el;
}

// Adjoint sweep from the fine cotangent y (level `depth`) down to level 0. Every kernel of
// the sweep does nothing while the device flag `halt` is set (NULL: never).
// With top < depth the sweep starts at level `top`, whose cotangent is y (the metric's
// fused finest level leaves it in the workspace).
icr_status run_adjoint(const icr_plan* p, int64_t batch, const void* y, int64_t y_bs, void* xi_bar,
                       void* ws, int64_t ws_bs, const void* add, hipStream_t st, const int32_t* halt = nullptr,
                       int top = -1) {
  const int el = p->elem_bytes;
  const int L = top < 0 ? p->depth : top;
  if (L == 0) {
    icr::Level0Args a{y, y_bs, xi_bar, p->n_xi, nullptr, 0, add, add ? p->n_xi : 0, batch, halt};
    ICR_HIP_TRY(icr::launch_level0_adj(p, a, st));
    return ICR_OK;
  }
  bool fuse0 = false;
  const int K = icr::fused_levels(p, &fuse0);  // the smallest levels in one launch
  if (K > L) return fail(ICR_ERR_UNSUPPORTED, "adjoint sweep starts inside the fused levels");
  for (int l = L - 1; l >= K; --l) {
    icr::RefineAdjArgs a;
    a.y = l == L - 1 ? y : at(ws, p->offsets[l + 1], el);
    a.y_bs = l == L - 1 ? y_bs : ws_bs;
    a.xi_bar = at(xi_bar, p->offsets[l + 1], el);
    a.xi_bar_bs = p->n_xi;
    a.s_bar = at(ws, p->offsets[l], el);
    a.s_bar_bs = ws_bs;
    a.add = add ? at(add, p->offsets[l + 1], el) : nullptr;
    a.add_bs = add ? p->n_xi : 0;
    a.batch = batch;
    a.halt = halt;
    ICR_HIP_TRY(icr::launch_refine_adj(p, l, a, st));
  }
  if (K > 0)
    ICR_HIP_TRY(icr::launch_fused_adj(p, K, fuse0, batch, K == L ? y : at(ws, p->offsets[K], el),
                                      K == L ? y_bs : ws_bs, xi_bar, ws, ws_bs, add, halt, st));
  if (!fuse0) {
    icr::Level0Args a{ws, ws_bs, xi_bar, p->n_xi, nullptr, 0, add, add ? p->n_xi : 0, batch, halt};
    ICR_HIP_TRY(icr::launch_level0_adj(p, a, st));
  }
  return ICR_OK;
}

// Forward sweep; the last level goes to `out` (stride out_bs), optionally times w. Every
// kernel does nothing while the device flag `halt` is set (NULL: never).
// With stop < depth the sweep ends at level `stop`, which stays in the workspace (out
// and w are not used).
icr_status run_forward(const icr_plan* p, int64_t batch, const void* xi, void* out, int64_t out_bs,
                       void* ws, int64_t ws_bs, const void* w, int64_t w_bs, hipStream_t st,
                       const int32_t* halt = nullptr, int stop = -1) {
  const int el = p->elem_bytes;
  const int L = stop < 0 ? p->depth : stop;
  if (L < p->depth) {  // level L is an intermediate: it goes to the workspace
    out = at(ws, p->offsets[L], el);
    out_bs = ws_bs;
    w = nullptr;
  }
  if (L == 0) {
    icr::Level0Args a{xi, p->n_xi, out, out_bs, w, w_bs, nullptr, 0, batch, halt};
    ICR_HIP_TRY(icr::launch_level0_fwd(p, a, st));
    return ICR_OK;
  }
  bool fuse0 = false;
  const int K = icr::fused_levels(p, &fuse0);  // the smallest levels in one launch
  if (K > L) return fail(ICR_ERR_UNSUPPORTED, "forward sweep ends inside the fused levels");
  if (!fuse0) {
    icr::Level0Args a0{xi, p->n_xi, at(ws, p->offsets[0], el), ws_bs, nullptr, 0, nullptr, 0, batch, halt};
    ICR_HIP_TRY(icr::launch_level0_fwd(p, a0, st));
  }
  if (K > 0)
    ICR_HIP_TRY(icr::launch_fused_fwd(p, K, fuse0, batch, xi, ws, ws_bs, K == L ? out : nullptr, out_bs,
                                      K == L ? w : nullptr, w_bs, halt, st));
  for (int l = K; l < L; ++l) {
    icr::RefineFwdArgs a;
    a.s_in = at(ws, p->offsets[l], el);
    a.s_in_bs = ws_bs;
    a.xi = at(xi, p->offsets[l + 1], el);
    a.xi_bs = p->n_xi;
    a.s_out = l == L - 1 ? out : at(ws, p->offsets[l + 1], el);
    a.s_out_bs = l == L - 1 ? out_bs : ws_bs;
    a.w = l == L - 1 ? w : nullptr;
    a.w_bs = w_bs;
    a.batch = batch;
    a.halt = halt;
    ICR_HIP_TRY(icr::launch_refine_fwd(p, l, a, st));
  }
  return ICR_OK;
}

icr_status check_call(const icr_plan* p, int64_t batch) {
  if (!p) return fail(ICR_ERR_INVALID_ARG, "plan is NULL");
  if (batch < 0) return fail(ICR_ERR_INVALID_ARG, "batch must be >= 0");
  return ICR_OK;
}

// The metric v -> L^T (w * L v) + v on `batch` samples, with a workspace of n_xi elements
// per sample (the levels at their offsets). The finest level's weighted field goes to
// offsets[depth] and the adjoint reads it back, except where a fused kernel takes the
// finest level both ways: the forward then stops one level short and that kernel leaves
// the coarse cotangent at offsets[depth] (not at offsets[depth-1], where the coarse
// field it reads lies). The kernels do nothing while the device flag `halt` is set
// (NULL: never). With `dot` (see MetricFn) the fused kernel also writes its partial sums
// of <L v, w * L v>; *ndot gets their count per sample, 0 where none were written.
icr_status run_metric(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* v, void* out,
                      void* ws, hipStream_t st, const int32_t* halt = nullptr, double* dot = nullptr,
                      int dot_cap = 0, int* ndot = nullptr) {
  if (ndot) *ndot = 0;
  const int el = p->elem_bytes;
  const int64_t bs = p->n_xi;
  const int L = p->depth;
  void* top = at(ws, p->offsets[L], el);
  bool fuse0 = false;
  if (L >= 1 && icr::fused_levels(p, &fuse0) < L) {
    icr::RefineMetricArgs a;
    a.s_in = at(ws, p->offsets[L - 1], el);
    a.s_in_bs = bs;
    a.v = at(v, p->offsets[L], el);
    a.v_bs = bs;
    a.w = w;
    a.w_bs = w_bs;
    a.out = at(out, p->offsets[L], el);
    a.out_bs = bs;
    a.s_bar = top;
    a.s_bar_bs = bs;
    a.batch = batch;
    a.halt = halt;
    if (icr::refine2_metric_ok(p, L - 1, a)) {
      const int64_t parts = icr::refine2_metric_partials(p, L - 1, batch);
      if (dot && ndot && parts <= dot_cap) {
        a.dot = dot;
        a.dot_bs = dot_cap;
        *ndot = static_cast<int>(parts);
      }
      icr_status r = run_forward(p, batch, v, nullptr, 0, ws, bs, nullptr, 0, st, halt, L - 1);
      if (r != ICR_OK) return r;
      ICR_HIP_TRY(icr::launch_refine2_metric(p, L - 1, a, st));
      return run_adjoint(p, batch, top, bs, out, ws, bs, v, st, halt, L - 1);
    }
  }
  icr_status r = run_forward(p, batch, v, top, bs, ws, bs, w, w_bs, st, halt);
  if (r != ICR_OK) return r;
  return run_adjoint(p, batch, top, bs, out, ws, bs, v, st, halt);
}

// The metric as CG applies it (see run_metric and MetricFn).
hipError_t metric_for_cg(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* v,
                         void* out, void* ws, const int32_t* halt, hipStream_t st, double* dot, int dot_cap,
                         int* ndot) {
  return run_metric(p, batch, w, w_bs, v, out, ws, st, halt, dot, dot_cap, ndot) == ICR_OK ? hipSuccess
                                                                                          : hipErrorLaunchFailure;
}

// Argument checks shared by the CG entry points.
icr_status check_cg_call(const icr_plan* p, int64_t batch, const void* w, int64_t w_batch_stride, const void* b,
                         const void* x, int32_t iterations, const double* residual_norms, const void* workspace) {
  if (p->precision == ICR_BF16_F32ACC) return fail(ICR_ERR_UNSUPPORTED, "CG needs an FP64 or FP32 plan");
  if (iterations < 0) return fail(ICR_ERR_INVALID_ARG, "iterations must be >= 0");
  if (batch > 65535) return fail(ICR_ERR_INVALID_ARG, "CG takes at most 65535 right-hand sides per call");
  if (batch == 0) return ICR_OK;
  const int el = p->elem_bytes;
  if (!w || !b || !x || !workspace) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (w_batch_stride != 0 && w_batch_stride < p->n_out)
    return fail(ICR_ERR_INVALID_ARG, "w_batch_stride must be 0 or >= n_out");
  if (!aligned(b, el) || !aligned(x, el) || !aligned(w, el) || !aligned(workspace, 256) ||
      (residual_norms && !aligned(residual_norms, 8)))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned (workspace needs 256 bytes)");
  const size_t nx = size_t(batch) * p->n_xi * el;
  const size_t nw = size_t(icr::cg_workspace_bytes(p, batch));
  if (icr::overlaps(b, nx, x, nx) || icr::overlaps(b, nx, workspace, nw) || icr::overlaps(x, nx, workspace, nw))
    return fail(ICR_ERR_INVALID_ARG, "b, x and workspace overlap");
  return ICR_OK;
}

// Host copies of a level's device results that the fast kernels need on the host:
// staged by asynchronous copies on the build stream, used after one synchronisation.
struct HostStage {
  std::vector<double> chk, dchk;    // shell symmetry checks (value, derivative)
  double sec[3 * 27], dsec[3 * 27]; // sector forms (value, derivative)
  float hr[8 * 27], hs[8 * 8], hds[8 * 8];
};

// Worst off-pattern / on-pattern ratio over a shell table's sets (host copy of the check array).
double shell_asymmetry(const std::vector<double>& chk, int64_t nsets) {
  double w = 0.0;
  for (int64_t s = 0; s < nsets; ++s) {
    const double off = chk[2 * s], on = chk[2 * s + 1];
    w = std::fmax(w, on > 0.0 ? off / on : 1.0);
    if (!std::isfinite(off) || !std::isfinite(on)) w = 1.0;
  }
  return w;
}

// Sector coefficients (FP32) and the off / on-pattern ratio of a host copy of a sector array.
void sector_host(const double* sec, int nw, float* coef, double* asym) {
  double off = 0.0, on = 0.0;
  for (int t = 0; t < nw; ++t) {
    coef[t] = static_cast<float>(sec[t]);
    off = std::fmax(off, sec[nw + t]);
    on = std::fmax(on, sec[2 * nw + t]);
  }
  *asym = on > 0.0 ? off / on : 1.0;
}

// Enqueue on `st` the copies of a level's device results its host copies are made from
// (nothing for FP64 plans and dense 2-D shell rows).
icr_status stage_host_copies(const icr_plan* p, int level, HostStage* hs, hipStream_t st) {
  const icr::LevelMats& m = p->lev[level];
  if (p->precision == ICR_F64 || (icr::shell_tables(p) && p->ndim == 2)) return ICR_OK;
  if (icr::shell_tables(p)) {
    hs->chk.resize(static_cast<size_t>(2 * m.nsets));
    ICR_HIP_TRY(hipMemcpyAsync(hs->chk.data(), m.shell_chk, sizeof(double) * hs->chk.size(), hipMemcpyDeviceToHost, st));
    if (m.dshell_tab) {
      hs->dchk.resize(static_cast<size_t>(2 * m.nsets));
      ICR_HIP_TRY(hipMemcpyAsync(hs->dchk.data(), m.dshell_chk, sizeof(double) * hs->dchk.size(),
                                 hipMemcpyDeviceToHost, st));
    }
    return ICR_OK;
  }
  if (p->charted) return ICR_OK;
  const int nc = 1 << p->ndim, nw = icr::pow3(p->ndim);
  ICR_HIP_TRY(hipMemcpyAsync(hs->hr, m.r_c, sizeof(float) * nc * nw, hipMemcpyDeviceToHost, st));
  ICR_HIP_TRY(hipMemcpyAsync(hs->hs, m.s_c, sizeof(float) * nc * nc, hipMemcpyDeviceToHost, st));
  ICR_HIP_TRY(hipMemcpyAsync(hs->sec, m.sector64, sizeof(double) * 3 * nw, hipMemcpyDeviceToHost, st));
  if (m.dsector64) {
    ICR_HIP_TRY(hipMemcpyAsync(hs->hds, m.ds_c, sizeof(float) * nc * nc, hipMemcpyDeviceToHost, st));
    ICR_HIP_TRY(hipMemcpyAsync(hs->dsec, m.dsector64, sizeof(double) * 3 * nw, hipMemcpyDeviceToHost, st));
  }
  return ICR_OK;
}

// Host copies of a stationary level's FP32 matrices and its sector form (the fast
// kernels take them by value), and the symmetry checks of the sector and shell forms
// (also of the length derivatives on plans built for hyperparameter gradients), from a
// completed stage_host_copies.
void apply_host_copies(icr_plan* p, int level, const HostStage& hs) {
  icr::LevelMats& m = p->lev[level];
  m.sector_ok = m.shell_ok = m.dsector_ok = m.dshell_ok = false;
  m.sector_asym = 1.0;
  m.shell_asym = 1.0;
  if (p->precision == ICR_F64) return;
  const auto ok = [](double asym) { return std::isfinite(asym) && asym <= icr::kSectorTolerance; };
  if (icr::shell_tables(p) && p->ndim == 2) {  // dense rows: always usable
    m.shell_ok = true;
    return;
  }
  if (icr::shell_tables(p)) {
    m.shell_asym = shell_asymmetry(hs.chk, m.nsets);
    m.shell_ok = ok(m.shell_asym);
    if (m.dshell_tab) m.dshell_ok = ok(shell_asymmetry(hs.dchk, m.nsets));
    return;
  }
  if (p->charted) return;
  const int nc = 1 << p->ndim, nw = icr::pow3(p->ndim);
  std::memcpy(m.h_r, hs.hr, sizeof(float) * nc * nw);
  std::memcpy(m.h_s, hs.hs, sizeof(float) * nc * nc);
  sector_host(hs.sec, nw, m.h_sector, &m.sector_asym);
  m.sector_ok = ok(m.sector_asym);
  if (m.dsector64) {
    std::memcpy(m.h_ds, hs.hds, sizeof(float) * nc * nc);
    double asym = 1.0;
    sector_host(hs.dsec, nw, m.h_dsector, &asym);
    m.dsector_ok = ok(asym);
  }
}

// The same for one level, synchronously on `st` (after icr_plan_set_refinement).
icr_status refresh_host_copies(icr_plan* p, int level, hipStream_t st) {
  HostStage hs;
  icr_status r = stage_host_copies(p, level, &hs, st);
  if (r != ICR_OK) return r;
  ICR_HIP_TRY(hipStreamSynchronize(st));
  apply_host_copies(p, level, hs);
  return ICR_OK;
}

// Device scratch of icr_metric_apply_static: a file-scope array every GPU the library runs
// on holds until the process ends (64 MiB each). Host code never uses the array's name as
// an address: each device's copy sits at its own device address, looked up once per device
// with hipGetSymbolAddress and kept in scratch_ptr.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (looked up on the first call on that device).
icr_status scratch_ptr(void** out) {
  int dev = 0;
  ICR_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ICR_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    ICR_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(ICR_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ICR_OK;
}

}  // namespace

namespace icr {
hipError_t launch_refine_fwd(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (try_refine3_fwd_sector(p, level, a, st, &e)) return e;
  if (try_refine2_fwd(p, level, a, st, &e)) return e;
  return launch_refine_fwd_generic(p, level, a, st);
}
hipError_t launch_refine_adj(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (try_refine3_adj_sector(p, level, a, st, &e)) return e;
  if (try_refine2_adj(p, level, a, st, &e)) return e;
  return launch_refine_adj_generic(p, level, a, st);
}
}  // namespace icr

extern "C" {

int32_t icr_version(void) { return 100; }

const char* icr_last_error(void) { return icr::g_error.c_str(); }

icr_status icr_build_matrices(const icr_config* cfg, void* hip_stream, icr_plan** out_plan) {
  icr::clear_error();
  if (!out_plan) return fail(ICR_ERR_INVALID_ARG, "out_plan is NULL");
  *out_plan = nullptr;
  const icr_status cs = check_config(cfg);
  if (cs != ICR_OK) return cs;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // launch checks below read the thread's last error: start from a clean one, so an
  // earlier unchecked call of this thread cannot fail the build
  (void)hipGetLastError();

  icr_plan* p = new (std::nothrow) icr_plan;
  if (!p) return fail(ICR_ERR_OUT_OF_MEMORY, "host allocation of the plan failed");
  p->cfg = *cfg;
  p->ndim = cfg->ndim;
  p->depth = cfg->depth;
  p->precision = cfg->precision;
  p->charted = cfg->chart != ICR_CHART_REGULAR;
  // both charts are invariant along their angular (and height) axes: one matrix set per
  // interior coarse index along the first (radial) axis describes a level exactly
  p->shell = cfg->chart == ICR_CHART_LOGRADIAL_CYL_3D || cfg->chart == ICR_CHART_LOGRADIAL_2D;
  p->hypergrad = (cfg->flags & ICR_FLAG_HYPERGRAD) ? 1 : 0;
  p->elem_bytes = elem_bytes_of(cfg->precision);
  const int d = p->ndim;
  for (int l = 0; l < kMaxLevels; ++l)
    for (int a = 0; a < 3; ++a) p->shapes[l][a] = 1;
  for (int a = 0; a < d; ++a) {
    int n = cfg->shape0[a];
    for (int l = 0; l <= p->depth; ++l) {
      p->shapes[l][3 - d + a] = n;
      n = 2 * (n - 2);
    }
  }
  int64_t off = 0;
  for (int l = 0; l <= p->depth; ++l) {
    p->offsets[l] = off;
    off += int64_t(p->shapes[l][0]) * p->shapes[l][1] * p->shapes[l][2];
  }
  p->offsets[p->depth + 1] = off;
  p->n_xi = off;
  p->n_out = off - p->offsets[p->depth];
  p->n0 = p->offsets[1] - p->offsets[0];
  for (int a = 0; a < 3; ++a) {
    double delta = a < d ? cfg->distances0[a] : 0.0, origin = 0.0;
    for (int l = 0; l <= p->depth; ++l) {
      p->spacings[l][a] = delta;
      p->origins[l][a] = origin;
      origin += 0.75 * delta;
      delta *= 0.5;
    }
  }
  for (int l = 0; l < kMaxLevels; ++l) p->clamped[l] = 0;

  // one pool: level-0 factors, per-level matrices, status words
  const int ab = acc_bytes_of(p->precision);
  const int nc = 1 << d, nw = icr::pow3(d);
  size_t bytes = 0;
  const size_t off_l64 = bytes; bytes = align_up(bytes + size_t(p->n0) * p->n0 * 8);
  const size_t off_lc = bytes; bytes = align_up(bytes + size_t(p->n0) * p->n0 * ab);
  const size_t off_uc = bytes; bytes = align_up(bytes + size_t(p->n0) * p->n0 * ab);
  const size_t off_dl00 = bytes; bytes = align_up(bytes + (p->hypergrad ? size_t(p->n0) * p->n0 * 8 : 0));
  size_t off_lev[ICR_MAX_DEPTH][14];
  for (int l = 0; l < p->depth; ++l) {
    int64_t nsets = 1;
    if (p->shell)
      nsets = p->shapes[l][3 - d] - 2;  // one set per radial shell (first axis)
    else if (p->charted)
      for (int a = 0; a < d; ++a) nsets *= p->shapes[l][3 - d + a] - 2;
    p->lev[l].nsets = nsets;
    off_lev[l][0] = bytes; bytes = align_up(bytes + size_t(nsets) * nc * nw * 8);
    off_lev[l][1] = bytes; bytes = align_up(bytes + size_t(nsets) * nc * nc * 8);
    off_lev[l][2] = bytes; bytes = align_up(bytes + size_t(nsets) * nc * nw * ab);
    off_lev[l][3] = bytes; bytes = align_up(bytes + size_t(nsets) * nc * nc * ab);
    off_lev[l][4] = bytes; bytes = align_up(bytes + size_t(3) * nw * 8);
    const int64_t shell_sets = icr::shell_tables(p) ? nsets : 0;
    off_lev[l][5] = bytes; bytes = align_up(bytes + size_t(shell_sets) * icr::kShellStride * 4);
    off_lev[l][6] = bytes; bytes = align_up(bytes + size_t(shell_sets) * 2 * 8);  // symmetry check (3-D)
    const int64_t dsets = p->hypergrad ? nsets : 0;
    off_lev[l][7] = bytes; bytes = align_up(bytes + size_t(dsets) * nc * nw * 8);
    off_lev[l][8] = bytes; bytes = align_up(bytes + size_t(dsets) * nc * nc * 8);
    off_lev[l][9] = bytes; bytes = align_up(bytes + size_t(dsets) * nc * nw * ab);
    off_lev[l][10] = bytes; bytes = align_up(bytes + size_t(dsets) * nc * nc * ab);
    off_lev[l][11] = bytes; bytes = align_up(bytes + (p->hypergrad && !p->charted ? size_t(3) * nw * 8 : 0));
    const int64_t dshell = p->hypergrad && icr::shell_tables(p) && d == 3 ? nsets : 0;
    off_lev[l][12] = bytes; bytes = align_up(bytes + size_t(dshell) * icr::kShellStride * 4);
    off_lev[l][13] = bytes; bytes = align_up(bytes + size_t(dshell) * 2 * 8);
  }
  const size_t off_status = bytes; bytes = align_up(bytes + sizeof(int32_t) * (kMaxLevels + 1));

  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipMalloc(&p->pool, bytes);
  if (e != hipSuccess) {
    delete p;
    if (e == hipErrorOutOfMemory) return fail(ICR_ERR_OUT_OF_MEMORY, "device allocation of the plan failed");
    return fail(ICR_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  p->pool_bytes = static_cast<int64_t>(bytes);
  char* base = static_cast<char*>(p->pool);
  p->l00_64 = reinterpret_cast<double*>(base + off_l64);
  p->l00_c = base + off_lc;
  p->u00_c = base + off_uc;
  if (p->hypergrad) p->dl00_64 = reinterpret_cast<double*>(base + off_dl00);
  for (int l = 0; l < p->depth; ++l) {
    p->lev[l].r64 = reinterpret_cast<double*>(base + off_lev[l][0]);
    p->lev[l].s64 = reinterpret_cast<double*>(base + off_lev[l][1]);
    p->lev[l].r_c = base + off_lev[l][2];
    p->lev[l].s_c = base + off_lev[l][3];
    p->lev[l].sector64 = reinterpret_cast<double*>(base + off_lev[l][4]);
    if (icr::shell_tables(p)) {
      p->lev[l].shell_tab = reinterpret_cast<float*>(base + off_lev[l][5]);
      p->lev[l].shell_chk = reinterpret_cast<double*>(base + off_lev[l][6]);
    }
    if (p->hypergrad) {
      p->lev[l].dr64 = reinterpret_cast<double*>(base + off_lev[l][7]);
      p->lev[l].ds64 = reinterpret_cast<double*>(base + off_lev[l][8]);
      p->lev[l].dr_c = base + off_lev[l][9];
      p->lev[l].ds_c = base + off_lev[l][10];
      if (!p->charted) p->lev[l].dsector64 = reinterpret_cast<double*>(base + off_lev[l][11]);
      if (icr::shell_tables(p) && d == 3) {
        p->lev[l].dshell_tab = reinterpret_cast<float*>(base + off_lev[l][12]);
        p->lev[l].dshell_chk = reinterpret_cast<double*>(base + off_lev[l][13]);
      }
    }
  }
  int32_t* status = reinterpret_cast<int32_t*>(base + off_status);
  int32_t* counts = status + 1;

  auto bail = [&](icr_status s, const std::string& msg) {
    (void)hipFree(p->pool);
    delete p;
    return fail(s, msg);
  };
#define BUILD_TRY(expr)                                                                   \
  do {                                                                                    \
    const hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return bail(ICR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

  BUILD_TRY(hipMemsetAsync(status, 0, sizeof(int32_t) * (kMaxLevels + 1), st));
  BUILD_TRY(icr::launch_build_k00(p, p->l00_64, st));
  BUILD_TRY(icr::launch_cholesky_level0(p, p->l00_64, counts + 0, status, st));
  BUILD_TRY(icr::launch_level0_convert(p, st));
  double* dl_scratch = nullptr;  // 2 n0^2 doubles for the level-0 derivative, freed after the build
  if (p->hypergrad) {
    BUILD_TRY(hipMalloc(&dl_scratch, sizeof(double) * 2 * size_t(p->n0) * p->n0));
    const hipError_t e = icr::launch_level0_length_derivative(p, dl_scratch, st);
    if (e != hipSuccess) {
      (void)hipFree(dl_scratch);
      return bail(ICR_ERR_HIP, std::string("level-0 length derivative: ") + hipGetErrorString(e));
    }
  }
  for (int l = 0; l < p->depth; ++l) {
    BUILD_TRY(icr::launch_build_level(p, l, counts + 1 + l, status, st));
    BUILD_TRY(icr::launch_level_convert(p, l, st));
    if (!p->charted) BUILD_TRY(icr::launch_sector(p, l, st));
    if (icr::shell_tables(p)) BUILD_TRY(icr::launch_shell_sector(p, l, st));
  }
  // everything the host needs back comes in one round: the status words and every
  // level's host copies, then a single synchronisation
  int32_t host_status[kMaxLevels + 1];
  BUILD_TRY(hipMemcpyAsync(host_status, status, sizeof(host_status), hipMemcpyDeviceToHost, st));
  std::vector<HostStage> stages(static_cast<size_t>(p->depth));
  for (int l = 0; l < p->depth; ++l) {
    const icr_status hs = stage_host_copies(p, l, &stages[l], st);
    if (hs != ICR_OK) {
      (void)hipStreamSynchronize(st);
      if (dl_scratch) (void)hipFree(dl_scratch);
      const std::string msg = icr_last_error();
      return bail(hs, msg);
    }
  }
  {
    const hipError_t e = hipStreamSynchronize(st);
    if (dl_scratch) (void)hipFree(dl_scratch);
    if (e != hipSuccess) return bail(ICR_ERR_HIP, std::string("build: ") + hipGetErrorString(e));
  }
#undef BUILD_TRY
  for (int l = 0; l <= p->depth; ++l) p->clamped[l] = host_status[1 + l];
  for (int l = 0; l < p->depth; ++l) apply_host_copies(p, l, stages[l]);
  if (host_status[0] & 2)
    return bail(ICR_ERR_NOT_PD, "K_00 is not positive definite (a pivot needed clamping; clamping disabled)");
  if (p->hypergrad) {
    bool clamped = (host_status[0] & 4) != 0;
    for (int l = 0; l <= p->depth; ++l) clamped = clamped || p->clamped[l] > 0;
    if (clamped)
      return bail(ICR_ERR_NOT_PD,
                  "hyperparameter gradients need factors without clamped pivots (their derivative is undefined)");
  }
  if (host_status[0] & 1)
    return bail(ICR_ERR_NOT_PD,
                "a window covariance K_cc is not positive definite, or a pivot of D needed "
                "clamping with clamping disabled");
  *out_plan = p;
  return ICR_OK;
}

icr_status icr_plan_get_info(const icr_plan* p, icr_plan_info* info) {
  icr::clear_error();
  if (!p || !info) return fail(ICR_ERR_INVALID_ARG, "plan or info is NULL");
  std::memset(info, 0, sizeof(*info));
  const int d = p->ndim;
  info->ndim = d;
  info->depth = p->depth;
  info->precision = p->precision;
  info->chart = p->cfg.chart;
  info->elem_bytes = p->elem_bytes;
  for (int l = 0; l <= p->depth; ++l) {
    info->clamped_pivots[l] = p->clamped[l];
    for (int a = 0; a < 3; ++a) info->level_shapes[l][a] = a < d ? p->shapes[l][3 - d + a] : 1;
    info->level_offsets[l] = p->offsets[l];
  }
  info->level_offsets[p->depth + 1] = p->n_xi;
  info->n_xi = p->n_xi;
  info->n_out = p->n_out;
  info->workspace_elems = p->n_xi - p->n_out;
  info->metric_workspace_elems = p->n_xi;
  info->device_bytes = p->pool_bytes;
  for (int l = 0; l < p->depth; ++l) info->level_sets[l] = p->lev[l].nsets;
  info->hypergrad_workspace_elems = p->hypergrad ? icr::hypergrad_partials(p) : 0;
  return ICR_OK;
}

icr_status icr_plan_copy_level0(const icr_plan* p, double* l00) {
  icr::clear_error();
  if (!p || !l00) return fail(ICR_ERR_INVALID_ARG, "plan or l00 is NULL");
  ICR_HIP_TRY(hipMemcpy(l00, p->l00_64, size_t(p->n0) * p->n0 * 8, hipMemcpyDeviceToHost));
  return ICR_OK;
}

icr_status icr_plan_copy_refinement(const icr_plan* p, int32_t level, double* r, double* sqrtd) {
  icr::clear_error();
  if (!p) return fail(ICR_ERR_INVALID_ARG, "plan is NULL");
  if (level < 0 || level >= p->depth) return fail(ICR_ERR_INVALID_ARG, "level out of range");
  const int nc = 1 << p->ndim, nw = icr::pow3(p->ndim);
  const icr::LevelMats& m = p->lev[level];
  if (r) ICR_HIP_TRY(hipMemcpy(r, m.r64, size_t(m.nsets) * nc * nw * 8, hipMemcpyDeviceToHost));
  if (sqrtd) ICR_HIP_TRY(hipMemcpy(sqrtd, m.s64, size_t(m.nsets) * nc * nc * 8, hipMemcpyDeviceToHost));
  return ICR_OK;
}

icr_status icr_plan_set_level0(icr_plan* p, const double* l00, void* hip_stream) {
  icr::clear_error();
  if (!p || !l00) return fail(ICR_ERR_INVALID_ARG, "plan or l00 is NULL");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  ICR_HIP_TRY(hipMemcpyAsync(p->l00_64, l00, size_t(p->n0) * p->n0 * 8, hipMemcpyHostToDevice, st));
  ICR_HIP_TRY(icr::launch_level0_convert(p, st));
  ICR_HIP_TRY(hipStreamSynchronize(st));
  return ICR_OK;
}

icr_status icr_plan_set_refinement(icr_plan* p, int32_t level, const double* r, const double* sqrtd,
                                   void* hip_stream) {
  icr::clear_error();
  if (!p || !r || !sqrtd) return fail(ICR_ERR_INVALID_ARG, "plan, r or sqrtd is NULL");
  if (level < 0 || level >= p->depth) return fail(ICR_ERR_INVALID_ARG, "level out of range");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nc = 1 << p->ndim, nw = icr::pow3(p->ndim);
  const icr::LevelMats& m = p->lev[level];
  ICR_HIP_TRY(hipMemcpyAsync(m.r64, r, size_t(m.nsets) * nc * nw * 8, hipMemcpyHostToDevice, st));
  ICR_HIP_TRY(hipMemcpyAsync(m.s64, sqrtd, size_t(m.nsets) * nc * nc * 8, hipMemcpyHostToDevice, st));
  ICR_HIP_TRY(icr::launch_level_convert(p, level, st));
  if (!p->charted) ICR_HIP_TRY(icr::launch_sector(p, level, st));
  if (icr::shell_tables(p)) ICR_HIP_TRY(icr::launch_shell_sector(p, level, st));
  return refresh_host_copies(p, level, st);
}

icr_status icr_forward(const icr_plan* p, int64_t batch, const void* xi, void* s, void* workspace,
                       void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK || batch == 0) return cs;
  const int el = p->elem_bytes;
  if (!xi || !s || (p->depth > 0 && !workspace)) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (!aligned(xi, el) || !aligned(s, el) || (workspace && !aligned(workspace, el)))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  const size_t nx = size_t(batch) * p->n_xi * el, ns = size_t(batch) * p->n_out * el;
  const size_t nw = p->depth > 0 ? size_t(batch) * (p->n_xi - p->n_out) * el : 0;
  if (icr::overlaps(xi, nx, s, ns) || icr::overlaps(xi, nx, workspace, nw) || icr::overlaps(s, ns, workspace, nw))
    return fail(ICR_ERR_INVALID_ARG, "xi, s and workspace overlap");
  return run_forward(p, batch, xi, s, p->n_out, workspace, p->n_xi - p->n_out, nullptr, 0,
                     static_cast<hipStream_t>(hip_stream));
}

icr_status icr_adjoint(const icr_plan* p, int64_t batch, const void* s_bar, void* xi_bar,
                       void* workspace, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK || batch == 0) return cs;
  const int el = p->elem_bytes;
  if (!s_bar || !xi_bar || (p->depth > 0 && !workspace)) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (!aligned(s_bar, el) || !aligned(xi_bar, el) || (workspace && !aligned(workspace, el)))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  const size_t nx = size_t(batch) * p->n_xi * el, ns = size_t(batch) * p->n_out * el;
  const size_t nw = p->depth > 0 ? size_t(batch) * (p->n_xi - p->n_out) * el : 0;
  if (icr::overlaps(xi_bar, nx, s_bar, ns) || icr::overlaps(xi_bar, nx, workspace, nw) ||
      icr::overlaps(s_bar, ns, workspace, nw))
    return fail(ICR_ERR_INVALID_ARG, "s_bar, xi_bar and workspace overlap");
  return run_adjoint(p, batch, s_bar, p->n_out, xi_bar, workspace, p->n_xi - p->n_out, nullptr,
                     static_cast<hipStream_t>(hip_stream));
}

icr_status icr_metric_apply(const icr_plan* p, int64_t batch, const void* w, int64_t w_batch_stride,
                            const void* v, void* out, void* workspace, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK || batch == 0) return cs;
  const int el = p->elem_bytes;
  const int ab = acc_bytes_of(p->precision);
  if (!w || !v || !out || !workspace) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (w_batch_stride != 0 && w_batch_stride < p->n_out)
    return fail(ICR_ERR_INVALID_ARG, "w_batch_stride must be 0 or >= n_out");
  if (!aligned(v, el) || !aligned(out, el) || !aligned(workspace, el) || !aligned(w, ab))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  const size_t nx = size_t(batch) * p->n_xi * el;
  if (icr::overlaps(v, nx, out, nx) || icr::overlaps(v, nx, workspace, nx) || icr::overlaps(out, nx, workspace, nx))
    return fail(ICR_ERR_INVALID_ARG, "v, out and workspace overlap");
  return run_metric(p, batch, w, w_batch_stride, v, out, workspace, static_cast<hipStream_t>(hip_stream));
}

icr_status icr_metric_apply_static(const icr_plan* p, int64_t batch, const void* w, int64_t w_batch_stride,
                                   const void* v, void* out, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK || batch == 0) return cs;
  const int el = p->elem_bytes;
  const int ab = acc_bytes_of(p->precision);
  const size_t need = size_t(batch) * size_t(p->n_xi) * el;
  if (need > kStaticScratchBytes)
    return fail(ICR_ERR_INVALID_ARG, "the metric needs " + std::to_string(need) + " bytes of workspace; the static "
                "scratch holds " + std::to_string(kStaticScratchBytes) + " (use icr_metric_apply)");
  if (!w || !v || !out) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (w_batch_stride != 0 && w_batch_stride < p->n_out)
    return fail(ICR_ERR_INVALID_ARG, "w_batch_stride must be 0 or >= n_out");
  if (!aligned(v, el) || !aligned(out, el) || !aligned(w, ab))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  if (icr::overlaps(v, need, out, need)) return fail(ICR_ERR_INVALID_ARG, "v and out overlap");
  void* ws = nullptr;
  cs = scratch_ptr(&ws);
  if (cs != ICR_OK) return cs;
  // the same sweep as icr_metric_apply, its workspace in the scratch array: every element
  // it reads there is written earlier in the same call, so nothing needs clearing
  return run_metric(p, batch, w, w_batch_stride, v, out, ws, static_cast<hipStream_t>(hip_stream));
}

icr_status icr_hyper_grad(const icr_plan* p, int64_t batch, const void* xi, const void* s,
                          const void* s_levels, const void* s_bar, const void* sbar_levels,
                          double* grad, double* workspace, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK || batch == 0) return cs;
  if (!p->hypergrad) return fail(ICR_ERR_UNSUPPORTED, "the plan was built without ICR_FLAG_HYPERGRAD");
  if (batch > 65535) return fail(ICR_ERR_INVALID_ARG, "at most 65535 samples per call");
  const int el = p->elem_bytes;
  const bool levels = p->depth > 0;
  if (!xi || !s || !s_bar || !grad || !workspace || (levels && (!s_levels || !sbar_levels)))
    return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (!aligned(xi, el) || !aligned(s, el) || !aligned(s_bar, el) || (levels && !aligned(s_levels, el)) ||
      (levels && !aligned(sbar_levels, el)) || !aligned(grad, 8) || !aligned(workspace, 8))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  ICR_HIP_TRY(icr::launch_hyper_grad(p, batch, xi, s, s_levels, s_bar, sbar_levels, grad, workspace,
                                     static_cast<hipStream_t>(hip_stream)));
  return ICR_OK;
}

icr_status icr_cg_workspace_bytes(const icr_plan* p, int64_t batch, int64_t* bytes) {
  icr::clear_error();
  if (!p || !bytes || batch < 0) return fail(ICR_ERR_INVALID_ARG, "plan or bytes is NULL, or batch < 0");
  *bytes = icr::cg_workspace_bytes(p, batch);
  return ICR_OK;
}

icr_status icr_cg_metric(const icr_plan* p, int64_t batch, const void* w, int64_t w_batch_stride,
                         const void* b, void* x, int32_t iterations, double* residual_norms,
                         void* workspace, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK) return cs;
  cs = check_cg_call(p, batch, w, w_batch_stride, b, x, iterations, residual_norms, workspace);
  if (cs != ICR_OK || batch == 0) return cs;
  ICR_HIP_TRY(icr::launch_cg(p, batch, w, w_batch_stride, b, x, iterations, 0.0, nullptr, residual_norms,
                             workspace, static_cast<hipStream_t>(hip_stream), metric_for_cg));
  return ICR_OK;
}

icr_status icr_cg_metric_sl(const icr_plan* p, int64_t batch, const void* w, int64_t w_batch_stride,
                            const void* b, void* x, double absdelta, int32_t maxiter, int32_t* iterations_done,
                            double* residual_norms, void* workspace, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK) return cs;
  if (!(absdelta > 0.0) || !std::isfinite(absdelta)) return fail(ICR_ERR_INVALID_ARG, "absdelta must be finite and > 0");
  cs = check_cg_call(p, batch, w, w_batch_stride, b, x, maxiter, residual_norms, workspace);
  if (cs != ICR_OK || batch == 0) return cs;
  if (iterations_done && !aligned(iterations_done, 4))
    return fail(ICR_ERR_INVALID_ARG, "iterations_done not aligned");
  ICR_HIP_TRY(icr::launch_cg(p, batch, w, w_batch_stride, b, x, maxiter, absdelta, iterations_done,
                             residual_norms, workspace, static_cast<hipStream_t>(hip_stream), metric_for_cg));
  return ICR_OK;
}

icr_status icr_weighted_adjoint(const icr_plan* p, int64_t batch, const void* w, int64_t w_batch_stride,
                                int32_t half, const void* y, const void* add, void* out, void* workspace,
                                void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK || batch == 0) return cs;
  if (batch > 65535) return fail(ICR_ERR_INVALID_ARG, "at most 65535 samples per call");
  const int el = p->elem_bytes;
  const int ab = acc_bytes_of(p->precision);
  if (!w || !y || !out || !workspace) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (w_batch_stride != 0 && w_batch_stride < p->n_out)
    return fail(ICR_ERR_INVALID_ARG, "w_batch_stride must be 0 or >= n_out");
  if (!aligned(y, el) || !aligned(out, el) || !aligned(workspace, el) || !aligned(w, ab) || (add && !aligned(add, el)))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  const size_t nx = size_t(batch) * p->n_xi * el;
  if (icr::overlaps(out, nx, workspace, nx) || (add && icr::overlaps(add, nx, workspace, nx)) ||
      icr::overlaps(y, size_t(batch) * p->n_out * el, workspace, nx))
    return fail(ICR_ERR_INVALID_ARG, "workspace overlaps a buffer");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the weighted cotangent at the front of each sample's workspace row, the sweep's
  // levels behind it
  ICR_HIP_TRY(icr::launch_weight(p, batch, w, w_batch_stride, y, p->n_out, workspace, p->n_xi, p->n_out, half != 0,
                                 st));
  return run_adjoint(p, batch, workspace, p->n_xi, out, at(workspace, p->n_out, el), p->n_xi, add, st);
}

icr_status icr_mgvi_workspace_bytes(const icr_plan* p, int64_t batch, int64_t* bytes) {
  icr::clear_error();
  if (!p || !bytes || batch < 0) return fail(ICR_ERR_INVALID_ARG, "plan or bytes is NULL, or batch < 0");
  const int64_t vec = (batch * p->n_xi * p->elem_bytes + 255) & ~int64_t(255);
  *bytes = 2 * vec + icr::cg_workspace_bytes(p, batch);
  return ICR_OK;
}

icr_status icr_mgvi_newton_step(const icr_plan* p, int64_t batch, const void* w, int64_t w_batch_stride,
                                const void* b, void* mean, int32_t iterations, double* residual_norms,
                                void* workspace, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK) return cs;
  if (p->precision == ICR_BF16_F32ACC) return fail(ICR_ERR_UNSUPPORTED, "the Newton step needs an FP64 or FP32 plan");
  if (iterations < 0) return fail(ICR_ERR_INVALID_ARG, "iterations must be >= 0");
  if (batch > 65535) return fail(ICR_ERR_INVALID_ARG, "at most 65535 samples per call");
  if (batch == 0) return ICR_OK;
  const int el = p->elem_bytes;
  if (!w || !b || !mean || !workspace) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (w_batch_stride != 0 && w_batch_stride < p->n_out)
    return fail(ICR_ERR_INVALID_ARG, "w_batch_stride must be 0 or >= n_out");
  if (!aligned(b, el) || !aligned(mean, el) || !aligned(w, el) || !aligned(workspace, 256) ||
      (residual_norms && !aligned(residual_norms, 8)))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned (workspace needs 256 bytes)");
  int64_t wsb = 0;
  (void)icr_mgvi_workspace_bytes(p, batch, &wsb);
  const size_t nx = size_t(batch) * p->n_xi * el;
  if (icr::overlaps(b, nx, mean, nx) || icr::overlaps(b, nx, workspace, size_t(wsb)) ||
      icr::overlaps(mean, nx, workspace, size_t(wsb)))
    return fail(ICR_ERR_INVALID_ARG, "b, mean and workspace overlap");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t vec = (int64_t(nx) + 255) & ~int64_t(255);
  char* base = static_cast<char*>(workspace);
  void* g = base;
  void* delta = base + vec;
  void* cg_ws = base + 2 * vec;
  // g = M mean - b (the KL gradient over antithetic pairs), delta = M^-1 g, mean -= delta;
  // CG's own metric workspace serves the first product
  ICR_HIP_TRY(metric_for_cg(p, batch, w, w_batch_stride, mean, g, cg_ws, nullptr, st, nullptr, 0, nullptr));
  ICR_HIP_TRY(icr::launch_sub(p, batch, g, b, p->n_xi, st));
  ICR_HIP_TRY(icr::launch_cg(p, batch, w, w_batch_stride, g, delta, iterations, 0.0, nullptr, residual_norms,
                             cg_ws, st, metric_for_cg));
  ICR_HIP_TRY(icr::launch_sub(p, batch, mean, delta, p->n_xi, st));
  return ICR_OK;
}

icr_status icr_forward_level(const icr_plan* p, int32_t level, int64_t batch, const void* s_coarse,
                             int64_t coarse_stride, const void* xi_fine, int64_t xi_stride,
                             void* s_fine, int64_t fine_stride, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK) return cs;
  if (level < -1 || level >= p->depth) return fail(ICR_ERR_INVALID_ARG, "level out of range");
  if (batch == 0) return ICR_OK;
  const int el = p->elem_bytes;
  const int64_t nf = p->offsets[level + 2] - p->offsets[level + 1];
  const int64_t nc = level >= 0 ? p->offsets[level + 1] - p->offsets[level] : 0;
  if (!xi_fine || !s_fine || (level >= 0 && !s_coarse)) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (xi_stride < nf || fine_stride < nf || (level >= 0 && coarse_stride < nc))
    return fail(ICR_ERR_INVALID_ARG, "stride smaller than the level size");
  if (!aligned(xi_fine, el) || !aligned(s_fine, el) || (s_coarse && !aligned(s_coarse, el)))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  if (icr::overlaps_batched(s_fine, fine_stride * el, nf * el, xi_fine, xi_stride * el, nf * el, batch) ||
      (level >= 0 &&
       icr::overlaps_batched(s_fine, fine_stride * el, nf * el, s_coarse, coarse_stride * el, nc * el, batch)))
    return fail(ICR_ERR_INVALID_ARG, "s_fine overlaps an input");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (level < 0) {
    icr::Level0Args a{xi_fine, xi_stride, s_fine, fine_stride, nullptr, 0, nullptr, 0, batch};
    ICR_HIP_TRY(icr::launch_level0_fwd(p, a, st));
    return ICR_OK;
  }
  icr::RefineFwdArgs a{s_coarse, coarse_stride, xi_fine, xi_stride, s_fine, fine_stride, nullptr, 0, batch};
  ICR_HIP_TRY(icr::launch_refine_fwd(p, level, a, st));
  return ICR_OK;
}

icr_status icr_adjoint_level(const icr_plan* p, int32_t level, int64_t batch, const void* y_fine,
                             int64_t y_stride, void* xi_bar_fine, int64_t xi_bar_stride,
                             void* s_bar_coarse, int64_t coarse_stride, void* hip_stream) {
  icr::clear_error();
  icr_status cs = check_call(p, batch);
  if (cs != ICR_OK) return cs;
  if (level < -1 || level >= p->depth) return fail(ICR_ERR_INVALID_ARG, "level out of range");
  if (batch == 0) return ICR_OK;
  const int el = p->elem_bytes;
  const int64_t nf = p->offsets[level + 2] - p->offsets[level + 1];
  const int64_t nc = level >= 0 ? p->offsets[level + 1] - p->offsets[level] : 0;
  if (!y_fine || !xi_bar_fine || (level >= 0 && !s_bar_coarse)) return fail(ICR_ERR_INVALID_ARG, "NULL buffer");
  if (y_stride < nf || xi_bar_stride < nf || (level >= 0 && coarse_stride < nc))
    return fail(ICR_ERR_INVALID_ARG, "stride smaller than the level size");
  if (!aligned(y_fine, el) || !aligned(xi_bar_fine, el) || (s_bar_coarse && !aligned(s_bar_coarse, el)))
    return fail(ICR_ERR_INVALID_ARG, "buffer not aligned to its element size");
  const int64_t sy = y_stride * el, sx = xi_bar_stride * el, sc = coarse_stride * el;
  if (icr::overlaps_batched(xi_bar_fine, sx, nf * el, y_fine, sy, nf * el, batch) ||
      (level >= 0 && (icr::overlaps_batched(s_bar_coarse, sc, nc * el, y_fine, sy, nf * el, batch) ||
                      icr::overlaps_batched(s_bar_coarse, sc, nc * el, xi_bar_fine, sx, nf * el, batch))))
    return fail(ICR_ERR_INVALID_ARG, "buffers overlap");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (level < 0) {
    icr::Level0Args a{y_fine, y_stride, xi_bar_fine, xi_bar_stride, nullptr, 0, nullptr, 0, batch};
    ICR_HIP_TRY(icr::launch_level0_adj(p, a, st));
    return ICR_OK;
  }
  icr::RefineAdjArgs a{y_fine, y_stride, xi_bar_fine, xi_bar_stride, s_bar_coarse, coarse_stride,
                       nullptr, 0, batch};
  ICR_HIP_TRY(icr::launch_refine_adj(p, level, a, st));
  return ICR_OK;
}

icr_status icr_plan_destroy(icr_plan* p) {
  icr::clear_error();
  if (!p) return ICR_OK;
  const hipError_t e = p->pool ? hipFree(p->pool) : hipSuccess;
  delete p;
  if (e != hipSuccess) return fail(ICR_ERR_HIP, std::string("hipFree: ") + hipGetErrorString(e));
  return ICR_OK;
}

}  // extern "C"
