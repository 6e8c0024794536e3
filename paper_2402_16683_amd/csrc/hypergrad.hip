// Gradients of E = <s_bar, L xi> with respect to the kernel hyperparameters
// (scale sigma, length scale), from one forward and one adjoint sweep.
//
// Differentiating the level recursion s_0 = L00 xi_0, s_{l+1} = R_l s_l[window] +
// sqrtD_l xi_{l+1} and contracting with the adjoint's level cotangents sbar gives
//   dE/dlength = <sbar_0, dL00 xi_0> + sum_l sum_c <sbar_{l+1}[block c], dR_l s_l[c + W] + dsqrtD_l xi_{l+1}[block c]>
// with the FP64 length derivatives of the build, and dE/dsigma = <s_bar, s> / sigma
// (every covariance is proportional to sigma^2, so R does not depend on sigma while
// sqrtD and L00 are proportional to it). <s_bar, s> is not read from the final level:
// by the adjoint identity it equals <sbar_0, s_0> + sum_l <sbar_{l+1}, sqrtD_l xi_{l+1}>,
// which the level contractions add up from data they read anyway.
//
// Each term is reduced per sample in FP64: per thread in a fixed order, per workgroup by
// a fixed tree, and over the workgroups' partial sums (kHgSlots per term and sample) by
// one workgroup per sample in a fixed order, so results are bitwise reproducible.
// Per-term products use the plan's arithmetic type. 3-D levels with the reflection-
// sector form run the fast forward kernel with the derivative matrices and a dot
// epilogue; other levels run the generic contraction below (kHgBlocks workgroups).
#include "icr_internal.h"

namespace icr {
namespace {

constexpr int kHgBlocks = 512;   // workgroups per sample of the generic terms
constexpr int kHgSlots = 2048;   // partial sums per sample, term and gradient component
constexpr int kHgThreads = 256;

// Partial sums per sample: for each term (level 0, then each refinement) kHgSlots for
// the length gradient followed by kHgSlots for the scale gradient.
struct HgCounts {
  int32_t n[kMaxLevels + 1];     // partial sums written per term
};

struct HgGeom {
  int nc[3];        // coarse shape (first D axes)
  int nf[3];        // fine shape
  int mi[3];        // interior coarse pixels per axis
  int64_t ninterior;
  int64_t msets;    // charted: matrix sets (stride between a set's entries)
  int shell;
};

template <int D>
__device__ __forceinline__ int64_t lin(const int* idx, const int* shape) {
  int64_t v = idx[0];
  for (int a = 1; a < D; ++a) v = v * shape[a] + idx[a];
  return v;
}

// Fixed-order sums over the workgroup of two doubles per thread, written by thread 0 to
// out[0] and out[kHgSlots].
__device__ void block_sum_store(double v, double w, double* out) {
  __shared__ double red[2][kHgThreads];
  red[0][threadIdx.x] = v;
  red[1][threadIdx.x] = w;
  __syncthreads();
  for (int s = kHgThreads / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[kHgSlots] = red[1][0];
  }
}

// One refinement level: thread t takes interior coarse pixels t, t + stride, ... and
// accumulates <sbar block, dR s[window] + dsqrtD xi block> and <sbar block, sqrtD xi
// block> in FP64.
template <int D, typename TS, bool kCharted>
__global__ void __launch_bounds__(kHgThreads) hg_level_kernel(HgGeom g, const TS* __restrict__ s_in, int64_t s_bs,
                                                             const TS* __restrict__ xi, int64_t xi_bs,
                                                             const TS* __restrict__ sb, int64_t sb_bs,
                                                             const typename Acc<TS>::type* dR,
                                                             const typename Acc<TS>::type* dS,
                                                             const typename Acc<TS>::type* S,
                                                             double* __restrict__ part, int64_t part_bs) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  const int64_t b = blockIdx.y;
  __shared__ TA lds_r[kCharted ? 1 : NC * NW], lds_s[kCharted ? 1 : NC * NC], lds_v[kCharted ? 1 : NC * NC];
  if (!kCharted) {  // a stationary level's matrices, staged once per workgroup
    for (int e = threadIdx.x; e < NC * NW; e += blockDim.x) lds_r[e] = dR[e];
    for (int e = threadIdx.x; e < NC * NC; e += blockDim.x) {
      lds_s[e] = dS[e];
      lds_v[e] = S[e];
    }
    __syncthreads();
    dR = lds_r;
    dS = lds_s;
    S = lds_v;
  }
  s_in += b * s_bs;
  xi += b * xi_bs;
  sb += b * sb_bs;
  const int64_t stride = kCharted ? g.msets : 1;
  double acc = 0.0, acc_sig = 0.0;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < g.ninterior;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int c[D];
    int64_t rem = t;
    for (int ax = D - 1; ax >= 0; --ax) { c[ax] = static_cast<int>(rem % g.mi[ax]) + 1; rem /= g.mi[ax]; }
    const int64_t set = kCharted ? (g.shell ? c[0] - 1 : t) : 0;
    TA win[NW];
    for (int iw = 0; iw < NW; ++iw) {
      int q[D];
      int r = iw;
      for (int ax = D - 1; ax >= 0; --ax) { q[ax] = c[ax] + (r % 3) - 1; r /= 3; }
      win[iw] = load_acc(s_in + lin<D>(q, g.nc));
    }
    TA fresh[NC], cot[NC];
    for (int ib = 0; ib < NC; ++ib) {
      int q[D];
      for (int ax = 0; ax < D; ++ax) q[ax] = 2 * (c[ax] - 1) + ((ib >> (D - 1 - ax)) & 1);
      const int64_t f = lin<D>(q, g.nf);
      fresh[ib] = load_acc(xi + f);
      cot[ib] = load_acc(sb + f);
    }
    for (int ib = 0; ib < NC; ++ib) {
      TA o = 0, v = 0;
      for (int iw = 0; iw < NW; ++iw) o += dR[(ib * NW + iw) * stride + set] * win[iw];
      for (int jb = 0; jb <= ib; ++jb) {
        o += dS[(ib * NC + jb) * stride + set] * fresh[jb];
        v += S[(ib * NC + jb) * stride + set] * fresh[jb];
      }
      acc += static_cast<double>(cot[ib]) * static_cast<double>(o);
      acc_sig += static_cast<double>(cot[ib]) * static_cast<double>(v);
    }
  }
  block_sum_store(acc, acc_sig, part + b * part_bs + blockIdx.x);
}

// Level 0: sum_i sbar_0[i] sum_{j <= i} dL00[i][j] xi_0[j] with the FP64 derivative
// (one wavefront per row: lanes stride the row, butterfly sum in a fixed order), and
// sum_i sbar_0[i] s_0[i].
template <typename TS>
__global__ void __launch_bounds__(kHgThreads) hg_level0_kernel(const double* __restrict__ dl, int64_t n,
                                                              const TS* __restrict__ xi, int64_t xi_bs,
                                                              const TS* __restrict__ sb, int64_t sb_bs,
                                                              const TS* __restrict__ s0, int64_t s0_bs,
                                                              double* __restrict__ part, int64_t part_bs) {
  const int64_t b = blockIdx.y;
  xi += b * xi_bs;
  sb += b * sb_bs;
  s0 += b * s0_bs;
  double acc_sig = 0.0;
  const int lane = threadIdx.x & 63;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / 64);
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x / 64) + threadIdx.x / 64; i < n; i += waves) {
    double r = 0.0;
    for (int64_t j = lane; j <= i; j += 64) r += dl[i * n + j] * static_cast<double>(load_acc(xi + j));
    for (int m = 32; m > 0; m >>= 1) r += __shfl_xor(r, m, 64);
    if (lane == 0) {
      const double c = static_cast<double>(load_acc(sb + i));
      acc += c * r;
      acc_sig += c * static_cast<double>(load_acc(s0 + i));
    }
  }
  block_sum_store(acc, acc_sig, part + b * part_bs + blockIdx.x);
}

// Per sample: grad = (sum of the scale partials / sigma, sum of the length partials).
constexpr int kHgFinalThreads = 1024;
__global__ void __launch_bounds__(kHgFinalThreads) hg_final_kernel(const double* __restrict__ part,
                                                                  int64_t part_bs, int terms, HgCounts cnt,
                                                                  double inv_sigma, double* __restrict__ grad) {
  const int64_t b = blockIdx.x;
  const double* p = part + b * part_bs;
  __shared__ double red[2][kHgFinalThreads];
  double v[2] = {0.0, 0.0};
  for (int term = 0; term < terms; ++term)
    for (int64_t k = threadIdx.x; k < cnt.n[term]; k += blockDim.x) {
      v[0] += p[int64_t(term) * 2 * kHgSlots + k];             // length
      v[1] += p[int64_t(term) * 2 * kHgSlots + kHgSlots + k];  // scale
    }
  red[0][threadIdx.x] = v[0];
  red[1][threadIdx.x] = v[1];
  __syncthreads();
  for (int s = kHgFinalThreads / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    grad[2 * b] = red[1][0] * inv_sigma;
    grad[2 * b + 1] = red[0][0];
  }
}

template <int D, typename TS>
hipError_t level_term(const icr_plan* p, int l, int64_t batch, const TS* s_in, int64_t s_bs, const TS* xi,
                      int64_t xi_bs, const TS* sb, int64_t sb_bs, double* part, int64_t part_bs,
                      hipStream_t st, int32_t* written) {
  using TA = typename Acc<TS>::type;
  if (D == 3) {
    RefineFwdArgs a{s_in, s_bs, xi, xi_bs, nullptr, 0, nullptr, 0, batch};
    a.dot = sb;
    a.dot_bs = sb_bs;
    a.partial = part;
    a.partial_sig = part + kHgSlots;
    a.partial_bs = part_bs;
    hipError_t e = hipSuccess;
    int64_t wgs = 0;
    if (try_refine3_dot_sector(p, l, a, kHgSlots, st, &e, &wgs)) {
      *written = static_cast<int32_t>(wgs);
      return e;
    }
  }
  *written = kHgBlocks;
  HgGeom g;
  const int d = p->ndim;
  g.ninterior = 1;
  for (int a = 0; a < 3; ++a) {
    g.nc[a] = a < d ? p->shapes[l][3 - d + a] : 1;
    g.nf[a] = a < d ? p->shapes[l + 1][3 - d + a] : 1;
    g.mi[a] = a < d ? g.nc[a] - 2 : 1;
    if (a < d) g.ninterior *= g.mi[a];
  }
  g.msets = p->lev[l].nsets;
  g.shell = p->shell;
  const dim3 grid(kHgBlocks, static_cast<unsigned>(batch));
  const TA* dr = static_cast<const TA*>(p->lev[l].dr_c);
  const TA* ds = static_cast<const TA*>(p->lev[l].ds_c);
  const TA* sv = static_cast<const TA*>(p->lev[l].s_c);
  if (p->charted)
    hg_level_kernel<D, TS, true><<<grid, kHgThreads, 0, st>>>(g, s_in, s_bs, xi, xi_bs, sb, sb_bs, dr, ds, sv, part,
                                                             part_bs);
  else
    hg_level_kernel<D, TS, false><<<grid, kHgThreads, 0, st>>>(g, s_in, s_bs, xi, xi_bs, sb, sb_bs, dr, ds, sv, part,
                                                              part_bs);
  return hipGetLastError();
}

template <typename TS>
hipError_t hyper_grad_t(const icr_plan* p, int64_t batch, const TS* xi, const TS* s, const TS* s_levels,
                        const TS* s_bar, const TS* sbar_levels, double* grad, double* part, hipStream_t st) {
  const int L = p->depth;
  const int64_t pbs = hypergrad_partials(p);
  const int64_t ws_bs = p->n_xi - p->n_out;
  const dim3 grid(kHgBlocks, static_cast<unsigned>(batch));
  HgCounts cnt;
  cnt.n[0] = kHgBlocks;
  const TS* sb0 = L > 0 ? sbar_levels : s_bar;
  const TS* s0 = L > 0 ? s_levels : s;
  const int64_t lv0_bs = L > 0 ? ws_bs : p->n_out;
  hg_level0_kernel<TS><<<grid, kHgThreads, 0, st>>>(p->dl00_64, p->n0, xi, p->n_xi, sb0, lv0_bs, s0, lv0_bs, part,
                                                    pbs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int l = 0; l < L; ++l) {
    const TS* s_in = s_levels + p->offsets[l];
    const TS* xf = xi + p->offsets[l + 1];
    const TS* sb = l + 1 < L ? sbar_levels + p->offsets[l + 1] : s_bar;
    const int64_t sb_bs = l + 1 < L ? ws_bs : p->n_out;
    double* pl = part + int64_t(1 + l) * 2 * kHgSlots;
    int32_t* w = &cnt.n[1 + l];
    switch (p->ndim) {
      case 1: e = level_term<1, TS>(p, l, batch, s_in, ws_bs, xf, p->n_xi, sb, sb_bs, pl, pbs, st, w); break;
      case 2: e = level_term<2, TS>(p, l, batch, s_in, ws_bs, xf, p->n_xi, sb, sb_bs, pl, pbs, st, w); break;
      default: e = level_term<3, TS>(p, l, batch, s_in, ws_bs, xf, p->n_xi, sb, sb_bs, pl, pbs, st, w); break;
    }
    if (e != hipSuccess) return e;
  }
  hg_final_kernel<<<static_cast<unsigned>(batch), kHgFinalThreads, 0, st>>>(part, pbs, L + 1, cnt,
                                                                            1.0 / p->cfg.scale, grad);
  return hipGetLastError();
}

}  // namespace

int64_t hypergrad_partials(const icr_plan* p) { return int64_t(p->depth + 1) * 2 * kHgSlots; }

hipError_t launch_hyper_grad(const icr_plan* p, int64_t batch, const void* xi, const void* s,
                             const void* s_levels, const void* s_bar, const void* sbar_levels,
                             double* grad, double* partials, hipStream_t st) {
  switch (p->precision) {
    case ICR_F64:
      return hyper_grad_t<double>(p, batch, static_cast<const double*>(xi), static_cast<const double*>(s),
                                  static_cast<const double*>(s_levels), static_cast<const double*>(s_bar),
                                  static_cast<const double*>(sbar_levels), grad, partials, st);
    case ICR_F32:
      return hyper_grad_t<float>(p, batch, static_cast<const float*>(xi), static_cast<const float*>(s),
                                 static_cast<const float*>(s_levels), static_cast<const float*>(s_bar),
                                 static_cast<const float*>(sbar_levels), grad, partials, st);
    default:
      return hyper_grad_t<bf16_t>(p, batch, static_cast<const bf16_t*>(xi), static_cast<const bf16_t*>(s),
                                  static_cast<const bf16_t*>(s_levels), static_cast<const bf16_t*>(s_bar),
                                  static_cast<const bf16_t*>(sbar_levels), grad, partials, st);
  }
}

}  // namespace icr
