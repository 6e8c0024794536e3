// Gradients of E = <s_bar, L xi> with respect to the kernel hyperparameters
// (scale sigma, length scale), from one forward and one adjoint sweep.
//
// Differentiating the level recursion s_0 = L00 xi_0, s_{l+1} = R_l s_l[window] +
// sqrtD_l xi_{l+1} and contracting with the adjoint's level cotangents sbar gives
//   dE/dlength = <sbar_0, dL00 xi_0> + sum_l sum_c <sbar_{l+1}[block c], dR_l s_l[c + W] + dsqrtD_l xi_{l+1}[block c]>
// with the FP64 length derivatives of the build, and dE/dsigma = <s_bar, s> / sigma
// (every covariance is proportional to sigma^2, so R does not depend on sigma while
// sqrtD and L00 are proportional to it).
//
// Each term is reduced per sample over a fixed grid of workgroups (kHgBlocks) in FP64:
// per thread in a fixed grid-stride order, per workgroup by a fixed tree, and over the
// workgroups' partial sums by one workgroup per sample in a fixed order, so results
// are bitwise reproducible. Per-term products use the plan's arithmetic type.
#include "icr_internal.h"

namespace icr {
namespace {

constexpr int kHgBlocks = 512;   // workgroups per sample and term
constexpr int kHgThreads = 256;

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

// Fixed-order sum over the workgroup of one double per thread, written by thread 0.
__device__ void block_sum_store(double v, double* out) {
  __shared__ double red[kHgThreads];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kHgThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// One refinement level: thread t takes interior coarse pixels t, t + stride, ... and
// accumulates <sbar block, dR s[window] + dsqrtD xi block> in FP64.
template <int D, typename TS, bool kCharted>
__global__ void __launch_bounds__(kHgThreads) hg_level_kernel(HgGeom g, const TS* __restrict__ s_in, int64_t s_bs,
                                                             const TS* __restrict__ xi, int64_t xi_bs,
                                                             const TS* __restrict__ sb, int64_t sb_bs,
                                                             const typename Acc<TS>::type* dR,
                                                             const typename Acc<TS>::type* dS,
                                                             double* __restrict__ part, int64_t part_bs) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  const int64_t b = blockIdx.y;
  __shared__ TA lds_r[kCharted ? 1 : NC * NW], lds_s[kCharted ? 1 : NC * NC];
  if (!kCharted) {  // a stationary level's matrices, staged once per workgroup
    for (int e = threadIdx.x; e < NC * NW; e += blockDim.x) lds_r[e] = dR[e];
    for (int e = threadIdx.x; e < NC * NC; e += blockDim.x) lds_s[e] = dS[e];
    __syncthreads();
    dR = lds_r;
    dS = lds_s;
  }
  s_in += b * s_bs;
  xi += b * xi_bs;
  sb += b * sb_bs;
  const int64_t stride = kCharted ? g.msets : 1;
  double acc = 0.0;
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
      TA o = 0;
      for (int iw = 0; iw < NW; ++iw) o += dR[(ib * NW + iw) * stride + set] * win[iw];
      for (int jb = 0; jb <= ib; ++jb) o += dS[(ib * NC + jb) * stride + set] * fresh[jb];
      acc += static_cast<double>(cot[ib]) * static_cast<double>(o);
    }
  }
  block_sum_store(acc, part + b * part_bs + blockIdx.x);
}

// Level 0: sum_i sbar_0[i] sum_{j <= i} dL00[i][j] xi_0[j] with the FP64 derivative;
// one wavefront per row (lanes stride the row, butterfly sum in a fixed order).
template <typename TS>
__global__ void __launch_bounds__(kHgThreads) hg_level0_kernel(const double* __restrict__ dl, int64_t n,
                                                              const TS* __restrict__ xi, int64_t xi_bs,
                                                              const TS* __restrict__ sb, int64_t sb_bs,
                                                              double* __restrict__ part, int64_t part_bs) {
  const int64_t b = blockIdx.y;
  xi += b * xi_bs;
  sb += b * sb_bs;
  const int lane = threadIdx.x & 63;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / 64);
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x / 64) + threadIdx.x / 64; i < n; i += waves) {
    double r = 0.0;
    for (int64_t j = lane; j <= i; j += 64) r += dl[i * n + j] * static_cast<double>(load_acc(xi + j));
    for (int m = 32; m > 0; m >>= 1) r += __shfl_xor(r, m, 64);
    if (lane == 0) acc += static_cast<double>(load_acc(sb + i)) * r;
  }
  block_sum_store(acc, part + b * part_bs + blockIdx.x);
}

// <a, b> over n elements per sample.
template <typename TS>
__global__ void __launch_bounds__(kHgThreads) hg_dot_kernel(const TS* __restrict__ a, int64_t a_bs,
                                                           const TS* __restrict__ c, int64_t c_bs, int64_t n,
                                                           double* __restrict__ part, int64_t part_bs) {
  const int64_t b = blockIdx.y;
  a += b * a_bs;
  c += b * c_bs;
  double acc = 0.0;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x)
    acc += static_cast<double>(load_acc(a + k)) * static_cast<double>(load_acc(c + k));
  block_sum_store(acc, part + b * part_bs + blockIdx.x);
}

// Per sample: grad = (sum of the sigma partials / sigma, sum of all length partials).
__global__ void __launch_bounds__(kHgThreads) hg_final_kernel(const double* __restrict__ part, int64_t part_bs,
                                                             int64_t len_parts, double inv_sigma,
                                                             double* __restrict__ grad) {
  const int64_t b = blockIdx.x;
  const double* p = part + b * part_bs;
  __shared__ double out[2];
  for (int which = 0; which < 2; ++which) {
    const double* q = which == 0 ? p : p + kHgBlocks;
    const int64_t cnt = which == 0 ? kHgBlocks : len_parts;
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < cnt; k += blockDim.x) v += q[k];
    __shared__ double red[kHgThreads];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kHgThreads / 2; w > 0; w >>= 1) {
      if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[which] = red[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    grad[2 * b] = out[0] * inv_sigma;
    grad[2 * b + 1] = out[1];
  }
}

template <int D, typename TS>
hipError_t level_term(const icr_plan* p, int l, int64_t batch, const TS* s_in, int64_t s_bs, const TS* xi,
                      int64_t xi_bs, const TS* sb, int64_t sb_bs, double* part, int64_t part_bs,
                      hipStream_t st) {
  using TA = typename Acc<TS>::type;
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
  if (p->charted)
    hg_level_kernel<D, TS, true><<<grid, kHgThreads, 0, st>>>(g, s_in, s_bs, xi, xi_bs, sb, sb_bs, dr, ds, part, part_bs);
  else
    hg_level_kernel<D, TS, false><<<grid, kHgThreads, 0, st>>>(g, s_in, s_bs, xi, xi_bs, sb, sb_bs, dr, ds, part, part_bs);
  return hipGetLastError();
}

template <typename TS>
hipError_t hyper_grad_t(const icr_plan* p, int64_t batch, const TS* xi, const TS* s, const TS* s_levels,
                        const TS* s_bar, const TS* sbar_levels, double* grad, double* part, hipStream_t st) {
  const int L = p->depth;
  const int64_t pbs = hypergrad_partials(p);
  const int64_t ws_bs = p->n_xi - p->n_out;
  const dim3 grid(kHgBlocks, static_cast<unsigned>(batch));
  // partial sums per sample: [sigma][level 0][level 0 -> 1] ... [level L-1 -> L]
  hg_dot_kernel<TS><<<grid, kHgThreads, 0, st>>>(s_bar, p->n_out, s, p->n_out, p->n_out, part, pbs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const TS* sb0 = L > 0 ? sbar_levels : s_bar;
  const int64_t sb0_bs = L > 0 ? ws_bs : p->n_out;
  hg_level0_kernel<TS><<<grid, kHgThreads, 0, st>>>(p->dl00_64, p->n0, xi, p->n_xi, sb0, sb0_bs, part + kHgBlocks, pbs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int l = 0; l < L; ++l) {
    const TS* s_in = s_levels + p->offsets[l];
    const TS* xf = xi + p->offsets[l + 1];
    const TS* sb = l + 1 < L ? sbar_levels + p->offsets[l + 1] : s_bar;
    const int64_t sb_bs = l + 1 < L ? ws_bs : p->n_out;
    double* pl = part + int64_t(2 + l) * kHgBlocks;
    switch (p->ndim) {
      case 1: e = level_term<1, TS>(p, l, batch, s_in, ws_bs, xf, p->n_xi, sb, sb_bs, pl, pbs, st); break;
      case 2: e = level_term<2, TS>(p, l, batch, s_in, ws_bs, xf, p->n_xi, sb, sb_bs, pl, pbs, st); break;
      default: e = level_term<3, TS>(p, l, batch, s_in, ws_bs, xf, p->n_xi, sb, sb_bs, pl, pbs, st); break;
    }
    if (e != hipSuccess) return e;
  }
  hg_final_kernel<<<static_cast<unsigned>(batch), kHgThreads, 0, st>>>(part, pbs, int64_t(L + 1) * kHgBlocks,
                                                                       1.0 / p->cfg.scale, grad);
  return hipGetLastError();
}

}  // namespace

int64_t hypergrad_partials(const icr_plan* p) { return int64_t(p->depth + 2) * kHgBlocks; }

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
