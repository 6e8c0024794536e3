// One ICR refinement level, general form: any d in {1,2,3}, any precision,
// shared (stationary), per-pixel or per-shell (charted) matrices, any alignment.
//
// Forward (one thread per interior coarse pixel c and sample):
//   s_{l+1}[2(c-1)+b] = sum_w R[b,w] s_l[c+w] + sum_{b'<=b} sqrtD[b,b'] xi_{l+1}[2(c-1)+b']
// Adjoint (one thread per coarse pixel p and sample), the transpose as a gather:
//   s_bar_l[p] = sum_w sum_b R_c[b,w] y[2(c-1)+b]  over interior c = p - w,
//   xi_bar_{l+1}[2(p-1)+b'] = sum_{b>=b'} sqrtD[b,b'] y[2(p-1)+b]   (p interior).
// Every output element is written by exactly one thread in a fixed summation
// order, so there are no atomics and results are bitwise reproducible.
#include "icr_internal.h"

namespace icr {
namespace {

struct Geom {
  int nc[3];  // coarse shape, natural axis order (first D used)
  int nf[3];  // fine shape
  int mi[3];  // interior coarse pixels per axis
  int64_t nsets;  // interior coarse pixels (= prod mi)
  int64_t msets;  // charted: matrix sets, the stride between a set's entries
  int shell;      // charted with one set per interior index of the first axis
};

template <int D>
__device__ __forceinline__ int64_t lin(const int* idx, const int* shape) {
  int64_t v = idx[0];
  for (int a = 1; a < D; ++a) v = v * shape[a] + idx[a];
  return v;
}

template <int D, typename TS, bool kCharted>
__global__ void __launch_bounds__(256) refine_fwd_generic(Geom g, RefineFwdArgs a,
                                                          const typename Acc<TS>::type* R,
                                                          const typename Acc<TS>::type* S) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  if (halted(a.halt)) return;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t b = blockIdx.y;
  // a stationary level's R and sqrtD are staged in LDS with one cooperative load (read
  // element by element from memory they would be a long chain of dependent loads)
  __shared__ TA lds_r[kCharted ? 1 : NC * NW], lds_s[kCharted ? 1 : NC * NC];
  if (!kCharted) {
    for (int e = threadIdx.x; e < NC * NW; e += blockDim.x) lds_r[e] = R[e];
    for (int e = threadIdx.x; e < NC * NC; e += blockDim.x) lds_s[e] = S[e];
    __syncthreads();
    R = lds_r;
    S = lds_s;
  }
  if (t >= g.nsets) return;  // nsets = prod(mi) for both stationary and charted here
  int c[D];
  {
    int64_t rem = t;
    for (int ax = D - 1; ax >= 0; --ax) { c[ax] = static_cast<int>(rem % g.mi[ax]) + 1; rem /= g.mi[ax]; }
  }
  const TS* s_in = static_cast<const TS*>(a.s_in) + b * a.s_in_bs;
  const TS* xi = static_cast<const TS*>(a.xi) + b * a.xi_bs;
  TS* s_out = static_cast<TS*>(a.s_out) + b * a.s_out_bs;
  const TA* w = a.w ? static_cast<const TA*>(a.w) + b * a.w_bs : nullptr;

  TA win[NW];
  for (int iw = 0; iw < NW; ++iw) {
    int q[D];
    int rem = iw;
    for (int ax = D - 1; ax >= 0; --ax) { q[ax] = c[ax] + (rem % 3) - 1; rem /= 3; }
    win[iw] = load_acc(s_in + lin<D>(q, g.nc));
  }
  TA fresh[NC];
  int64_t fidx[NC];
  for (int ib = 0; ib < NC; ++ib) {
    int q[D];
    for (int ax = 0; ax < D; ++ax) q[ax] = 2 * (c[ax] - 1) + ((ib >> (D - 1 - ax)) & 1);
    fidx[ib] = lin<D>(q, g.nf);
    fresh[ib] = load_acc(xi + fidx[ib]);
  }
  const int64_t stride = kCharted ? g.msets : 1;
  const int64_t base = kCharted ? (g.shell ? c[0] - 1 : t) : 0;
  for (int ib = 0; ib < NC; ++ib) {
    TA acc = 0;
    for (int iw = 0; iw < NW; ++iw) acc += R[(ib * NW + iw) * stride + base] * win[iw];
    for (int jb = 0; jb <= ib; ++jb) acc += S[(ib * NC + jb) * stride + base] * fresh[jb];
    if (w) acc *= w[fidx[ib]];
    store_acc(s_out + fidx[ib], acc);
  }
}

template <int D, typename TS, bool kCharted>
__global__ void __launch_bounds__(256) refine_adj_generic(Geom g, int64_t ncoarse, RefineAdjArgs a,
                                                          const typename Acc<TS>::type* R,
                                                          const typename Acc<TS>::type* S) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  if (halted(a.halt)) return;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t b = blockIdx.y;
  __shared__ TA lds_r[kCharted ? 1 : NC * NW], lds_s[kCharted ? 1 : NC * NC];  // as in the forward
  if (!kCharted) {
    for (int e = threadIdx.x; e < NC * NW; e += blockDim.x) lds_r[e] = R[e];
    for (int e = threadIdx.x; e < NC * NC; e += blockDim.x) lds_s[e] = S[e];
    __syncthreads();
    R = lds_r;
    S = lds_s;
  }
  if (t >= ncoarse) return;
  int p[D];
  {
    int64_t rem = t;
    for (int ax = D - 1; ax >= 0; --ax) { p[ax] = static_cast<int>(rem % g.nc[ax]); rem /= g.nc[ax]; }
  }
  const TS* y = static_cast<const TS*>(a.y) + b * a.y_bs;
  const int64_t stride = kCharted ? g.msets : 1;

  // coarse cotangent: gather the blocks c = p - w that read p at window slot w. A block
  // outside the interior is read at a clamped (in-bounds) position and weighted by zero,
  // so no load sits under a branch and all of them can be in flight at once.
  TA acc = 0;
#pragma unroll
  for (int iw = 0; iw < NW; ++iw) {
    int c[D];
    bool inside = true;
    int rem = iw;
#pragma unroll
    for (int ax = D - 1; ax >= 0; --ax) {
      const int cv = p[ax] - ((rem % 3) - 1);
      rem /= 3;
      inside = inside && cv >= 1 && cv <= g.nc[ax] - 2;
      c[ax] = min(max(cv, 1), g.nc[ax] - 2);
    }
    int64_t set = 0;
    if (kCharted) {
      int ci[D];
#pragma unroll
      for (int ax = 0; ax < D; ++ax) ci[ax] = c[ax] - 1;
      set = g.shell ? ci[0] : lin<D>(ci, g.mi);
    }
    TA part = 0;
#pragma unroll
    for (int ib = 0; ib < NC; ++ib) {
      int q[D];
#pragma unroll
      for (int ax = 0; ax < D; ++ax) q[ax] = 2 * (c[ax] - 1) + ((ib >> (D - 1 - ax)) & 1);
      part += R[(ib * NW + iw) * stride + set] * load_acc(y + lin<D>(q, g.nf));
    }
    acc += inside ? part : TA(0);
  }
  store_acc(static_cast<TS*>(a.s_bar) + b * a.s_bar_bs + t, acc);

  // excitation cotangent of the block spawned by p, if p is interior
  bool interior = true;
  for (int ax = 0; ax < D; ++ax) interior = interior && p[ax] >= 1 && p[ax] <= g.nc[ax] - 2;
  if (!interior) return;
  int64_t set = 0;
  if (kCharted) {
    int ci[D];
    for (int ax = 0; ax < D; ++ax) ci[ax] = p[ax] - 1;
    set = g.shell ? ci[0] : lin<D>(ci, g.mi);
  }
  TA yb[NC];
  int64_t fidx[NC];
  for (int ib = 0; ib < NC; ++ib) {
    int q[D];
    for (int ax = 0; ax < D; ++ax) q[ax] = 2 * (p[ax] - 1) + ((ib >> (D - 1 - ax)) & 1);
    fidx[ib] = lin<D>(q, g.nf);
    yb[ib] = load_acc(y + fidx[ib]);
  }
  TS* xb = static_cast<TS*>(a.xi_bar) + b * a.xi_bar_bs;
  const TS* add = a.add ? static_cast<const TS*>(a.add) + b * a.add_bs : nullptr;
  for (int jb = 0; jb < NC; ++jb) {
    TA v = 0;
    for (int ib = jb; ib < NC; ++ib) v += S[(ib * NC + jb) * stride + set] * yb[ib];
    if (add) v += load_acc(add + fidx[jb]);
    store_acc(xb + fidx[jb], v);
  }
}

Geom geom_of(const icr_plan* p, int level) {
  Geom g;
  const int d = p->ndim;
  for (int a = 0; a < 3; ++a) {
    g.nc[a] = a < d ? p->shapes[level][3 - d + a] : 1;
    g.nf[a] = a < d ? p->shapes[level + 1][3 - d + a] : 1;
    g.mi[a] = a < d ? g.nc[a] - 2 : 1;
  }
  g.nsets = 1;
  for (int a = 0; a < d; ++a) g.nsets *= g.mi[a];
  g.msets = p->lev[level].nsets;
  g.shell = p->shell;
  return g;
}

template <int D, typename TS, bool kCharted>
hipError_t fwd_one(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st) {
  using TA = typename Acc<TS>::type;
  const Geom g = geom_of(p, level);
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineFwdArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.s_in = static_cast<const TS*>(a.s_in) + b0 * a.s_in_bs;
    c.xi = static_cast<const TS*>(a.xi) + b0 * a.xi_bs;
    c.s_out = static_cast<TS*>(a.s_out) + b0 * a.s_out_bs;
    if (a.w) c.w = static_cast<const TA*>(a.w) + b0 * a.w_bs;
    const dim3 grid(static_cast<unsigned>((g.nsets + 255) / 256), static_cast<unsigned>(c.batch));
    refine_fwd_generic<D, TS, kCharted><<<grid, 256, 0, st>>>(
        g, c, static_cast<const TA*>(p->lev[level].r_c), static_cast<const TA*>(p->lev[level].s_c));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int D, typename TS, bool kCharted>
hipError_t adj_one(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st) {
  using TA = typename Acc<TS>::type;
  const Geom g = geom_of(p, level);
  int64_t ncoarse = 1;
  for (int ax = 0; ax < D; ++ax) ncoarse *= g.nc[ax];
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineAdjArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.y = static_cast<const TS*>(a.y) + b0 * a.y_bs;
    c.xi_bar = static_cast<TS*>(a.xi_bar) + b0 * a.xi_bar_bs;
    c.s_bar = static_cast<TS*>(a.s_bar) + b0 * a.s_bar_bs;
    if (a.add) c.add = static_cast<const TS*>(a.add) + b0 * a.add_bs;
    const dim3 grid(static_cast<unsigned>((ncoarse + 255) / 256), static_cast<unsigned>(c.batch));
    refine_adj_generic<D, TS, kCharted><<<grid, 256, 0, st>>>(
        g, ncoarse, c, static_cast<const TA*>(p->lev[level].r_c), static_cast<const TA*>(p->lev[level].s_c));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int D, typename TS>
hipError_t fwd_d(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st) {
  return p->charted ? fwd_one<D, TS, true>(p, level, a, st) : fwd_one<D, TS, false>(p, level, a, st);
}
template <int D, typename TS>
hipError_t adj_d(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st) {
  return p->charted ? adj_one<D, TS, true>(p, level, a, st) : adj_one<D, TS, false>(p, level, a, st);
}

template <typename TS>
hipError_t fwd_t(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st) {
  switch (p->ndim) {
    case 1: return fwd_d<1, TS>(p, level, a, st);
    case 2: return fwd_d<2, TS>(p, level, a, st);
    default: return fwd_d<3, TS>(p, level, a, st);
  }
}
template <typename TS>
hipError_t adj_t(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st) {
  switch (p->ndim) {
    case 1: return adj_d<1, TS>(p, level, a, st);
    case 2: return adj_d<2, TS>(p, level, a, st);
    default: return adj_d<3, TS>(p, level, a, st);
  }
}

}  // namespace

hipError_t launch_refine_fwd_generic(const icr_plan* p, int level, const RefineFwdArgs& a,
                                     hipStream_t st) {
  switch (p->precision) {
    case ICR_F64: return fwd_t<double>(p, level, a, st);
    case ICR_F32: return fwd_t<float>(p, level, a, st);
    default: return fwd_t<bf16_t>(p, level, a, st);
  }
}

hipError_t launch_refine_adj_generic(const icr_plan* p, int level, const RefineAdjArgs& a,
                                     hipStream_t st) {
  switch (p->precision) {
    case ICR_F64: return adj_t<double>(p, level, a, st);
    case ICR_F32: return adj_t<float>(p, level, a, st);
    default: return adj_t<bf16_t>(p, level, a, st);
  }
}

}  // namespace icr
