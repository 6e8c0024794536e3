// The smallest levels of a sweep in one launch: one workgroup per sample runs level 0
// (when its factor is small) and the first K refinement levels back to back, keeping
// each level's field in LDS for the next. Small levels are bound by the latency of a
// launch and of a dependent load chain, not by bandwidth, so one launch in place of
// K (+1) saves that latency K times.
//
// Forward, level l -> l+1, per interior coarse block c and child b (dense R, lower sqrtD):
//   s_{l+1}[2(c-1)+b] = sum_w R_l[b,w] s_l[c+w] + sum_{b'<=b} sqrtD_l[b,b'] xi_{l+1}[2(c-1)+b']
// Adjoint, level l+1 -> l (a gather, no atomics):
//   xi_bar_{l+1}[2(c-1)+b'] = sum_{b>=b'} sqrtD_l[b,b'] y[2(c-1)+b],
//   s_bar_l[p] = sum_{w, c = p - w interior} sum_b R_l[b,w] y[2(c-1)+b].
// Every level is also written to the workspace (as the per-level kernels do), so the
// sweep's outputs and intermediates are laid out exactly as without fusion. Each value
// is summed by one thread in a fixed order: results are bitwise reproducible.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "icr_internal.h"

namespace icr {
namespace {

constexpr int kFusedThreads = 1024;
constexpr int kMaxFused = 8;               // refinement levels in one launch
// fine elements (summed over the fused levels) one workgroup takes on per sample: beyond
// these a workgroup's own latency outgrows the launches it saves (measured: the 3-D
// 16^3 and 28^3 levels and the 2-D levels up to 100^2 are faster as separate launches)
constexpr int64_t kMaxFusedElems[3] = {32768, 2048, 512};
constexpr int64_t kFusedLds = 160 * 1024 - 4096;
constexpr int64_t kMaxLevel0 = 64;         // level-0 sizes whose factor is applied in the launch

struct FusedArgs {
  int K;                          // refinements 0 .. K-1
  int level0;                     // apply the level-0 factor in the launch
  int n0;                         // level-0 size
  const void* l0;                 // forward: lower factor L00, adjoint: U00 = L00^T (row-major)
  int shape[kMaxFused + 1][3];    // level shapes, leading 1s
  int64_t off[kMaxFused + 1];     // xi offsets of levels 0 .. K
  int64_t size[kMaxFused + 1];    // level sizes
  const void* r[kMaxFused];       // dense R_l [NC][NW], arithmetic type
  const void* s[kMaxFused];       // sqrtD_l [NC][NC]
  int64_t lds_even, lds_odd;      // LDS elements for the even / odd levels' fields
  int64_t pre;                    // LDS elements of the prefetched xi (forward) / add (adjoint)
  // forward
  const void* xi;                 // [batch][n_xi]
  void* ws; int64_t ws_bs;        // workspace, levels at their xi offsets
  void* out; int64_t out_bs;      // level K when it is the last level (else the workspace)
  const void* w; int64_t w_bs;    // final level times w (metric), arithmetic type
  // adjoint
  const void* y; int64_t y_bs;    // cotangent of level K
  void* xi_bar;                   // [batch][n_xi]
  const void* add;                // xi_bar += add (metric), [batch][n_xi]
  int64_t n_xi;
  int64_t batch0;                 // first sample of this launch
  const int32_t* halt;            // device flag: when set the launch does nothing
};

template <int D>
__device__ __forceinline__ int64_t lin3(const int* idx, const int* shape) {
  int64_t v = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) v = v * shape[3 - D + a] + idx[a];
  return v;
}

template <typename TA>
__device__ __forceinline__ TA wave_total(TA v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// a value as the storage type holds it (bfloat16 storage rounds every stored field; the
// LDS copies a fused level hands to the next are rounded alike)
template <typename TS, typename TA>
__device__ __forceinline__ TA as_stored(TA v) {
  TS tmp;
  store_acc(&tmp, v);
  return load_acc(&tmp);
}

// field of level l in LDS: even levels in the first region, odd levels in the second
template <typename TA>
__device__ __forceinline__ TA* level_lds(TA* base, const FusedArgs& g, int l) {
  return (l & 1) ? base + g.lds_even : base;
}

// Every fused level's R and sqrtD into LDS in one round: each thread loads its element
// of every level before storing any (a loop over the levels waited for each level's
// loads in turn). Levels past K reload the last one and are not stored.
template <int NC, int NW, typename TA>
__device__ __forceinline__ void copy_mats(TA* mats, const FusedArgs& g, int t) {
  constexpr int kPer = NC * NW + NC * NC;
  static_assert(kPer <= kFusedThreads, "one element of each level per thread");
  if (t >= kPer || g.K < 1) return;
  TA v[kMaxFused];
#pragma unroll
  for (int l = 0; l < kMaxFused; ++l) {
    const int lc = l < g.K ? l : g.K - 1;
    v[l] = t < NC * NW ? static_cast<const TA*>(g.r[lc])[t] : static_cast<const TA*>(g.s[lc])[t - NC * NW];
  }
#pragma unroll
  for (int l = 0; l < kMaxFused; ++l)
    if (l < g.K) mats[l * kPer + t] = v[l];
}

// rows of the level-0 factor a wavefront reduces (n0 <= kMaxLevel0, one row per wavefront
// of the workgroup at a time)
constexpr int kLevel0Rows = (kMaxLevel0 + kFusedThreads / 64 - 1) / (kFusedThreads / 64);

template <int D, typename TS>
__global__ void __launch_bounds__(kFusedThreads) fused_fwd(FusedArgs g) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D), NC = 1 << D;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TA* fields = reinterpret_cast<TA*>(lds_raw);
  TA* mats = fields + g.lds_even + g.lds_odd;  // R then sqrtD of every fused level
  TA* xl = mats + g.K * (NC * NW + NC * NC);     // the excitations of levels 0 .. K
  if (halted(g.halt)) return;
  const int t = threadIdx.x;
  const int64_t b = g.batch0 + blockIdx.x;
  const TS* xi = static_cast<const TS*>(g.xi) + b * g.n_xi;
  TS* ws = static_cast<TS*>(g.ws) + b * g.ws_bs;
  // every input is fetched in one round before any level is computed
  copy_widen<16>(xl, xi, g.pre, t, kFusedThreads);
  copy_mats<NC, NW>(mats, g, t);
  // level 0
  TA* s0 = level_lds(fields, g, 0);
  if (g.level0) {  // one wavefront per row of L00 (n0 <= 64: a lane per column)
    const TA* L = static_cast<const TA*>(g.l0);
    const int lane = t % 64, wv = t / 64;
    TA lrow[kLevel0Rows];  // this wavefront's rows, loaded with the other inputs
#pragma unroll
    for (int r = 0; r < kLevel0Rows; ++r) {
      const int i = min(wv + r * (kFusedThreads / 64), g.n0 - 1);
      lrow[r] = L[int64_t(i) * g.n0 + min(lane, g.n0 - 1)];
    }
    __syncthreads();  // the prefetched xi_0
#pragma unroll
    for (int r = 0; r < kLevel0Rows; ++r) {
      const int i = wv + r * (kFusedThreads / 64);
      if (i >= g.n0) break;  // uniform over the wavefront
      TA acc = lane <= i ? lrow[r] * xl[lane] : TA(0);
      acc = wave_total(acc);
      if (lane == 0) {
        s0[i] = as_stored<TS>(acc);
        store_acc(ws + i, acc);
      }
    }
  } else {
    for (int i = t; i < g.n0; i += kFusedThreads) s0[i] = load_acc(ws + i);
  }
  __syncthreads();
  for (int l = 0; l < g.K; ++l) {
    const int* C = g.shape[l];
    const int* F = g.shape[l + 1];
    const TA* sc = level_lds(fields, g, l);
    TA* sf = level_lds(fields, g, l + 1);
    const TA* R = mats + l * (NC * NW + NC * NC);
    const TA* S = R + NC * NW;
    const bool last = l == g.K - 1;
    const bool to_out = last && g.out;  // level K is the sweep's output
    TS* dst = to_out ? static_cast<TS*>(g.out) + b * g.out_bs : ws + g.off[l + 1];
    const TA* w = to_out && g.w ? static_cast<const TA*>(g.w) + b * g.w_bs : nullptr;
    const TA* xf = xl + g.off[l + 1];
    int mi[3];
    int64_t blocks = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) { mi[a] = C[3 - D + a] - 2; blocks *= mi[a]; }
    for (int64_t k = t; k < blocks; k += kFusedThreads) {
      int c[D];
      int64_t rem = k;
#pragma unroll
      for (int a = D - 1; a >= 0; --a) { c[a] = static_cast<int>(rem % mi[a]) + 1; rem /= mi[a]; }
      TA win[NW];
#pragma unroll
      for (int iw = 0; iw < NW; ++iw) {
        int q[D];
        int r = iw;
#pragma unroll
        for (int a = D - 1; a >= 0; --a) { q[a] = c[a] + (r % 3) - 1; r /= 3; }
        win[iw] = sc[lin3<D>(q, C)];
      }
      int64_t fi[NC];
      TA x[NC];
#pragma unroll
      for (int ib = 0; ib < NC; ++ib) {
        int q[D];
#pragma unroll
        for (int a = 0; a < D; ++a) q[a] = 2 * (c[a] - 1) + ((ib >> (D - 1 - a)) & 1);
        fi[ib] = lin3<D>(q, F);
        x[ib] = xf[fi[ib]];
      }
#pragma unroll
      for (int ib = 0; ib < NC; ++ib) {
        TA acc = 0;
#pragma unroll
        for (int iw = 0; iw < NW; ++iw) acc += R[ib * NW + iw] * win[iw];
#pragma unroll
        for (int jb = 0; jb <= ib; ++jb) acc += S[ib * NC + jb] * x[jb];
        if (!last) sf[fi[ib]] = as_stored<TS>(acc);
        store_acc(dst + fi[ib], w ? acc * w[fi[ib]] : acc);
      }
    }
    __syncthreads();
  }
}

template <int D, typename TS>
__global__ void __launch_bounds__(kFusedThreads) fused_adj(FusedArgs g) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D), NC = 1 << D;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TA* fields = reinterpret_cast<TA*>(lds_raw);
  TA* mats = fields + g.lds_even + g.lds_odd;
  TA* al = mats + g.K * (NC * NW + NC * NC);  // the metric's addends of levels 0 .. K
  if (halted(g.halt)) return;
  const int t = threadIdx.x;
  const int64_t b = g.batch0 + blockIdx.x;
  TS* xb = static_cast<TS*>(g.xi_bar) + b * g.n_xi;
  const bool add = g.add != nullptr;
  if (add) {  // fetched with the cotangent, in one round
    const TS* ag = static_cast<const TS*>(g.add) + b * g.n_xi;
    copy_widen<16>(al, ag, g.pre, t, kFusedThreads);
  }
  TS* ws = static_cast<TS*>(g.ws) + b * g.ws_bs;
  copy_mats<NC, NW>(mats, g, t);
  {  // the cotangent of level K
    const TS* y = static_cast<const TS*>(g.y) + b * g.y_bs;
    TA* yk = level_lds(fields, g, g.K);
    copy_widen<16>(yk, y, g.size[g.K], t, kFusedThreads);
  }
  // this wavefront's rows of U00 (n0 <= 64: a lane per column), loaded with the other inputs
  const int lane = t % 64, wv = t / 64;
  TA urow[kLevel0Rows];
  if (g.level0) {
    const TA* U = static_cast<const TA*>(g.l0);
#pragma unroll
    for (int r = 0; r < kLevel0Rows; ++r) {
      const int i = min(wv + r * (kFusedThreads / 64), g.n0 - 1);
      urow[r] = U[int64_t(i) * g.n0 + min(i + lane, g.n0 - 1)];
    }
  }
  __syncthreads();
  for (int l = g.K - 1; l >= 0; --l) {
    const int* C = g.shape[l];
    const int* F = g.shape[l + 1];
    const TA* y = level_lds(fields, g, l + 1);
    TA* sb = level_lds(fields, g, l);
    const TA* R = mats + l * (NC * NW + NC * NC);
    const TA* S = R + NC * NW;
    int mi[3];
    int64_t blocks = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) { mi[a] = C[3 - D + a] - 2; blocks *= mi[a]; }
    // excitation cotangents of the blocks of level l+1
    for (int64_t k = t; k < blocks; k += kFusedThreads) {
      int c[D];
      int64_t rem = k;
#pragma unroll
      for (int a = D - 1; a >= 0; --a) { c[a] = static_cast<int>(rem % mi[a]) + 1; rem /= mi[a]; }
      int64_t fi[NC];
      TA yv[NC];
#pragma unroll
      for (int ib = 0; ib < NC; ++ib) {
        int q[D];
#pragma unroll
        for (int a = 0; a < D; ++a) q[a] = 2 * (c[a] - 1) + ((ib >> (D - 1 - a)) & 1);
        fi[ib] = lin3<D>(q, F);
        yv[ib] = y[fi[ib]];
      }
#pragma unroll
      for (int jb = 0; jb < NC; ++jb) {
        TA v = 0;
#pragma unroll
        for (int ib = jb; ib < NC; ++ib) v += S[ib * NC + jb] * yv[ib];
        if (add) v += al[g.off[l + 1] + fi[jb]];
        store_acc(xb + g.off[l + 1] + fi[jb], v);
      }
    }
    // coarse cotangents of level l: gather from the blocks whose window holds each pixel
    const int64_t nc = g.size[l];
    for (int64_t k = t; k < nc; k += kFusedThreads) {
      int p[D];
      int64_t rem = k;
#pragma unroll
      for (int a = D - 1; a >= 0; --a) {
        const int n = C[3 - D + a];
        p[a] = static_cast<int>(rem % n);
        rem /= n;
      }
      TA acc = 0;
#pragma unroll
      for (int iw = 0; iw < NW; ++iw) {
        int c[D];
        bool inside = true;
        int r = iw;
#pragma unroll
        for (int a = D - 1; a >= 0; --a) {
          c[a] = p[a] - ((r % 3) - 1);
          r /= 3;
          inside = inside && c[a] >= 1 && c[a] <= C[3 - D + a] - 2;
        }
        if (!inside) continue;
#pragma unroll
        for (int ib = 0; ib < NC; ++ib) {
          int q[D];
#pragma unroll
          for (int a = 0; a < D; ++a) q[a] = 2 * (c[a] - 1) + ((ib >> (D - 1 - a)) & 1);
          acc += R[ib * NW + iw] * y[lin3<D>(q, F)];
        }
      }
      sb[k] = as_stored<TS>(acc);
      store_acc(ws + g.off[l] + k, acc);
    }
    __syncthreads();
  }
  if (g.level0) {  // xi_bar_0 = U00 s_bar_0 (+ add): one wavefront per row
    const TA* s0 = level_lds(fields, g, 0);
#pragma unroll
    for (int r = 0; r < kLevel0Rows; ++r) {
      const int i = wv + r * (kFusedThreads / 64);
      if (i >= g.n0) break;  // uniform over the wavefront
      TA acc = i + lane < g.n0 ? urow[r] * s0[i + lane] : TA(0);
      acc = wave_total(acc);
      if (lane == 0) {
        if (add) acc += al[i];
        store_acc(xb + i, acc);
      }
    }
  }
}

template <typename TS>
size_t lds_bytes(const FusedArgs& g, int d) {
  using TA = typename Acc<TS>::type;
  const int nc = 1 << d, nw = pow3(d);
  return sizeof(TA) * (size_t(g.lds_even + g.lds_odd + g.pre) + size_t(g.K) * (nc * nw + nc * nc));
}

template <typename TS, bool kFwd>
hipError_t launch_t(const icr_plan* p, FusedArgs g, int64_t batch, hipStream_t st) {
  const size_t lds = lds_bytes<TS>(g, p->ndim);
  if (lds > static_cast<size_t>(kFusedLds)) return hipErrorInvalidValue;  // excluded by fused_levels
  for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
    g.batch0 = b0;
    const dim3 grid(static_cast<unsigned>(std::min<int64_t>(batch - b0, 65535)));
    const void* fn = nullptr;
    switch (p->ndim) {
      case 1: fn = kFwd ? reinterpret_cast<const void*>(fused_fwd<1, TS>) : reinterpret_cast<const void*>(fused_adj<1, TS>); break;
      case 2: fn = kFwd ? reinterpret_cast<const void*>(fused_fwd<2, TS>) : reinterpret_cast<const void*>(fused_adj<2, TS>); break;
      default: fn = kFwd ? reinterpret_cast<const void*>(fused_fwd<3, TS>) : reinterpret_cast<const void*>(fused_adj<3, TS>); break;
    }
    // allow more than the default dynamic LDS (the device holds 160 KB per workgroup);
    // set once per kernel: the call costs host time a launch sequence cannot afford
    static std::once_flag once[3];
    static hipError_t set_err[3] = {hipSuccess, hipSuccess, hipSuccess};
    const int di = p->ndim - 1;
    std::call_once(once[di], [&] {
      set_err[di] = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kFusedLds));
    });
    if (set_err[di] != hipSuccess) return set_err[di];
    switch (p->ndim) {
      case 1:
        if (kFwd) fused_fwd<1, TS><<<grid, kFusedThreads, lds, st>>>(g);
        else fused_adj<1, TS><<<grid, kFusedThreads, lds, st>>>(g);
        break;
      case 2:
        if (kFwd) fused_fwd<2, TS><<<grid, kFusedThreads, lds, st>>>(g);
        else fused_adj<2, TS><<<grid, kFusedThreads, lds, st>>>(g);
        break;
      default:
        if (kFwd) fused_fwd<3, TS><<<grid, kFusedThreads, lds, st>>>(g);
        else fused_adj<3, TS><<<grid, kFusedThreads, lds, st>>>(g);
        break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Fill the static part of the arguments for the fused range; false if none is worth it.
bool plan_range(const icr_plan* p, int K, bool level0, FusedArgs* g) {
  std::memset(g, 0, sizeof(*g));
  g->K = K;
  g->level0 = level0 ? 1 : 0;
  g->n0 = static_cast<int>(p->offsets[1] - p->offsets[0]);
  for (int l = 0; l <= K; ++l) {
    for (int a = 0; a < 3; ++a) g->shape[l][a] = p->shapes[l][a];
    g->off[l] = p->offsets[l];
    g->size[l] = p->offsets[l + 1] - p->offsets[l];
    if (l % 2 == 0) g->lds_even = std::max(g->lds_even, g->size[l]);
    else g->lds_odd = std::max(g->lds_odd, g->size[l]);
  }
  for (int l = 0; l < K; ++l) {
    g->r[l] = p->lev[l].r_c;
    g->s[l] = p->lev[l].s_c;
  }
  g->n_xi = p->n_xi;
  g->pre = p->offsets[K + 1];
  return true;
}

}  // namespace

int fused_levels(const icr_plan* p, bool* level0) {
  *level0 = false;
  if (p->charted || p->depth < 1) return 0;
  const int d = p->ndim, nc = 1 << d, nw = pow3(d);
  const int64_t ta = p->precision == ICR_F64 ? 8 : 4;
  const int64_t n0 = p->offsets[1] - p->offsets[0];
  int64_t even = n0, odd = 0, fine = 0;
  int K = 0;
  while (K < p->depth && K < kMaxFused) {
    const int64_t nf = p->offsets[K + 2] - p->offsets[K + 1];
    if (fine + nf > kMaxFusedElems[d - 1]) break;
    const int64_t e2 = (K + 1) % 2 == 0 ? std::max(even, nf) : even;
    const int64_t o2 = (K + 1) % 2 == 1 ? std::max(odd, nf) : odd;
    const int64_t pre = p->offsets[K + 2];  // prefetched excitations / addends of levels 0 .. K+1
    if ((e2 + o2 + pre + int64_t(K + 1) * (nc * nw + nc * nc)) * ta > kFusedLds) break;
    even = e2;
    odd = o2;
    fine += nf;
    ++K;
  }
  *level0 = n0 <= kMaxLevel0;
  if (K >= 2 || (K >= 1 && *level0)) return K;
  *level0 = false;
  return 0;
}

hipError_t launch_fused_fwd(const icr_plan* p, int K, bool level0, int64_t batch, const void* xi, void* ws,
                            int64_t ws_bs, void* out, int64_t out_bs, const void* w, int64_t w_bs,
                            const int32_t* halt, hipStream_t st) {
  FusedArgs g;
  plan_range(p, K, level0, &g);
  g.halt = halt;
  g.l0 = p->l00_c;
  g.xi = xi;
  g.ws = ws;
  g.ws_bs = ws_bs;
  g.out = out;
  g.out_bs = out_bs;
  g.w = w;
  g.w_bs = w_bs;
  switch (p->precision) {
    case ICR_F64: return launch_t<double, true>(p, g, batch, st);
    case ICR_F32: return launch_t<float, true>(p, g, batch, st);
    default: return launch_t<bf16_t, true>(p, g, batch, st);
  }
}

hipError_t launch_fused_adj(const icr_plan* p, int K, bool level0, int64_t batch, const void* y, int64_t y_bs,
                            void* xi_bar, void* ws, int64_t ws_bs, const void* add, const int32_t* halt,
                            hipStream_t st) {
  FusedArgs g;
  plan_range(p, K, level0, &g);
  g.halt = halt;
  g.l0 = p->u00_c;
  g.y = y;
  g.y_bs = y_bs;
  g.xi_bar = xi_bar;
  g.ws = ws;
  g.ws_bs = ws_bs;
  g.add = add;
  switch (p->precision) {
    case ICR_F64: return launch_t<double, false>(p, g, batch, st);
    case ICR_F32: return launch_t<float, false>(p, g, batch, st);
    default: return launch_t<bf16_t, false>(p, g, batch, st);
  }
}

}  // namespace icr
