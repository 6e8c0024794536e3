// Level 0 of the ICR sweep: s_0 = L00 xi_0 with L00 the lower Cholesky factor of
// the kernel over the coarsest grid, and its transpose xi_bar_0 = L00^T s_bar_0
// (stored as the row-major upper factor U00 = L00^T so both directions stream
// rows). One wavefront per output element and sample; lanes stride the row with
// several loads in flight, and the partial sums are combined in a fixed order (pairwise,
// then a butterfly across lanes), so results are reproducible.
#include "icr_internal.h"

namespace icr {
namespace {

template <typename TA>
__device__ __forceinline__ TA wave_sum(TA v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// forward: out[i] = sum_{j <= i} L[i][j] in[j]      (lower = true)
// adjoint: out[i] = sum_{j >= i} U[i][j] in[j] + add (lower = false)
template <typename TS, bool kLower>
__global__ void __launch_bounds__(256) level0_kernel(const typename Acc<TS>::type* __restrict__ mat,
                                                     int64_t n, Level0Args a) {
  using TA = typename Acc<TS>::type;
  if (halted(a.halt)) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t b = blockIdx.y;
  if (row >= n) return;
  const TS* in = static_cast<const TS*>(a.in) + b * a.in_bs;
  const TA* m = mat + row * n;
  const int64_t j0 = kLower ? 0 : row;
  const int64_t j1 = kLower ? row + 1 : n;
  // kU independent partial sums so kU loads of the row are in flight at once (rows of up
  // to 1024, the 3-D workload's 10^3 level 0 included, in one round); a lane past the end
  // of the row reads an in-bounds element and adds zero, so no load sits in a divergent
  // branch. The input is loaded in its storage type and widened after the scheduling
  // barrier: widening each bfloat16 as it arrived made the compiler wait for every input
  // load in turn (8.6 against 4.2 us per product at 1000 x 1000).
  constexpr int kU = 16;
  TA part[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) part[u] = 0;
  for (int64_t base = j0; base < j1; base += 64 * kU) {
    TA mv[kU];
    TS xr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t j = base + u * 64 + lane;
      const int64_t jc = j < j1 ? j : j0;
      mv[u] = m[jc];
      xr[u] = in[jc];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kU; ++u) part[u] += (base + u * 64 + lane < j1 ? mv[u] : TA(0)) * load_acc(&xr[u]);
  }
#pragma unroll
  for (int w = kU / 2; w > 0; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) part[u] += part[u + w];
  const TA acc = wave_sum(part[0]);
  if (lane == 0) {
    TA r = acc;
    if (kLower && a.w) r *= static_cast<const TA*>(a.w)[b * a.w_bs + row];
    if (!kLower && a.add) r += load_acc(static_cast<const TS*>(a.add) + b * a.add_bs + row);
    store_acc(static_cast<TS*>(a.out) + b * a.out_bs + row, r);
  }
}

template <bool kLower>
hipError_t launch(const icr_plan* p, const Level0Args& a, hipStream_t st) {
  const int64_t n = p->n0;
  const void* mat = kLower ? p->l00_c : p->u00_c;
  const int el = p->elem_bytes;
  const int ab = p->precision == ICR_F64 ? 8 : 4;
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    Level0Args c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.in = static_cast<const char*>(a.in) + b0 * a.in_bs * el;
    c.out = static_cast<char*>(a.out) + b0 * a.out_bs * el;
    if (a.w) c.w = static_cast<const char*>(a.w) + b0 * a.w_bs * ab;
    if (a.add) c.add = static_cast<const char*>(a.add) + b0 * a.add_bs * el;
    const dim3 grid(static_cast<unsigned>((n + 3) / 4), static_cast<unsigned>(c.batch));
    switch (p->precision) {
      case ICR_F64:
        level0_kernel<double, kLower><<<grid, 256, 0, st>>>(static_cast<const double*>(mat), n, c);
        break;
      case ICR_F32:
        level0_kernel<float, kLower><<<grid, 256, 0, st>>>(static_cast<const float*>(mat), n, c);
        break;
      default:
        level0_kernel<bf16_t, kLower><<<grid, 256, 0, st>>>(static_cast<const float*>(mat), n, c);
        break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_level0_fwd(const icr_plan* p, const Level0Args& a, hipStream_t st) {
  return launch<true>(p, a, st);
}
hipError_t launch_level0_adj(const icr_plan* p, const Level0Args& a, hipStream_t st) {
  return launch<false>(p, a, st);
}

}  // namespace icr
