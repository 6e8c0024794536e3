// Conjugate gradients on the metric M = L^T W L + 1 (the Fisher metric of a Gaussian
// likelihood plus the identity, the operator MGVI/geoVI sampling solves with CG, section
// "Variational Inference" of NIFTy.re), entirely on the device: per-sample step sizes
// live in device memory, so a run of iterations is enqueued without host round trips.
//
// Per iteration, for every sample independently (x_0 = 0, r_0 = p_0 = b):
//   q = M p;  alpha = (r.r) / (p.q);  x += alpha p;  r -= alpha q;
//   beta = (r'.r') / (r.r);  p = r' + beta p.
// Dot products accumulate in FP64 in a fixed order (per-block partial sums, then one
// block sums the partials), so runs are bitwise reproducible.
#include "icr_internal.h"

namespace icr {
namespace {

constexpr int kDotThreads = 256;
constexpr int kDotBlocks = 256;  // partial sums per sample

struct CgScalars {
  double rr;     // r.r of the current residual
  double alpha;
  double beta;
  double pq;
};

template <typename T>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kDotThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// partial[b][blk] = sum over this block's strided share of a[b] * c[b]
template <typename T>
__global__ void __launch_bounds__(kDotThreads) dot_partial(const T* __restrict__ a, const T* __restrict__ c,
                                                           int64_t n, double* __restrict__ partial) {
  __shared__ double sh[kDotThreads];
  const int64_t b = blockIdx.y;
  const T* pa = a + b * n;
  const T* pc = c + b * n;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; i < n; i += int64_t(kDotBlocks) * kDotThreads)
    acc += static_cast<double>(pa[i]) * static_cast<double>(pc[i]);
  const double s = block_sum<T>(acc, sh);
  if (threadIdx.x == 0) partial[b * kDotBlocks + blockIdx.x] = s;
}

// which = 0: pq = sum, alpha = rr / pq;  which = 1: rr' = sum, beta = rr' / rr, rr = rr'
// (also records sqrt(rr') into norms[b][iter + 1] when norms is given);
// which = 2: rr = sum (initialisation, records norms[b][0]).
__global__ void __launch_bounds__(kDotThreads) dot_finish(const double* __restrict__ partial, CgScalars* sc,
                                                          int which, double* norms, int iter, int stride) {
  __shared__ double sh[kDotThreads];
  const int64_t b = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < kDotBlocks; k += kDotThreads) v += partial[b * kDotBlocks + k];
  const double s = block_sum<double>(v, sh);
  if (threadIdx.x != 0) return;
  CgScalars& c = sc[b];
  if (which == 0) {
    c.pq = s;
    c.alpha = s != 0.0 ? c.rr / s : 0.0;
  } else if (which == 1) {
    c.beta = c.rr != 0.0 ? s / c.rr : 0.0;
    c.rr = s;
    if (norms) norms[b * stride + iter + 1] = sqrt(s);
  } else {
    c.rr = s;
    if (norms) norms[b * stride] = sqrt(s);
  }
}

// x += alpha p; r -= alpha q; partial sums of r.r
template <typename T>
__global__ void __launch_bounds__(kDotThreads) update_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                         const T* __restrict__ q, int64_t n, const CgScalars* sc,
                                                         double* __restrict__ partial) {
  __shared__ double sh[kDotThreads];
  const int64_t b = blockIdx.y;
  const double alpha = sc[b].alpha;
  const T a = static_cast<T>(alpha);
  T* px = x + b * n;
  T* pr = r + b * n;
  const T* pp = p + b * n;
  const T* pq = q + b * n;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; i < n; i += int64_t(kDotBlocks) * kDotThreads) {
    px[i] += a * pp[i];
    const T rn = pr[i] - a * pq[i];
    pr[i] = rn;
    acc += static_cast<double>(rn) * static_cast<double>(rn);
  }
  const double s = block_sum<T>(acc, sh);
  if (threadIdx.x == 0) partial[b * kDotBlocks + blockIdx.x] = s;
}

// p = r + beta p
template <typename T>
__global__ void __launch_bounds__(kDotThreads) update_p(T* __restrict__ p, const T* __restrict__ r, int64_t n,
                                                        const CgScalars* sc) {
  const int64_t b = blockIdx.y;
  const T beta = static_cast<T>(sc[b].beta);
  T* pp = p + b * n;
  const T* pr = r + b * n;
  for (int64_t i = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; i < n; i += int64_t(kDotBlocks) * kDotThreads)
    pp[i] = pr[i] + beta * pp[i];
}

// x = 0, r = p = b, partial sums of b.b
template <typename T>
__global__ void __launch_bounds__(kDotThreads) cg_init(T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                                       const T* __restrict__ bvec, int64_t n,
                                                       double* __restrict__ partial) {
  __shared__ double sh[kDotThreads];
  const int64_t b = blockIdx.y;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; i < n; i += int64_t(kDotBlocks) * kDotThreads) {
    const T v = bvec[b * n + i];
    x[b * n + i] = T(0);
    r[b * n + i] = v;
    p[b * n + i] = v;
    acc += static_cast<double>(v) * static_cast<double>(v);
  }
  const double s = block_sum<T>(acc, sh);
  if (threadIdx.x == 0) partial[b * kDotBlocks + blockIdx.x] = s;
}

}  // namespace

int64_t cg_workspace_bytes(const icr_plan* p, int64_t batch) {
  const int el = p->elem_bytes;
  const int64_t vec = batch * p->n_xi * el;
  auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
  return up(batch * p->n_xi * el)          // metric workspace
         + 3 * up(vec)                     // r, p, q
         + up(batch * kDotBlocks * 8)      // partial sums
         + up(batch * int64_t(sizeof(CgScalars)));
}

hipError_t launch_cg(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* bvec,
                     void* x, int32_t iterations, double* norms, void* workspace, hipStream_t st,
                     hipError_t (*metric)(const icr_plan*, int64_t, const void*, int64_t, const void*, void*,
                                          void*, hipStream_t)) {
  const int el = p->elem_bytes;
  const int64_t n = p->n_xi;
  auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
  char* base = static_cast<char*>(workspace);
  void* mws = base;
  base += up(batch * n * el);
  void* r = base; base += up(batch * n * el);
  void* pv = base; base += up(batch * n * el);
  void* q = base; base += up(batch * n * el);
  double* partial = reinterpret_cast<double*>(base); base += up(batch * kDotBlocks * 8);
  CgScalars* sc = reinterpret_cast<CgScalars*>(base);
  const dim3 grid(kDotBlocks, static_cast<unsigned>(batch));
  const int stride = iterations + 1;
  const bool f64 = p->precision == ICR_F64;
#define AS(T, ptr) static_cast<T*>(ptr)
  if (f64) cg_init<double><<<grid, kDotThreads, 0, st>>>(AS(double, x), AS(double, r), AS(double, pv), static_cast<const double*>(bvec), n, partial);
  else cg_init<float><<<grid, kDotThreads, 0, st>>>(AS(float, x), AS(float, r), AS(float, pv), static_cast<const float*>(bvec), n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dot_finish<<<static_cast<unsigned>(batch), kDotThreads, 0, st>>>(partial, sc, 2, norms, 0, stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int it = 0; it < iterations; ++it) {
    if ((e = metric(p, batch, w, w_bs, pv, q, mws, st)) != hipSuccess) return e;
    if (f64) dot_partial<double><<<grid, kDotThreads, 0, st>>>(AS(double, pv), AS(double, q), n, partial);
    else dot_partial<float><<<grid, kDotThreads, 0, st>>>(AS(float, pv), AS(float, q), n, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    dot_finish<<<static_cast<unsigned>(batch), kDotThreads, 0, st>>>(partial, sc, 0, nullptr, it, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (f64) update_xr<double><<<grid, kDotThreads, 0, st>>>(AS(double, x), AS(double, r), AS(double, pv), AS(double, q), n, sc, partial);
    else update_xr<float><<<grid, kDotThreads, 0, st>>>(AS(float, x), AS(float, r), AS(float, pv), AS(float, q), n, sc, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    dot_finish<<<static_cast<unsigned>(batch), kDotThreads, 0, st>>>(partial, sc, 1, norms, it, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (f64) update_p<double><<<grid, kDotThreads, 0, st>>>(AS(double, pv), AS(double, r), n, sc);
    else update_p<float><<<grid, kDotThreads, 0, st>>>(AS(float, pv), AS(float, r), n, sc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
#undef AS
  return hipSuccess;
}

}  // namespace icr
