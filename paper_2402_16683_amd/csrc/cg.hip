// Conjugate gradients on the metric M = L^T W L + 1 (the Fisher metric of a Gaussian
// likelihood plus the identity, the operator MGVI/geoVI sampling solves with CG, section
// "Variational Inference" of NIFTy.re), entirely on the device: per-sample step sizes
// live in device memory, so a run of iterations is enqueued without host round trips.
//
// Per iteration, for every sample independently (x_0 = 0, r_0 = p_0 = b):
//   q = M p;  alpha = (r.r) / (p.q);  x += alpha p;  r -= alpha q;
//   beta = (r'.r') / (r.r);  p = r' + beta p.
// Dot products accumulate in FP64 in a fixed order (per-block partial sums, then a
// fixed-order sum of the partials), so runs are bitwise reproducible. Each update kernel
// sums the partials it needs itself (every workgroup the same way), so a step is three
// launches after the metric product: p.q partials; x, r and the r.r partials; p. Where the
// metric's finest level runs in the fused 2-D kernel, p.q comes without the first launch:
// p.q = p.(L^T W L p + p) = <L p, w * L p> + p.p, the first sum from that kernel (it sees
// L p and w * L p of the whole finest level), the second from the p update of the
// previous iteration (at the first, p = r: p.p = r.r).
//
// Early stopping by the change of the CG energy E(x) = x.Mx / 2 - b.x (the "absdelta"
// criterion of the sample-drawing CG in the paper's VI example): a step along p with the
// exact line search lowers E by alpha (r.r) / 2, so the decrease needs no extra dot. A
// sample whose step lowered E by less than absdelta keeps that step and is frozen (its x,
// r, p no longer change). Every iteration up to the maximum is enqueued at once; when the
// last sample freezes, a device flag makes the remaining kernels (metric sweeps included)
// return at once, so nothing waits on the host. The p update that raises the flag also
// writes it to a word of pinned host memory, which the host reads (without waiting)
// before it enqueues each iteration: once set, the rest are not enqueued at all.
#include <algorithm>
#include <mutex>
#include <vector>

#include "icr_internal.h"

namespace icr {
namespace {

constexpr int kDotThreads = 256;
constexpr int kDotBlocks = 1024;  // at most this many partial sums per sample
constexpr int kMetricDots = 1024; // partial sums of <L p, w * L p> per sample (fused metric level)

// Per-sample state. r.r and the active flag are kept per iteration parity: the p update
// of iteration i reads the entries of parity i and its workgroup 0 writes those of
// parity i + 1, so no workgroup reads an entry another one writes in the same launch.
struct CgScalars {
  double rr[2];      // r.r at the start of an iteration
  double alpha;      // of the last step taken
  double pq;
  int32_t active[2]; // whether the sample takes the iteration
  int32_t iters;     // steps taken
};

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

// V consecutive elements as one access: 16 bytes when the vectors are aligned (V * sizeof(T)
// == 16), else V = 1. Thread g of a sample handles groups g, g + G, g + 2G, ... of V
// elements (G = blocks x threads), so the partition, and with it every partial sum, is
// fixed by n alone.
template <typename T, int V>
struct Chunk {
  T v[V];
};
template <typename T, int V>
__device__ __forceinline__ Chunk<T, V> ldv(const T* p) {
  Chunk<T, V> c;
  if constexpr (V * sizeof(T) == 16) {
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    __builtin_memcpy(c.v, &u, 16);
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) c.v[k] = p[k];
  }
  return c;
}
template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const Chunk<T, V>& c) {
  if constexpr (V * sizeof(T) == 16) {
    uint4 u;
    __builtin_memcpy(&u, c.v, 16);
    *reinterpret_cast<uint4*>(p) = u;
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) p[k] = c.v[k];
  }
}

// Partial sums per sample: one per workgroup of the vector kernels, which stride over
// the sample's vector with `blocks` workgroups; `blocks` depends on n alone, so the
// partition and every partial sum are fixed by n. At least two workgroups per compute
// unit: on the charted 2-D workload (2.2 M elements) a CG step took 115.5, 96.7, 88.9,
// 86.1 and 86.5 us with 64, 128, 256, 512 and 1024 workgroups.
int dot_blocks(int64_t n, int v) {
  const int64_t b = (n / v + int64_t(kDotThreads) * 4 - 1) / (int64_t(kDotThreads) * 4);
  return static_cast<int>(std::min<int64_t>(kDotBlocks, std::max<int64_t>(512, b)));
}

// The sum of sample b's `count` partials (at partial[b * kStride + k], 1 <= count <=
// kStride) in a fixed order, in every thread (every workgroup that calls it gets the same
// value). Each thread loads all of its kStride / kDotThreads values before adding them (in
// index order): the partials were just written by other compute units, so each load waits
// on memory, and a loop of dependent loads waited once per value.
// load_partials issues the loads, reduce_partials adds them, so a kernel can have other
// loads in flight in the same round.
template <int kStride>
struct Partials {
  double u[kStride / kDotThreads];
};
template <int kStride = kDotBlocks>
__device__ __forceinline__ Partials<kStride> load_partials(const double* __restrict__ partial, int64_t b,
                                                           int count) {
  Partials<kStride> h;
#pragma unroll
  for (int i = 0; i < kStride / kDotThreads; ++i) {
    const int k = threadIdx.x + i * kDotThreads;
    h.u[i] = partial[b * kStride + min(k, count - 1)];  // in bounds; unused past count
  }
  return h;
}
template <int kStride>
__device__ __forceinline__ double reduce_partials(const Partials<kStride>& h, int count, double* sh) {
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < kStride / kDotThreads; ++i) v += threadIdx.x + i * kDotThreads < count ? h.u[i] : 0.0;
  const double s = block_sum(v, sh);
  __syncthreads();  // sh is reused by the caller
  return s;
}
template <int kStride = kDotBlocks>
__device__ __forceinline__ double sum_partials(const double* __restrict__ partial, int64_t b, int count,
                                               double* sh) {
  return reduce_partials(load_partials<kStride>(partial, b, count), count, sh);
}

// The update kernels load a thread's first kPre groups before the step size is known (the
// loads do not depend on it), so they are in flight with the loads of the partial sums
// instead of after them: one memory round for what took three to five. Groups past the
// end are loaded at the last group and left unused. A charted 2-D step (2.2 M elements,
// 537 workgroups) gives every thread four groups.
constexpr int kPre = 4;

// partial[b][blk] = sum over this block's share of a[b] * c[b]
template <typename T, int V>
__global__ void __launch_bounds__(kDotThreads) dot_partial(const T* __restrict__ a, const T* __restrict__ c,
                                                           int64_t n, double* __restrict__ partial,
                                                           const int32_t* halt) {
  __shared__ double sh[kDotThreads];
  if (halted(halt)) return;
  const int64_t b = blockIdx.y;
  const T* pa = a + b * n;
  const T* pc = c + b * n;
  double acc = 0.0;
  const int64_t step = int64_t(gridDim.x) * kDotThreads;
  for (int64_t g = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; g < n / V; g += step) {
    const Chunk<T, V> u = ldv<T, V>(pa + g * V), w = ldv<T, V>(pc + g * V);
#pragma unroll
    for (int k = 0; k < V; ++k) acc += static_cast<double>(u.v[k]) * static_cast<double>(w.v[k]);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[b * kDotBlocks + blockIdx.x] = s;
}

// Iteration with parity `par` of an active sample: p.q from its partials, alpha =
// (r.r) / (p.q); x += alpha p; r -= alpha q; partial sums of the new r.r. Workgroup 0
// records p.q and alpha for the p update. kSplit: p.q = <L p, w * L p> (npq partials of
// stride kMetricDots) + p.p (the p update's partials, or r.r when `first`).
template <typename T, int V, bool kSplit>
__global__ void __launch_bounds__(kDotThreads) update_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                         const T* __restrict__ q, int64_t n, CgScalars* sc,
                                                         const double* __restrict__ pq_partial, int npq,
                                                         const double* __restrict__ pp_partial, int first,
                                                         double* __restrict__ rr_partial, int par,
                                                         const int32_t* halt) {
  __shared__ double sh[kDotThreads];
  if (halted(halt)) return;
  const int64_t b = blockIdx.y;
  if (!sc[b].active[par]) return;  // uniform per workgroup (one sample per grid row)
  T* px = x + b * n;
  T* pr = r + b * n;
  const T* pp = p + b * n;
  const T* pqv = q + b * n;
  const int64_t ng = n / V;
  const int64_t step = int64_t(gridDim.x) * kDotThreads;
  const int64_t g0 = int64_t(blockIdx.x) * kDotThreads + threadIdx.x;
  Chunk<T, V> xv[kPre], rv[kPre], pv[kPre], qv[kPre];
#pragma unroll
  for (int j = 0; j < kPre; ++j) {
    const int64_t g = min(g0 + j * step, ng - 1) * V;
    xv[j] = ldv<T, V>(px + g);
    rv[j] = ldv<T, V>(pr + g);
    pv[j] = ldv<T, V>(pp + g);
    qv[j] = ldv<T, V>(pqv + g);
  }
  const double rr = sc[b].rr[par];
  double pq;
  if constexpr (kSplit) {
    const auto hl = load_partials<kMetricDots>(pq_partial, b, npq);
    const auto hp = load_partials(pp_partial, b, first ? 1 : gridDim.x);  // unused at the first
    const double lik = reduce_partials(hl, npq, sh);
    pq = lik + (first ? rr : reduce_partials(hp, gridDim.x, sh));
  } else {
    pq = sum_partials(pq_partial, b, gridDim.x, sh);
  }
  const double alpha = pq != 0.0 ? rr / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[b].pq = pq;
    sc[b].alpha = alpha;
  }
  const T a = static_cast<T>(alpha);
  double acc = 0.0;
  auto update = [&](Chunk<T, V>& xc, Chunk<T, V>& rc, const Chunk<T, V>& pc, const Chunk<T, V>& qc, int64_t g) {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      xc.v[k] += a * pc.v[k];
      rc.v[k] = rc.v[k] - a * qc.v[k];
      acc += static_cast<double>(rc.v[k]) * static_cast<double>(rc.v[k]);
    }
    stv<T, V>(px + g * V, xc);
    stv<T, V>(pr + g * V, rc);
  };
#pragma unroll
  for (int j = 0; j < kPre; ++j)
    if (g0 + j * step < ng) update(xv[j], rv[j], pv[j], qv[j], g0 + j * step);
  for (int64_t g = g0 + kPre * step; g < ng; g += step) {
    Chunk<T, V> xc = ldv<T, V>(px + g * V), rc = ldv<T, V>(pr + g * V);
    update(xc, rc, ldv<T, V>(pp + g * V), ldv<T, V>(pqv + g * V), g);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) rr_partial[b * kDotBlocks + blockIdx.x] = s;
}

// End of iteration `iter` (parity par): the new r.r from its partials, beta = r'.r' / r.r,
// and p = r + beta p. The sample stops when its step lowered the energy by less than
// absdelta (absdelta > 0) or r = 0; its step is kept and p is no longer needed.
// Workgroup 0 writes the sample's entries of the next parity, counts the step, records
// the residual norm (a stopped sample repeats its last one), and when the last active
// sample stops raises the halt flag (halt[1] counts the active samples). kPP: also the
// partial sums of the new p.p.
template <typename T, int V, bool kPP>
__global__ void __launch_bounds__(kDotThreads) update_p(T* __restrict__ p, const T* __restrict__ r, int64_t n,
                                                        CgScalars* sc, const double* __restrict__ rr_partial, int par,
                                                        int iter, double absdelta, double* norms, int stride,
                                                        int32_t* halt, int32_t* host_halt,
                                                        double* __restrict__ pp_partial) {
  __shared__ double sh[kDotThreads];
  if (halted(halt)) return;
  const int64_t b = blockIdx.y;
  const int nx = par ^ 1;
  CgScalars& c = sc[b];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (!c.active[par]) {
    if (lead) {
      c.active[nx] = 0;
      c.rr[nx] = c.rr[par];
      if (norms) norms[b * stride + iter + 1] = sqrt(c.rr[par]);
    }
    return;
  }
  T* pp = p + b * n;
  const T* pr = r + b * n;
  const int64_t ng = n / V;
  const int64_t step = int64_t(gridDim.x) * kDotThreads;
  const int64_t g0 = int64_t(blockIdx.x) * kDotThreads + threadIdx.x;
  Chunk<T, V> pv[kPre], rv[kPre];
#pragma unroll
  for (int j = 0; j < kPre; ++j) {
    const int64_t g = min(g0 + j * step, ng - 1) * V;
    pv[j] = ldv<T, V>(pp + g);
    rv[j] = ldv<T, V>(pr + g);
  }
  const double rr_new = sum_partials(rr_partial, b, gridDim.x, sh);
  const double rr = c.rr[par];
  const double beta = rr != 0.0 ? rr_new / rr : 0.0;
  const double decrease = 0.5 * c.alpha * rr;
  const bool stop = rr_new == 0.0 || (absdelta > 0.0 && !(decrease >= absdelta));
  if (lead) {
    c.rr[nx] = rr_new;
    c.active[nx] = stop ? 0 : 1;
    c.iters += 1;
    if (norms) norms[b * stride + iter + 1] = sqrt(rr_new);
    if (stop && halt && atomicSub(&halt[1], 1) == 1) {
      halt[0] = 1;
      if (host_halt) __hip_atomic_store(host_halt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  if (stop) return;
  const T bt = static_cast<T>(beta);
  double acc = 0.0;
  auto update = [&](Chunk<T, V>& pc, const Chunk<T, V>& rc, int64_t g) {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      pc.v[k] = rc.v[k] + bt * pc.v[k];
      if constexpr (kPP) acc += static_cast<double>(pc.v[k]) * static_cast<double>(pc.v[k]);
    }
    stv<T, V>(pp + g * V, pc);
  };
#pragma unroll
  for (int j = 0; j < kPre; ++j)
    if (g0 + j * step < ng) update(pv[j], rv[j], g0 + j * step);
  for (int64_t g = g0 + kPre * step; g < ng; g += step) {
    Chunk<T, V> pc = ldv<T, V>(pp + g * V);
    update(pc, ldv<T, V>(pr + g * V), g);
  }
  if constexpr (kPP) {
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) pp_partial[b * kDotBlocks + blockIdx.x] = s;
  }
}

// x = 0, r = p = b, partial sums of b.b; clears the halt flag and the active count
template <typename T, int V>
__global__ void __launch_bounds__(kDotThreads) cg_init(T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                                       const T* __restrict__ bvec, int64_t n,
                                                       double* __restrict__ partial, int32_t* halt) {
  __shared__ double sh[kDotThreads];
  const int64_t b = blockIdx.y;
  if (halt && blockIdx.x == 0 && b == 0 && threadIdx.x == 0) {
    halt[0] = 0;
    halt[1] = 0;
  }
  double acc = 0.0;
  Chunk<T, V> zero;
#pragma unroll
  for (int k = 0; k < V; ++k) zero.v[k] = T(0);
  const int64_t step = int64_t(gridDim.x) * kDotThreads;
  for (int64_t g = int64_t(blockIdx.x) * kDotThreads + threadIdx.x; g < n / V; g += step) {
    const Chunk<T, V> v = ldv<T, V>(bvec + b * n + g * V);
    stv<T, V>(x + b * n + g * V, zero);
    stv<T, V>(r + b * n + g * V, v);
    stv<T, V>(p + b * n + g * V, v);
#pragma unroll
    for (int k = 0; k < V; ++k) acc += static_cast<double>(v.v[k]) * static_cast<double>(v.v[k]);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[b * kDotBlocks + blockIdx.x] = s;
}

// r.r of the start (one workgroup per sample): a sample with b = 0 takes no step; the
// others are counted in halt[1]
__global__ void __launch_bounds__(kDotThreads) cg_start(const double* __restrict__ partial, CgScalars* sc,
                                                        double* norms, int stride, int blocks, int32_t* halt) {
  __shared__ double sh[kDotThreads];
  const int64_t b = blockIdx.x;
  const double s = sum_partials(partial, b, blocks, sh);
  if (threadIdx.x != 0) return;
  CgScalars& c = sc[b];
  c.rr[0] = c.rr[1] = s;
  c.active[0] = s != 0.0 ? 1 : 0;
  c.active[1] = 0;
  c.alpha = c.pq = 0.0;
  c.iters = 0;
  if (norms) norms[b * stride] = sqrt(s);
  if (halt && c.active[0]) atomicAdd(&halt[1], 1);
}

// norms[b][k] for k past the steps sample b took: its last residual norm
__global__ void cg_fill_norms(const CgScalars* sc, double* norms, int stride) {
  const int64_t b = blockIdx.x;
  const int taken = sc[b].iters;
  const double last = sqrt(sc[b].rr[taken & 1]);
  for (int k = taken + 1 + threadIdx.x; k < stride; k += blockDim.x) norms[b * stride + k] = last;
}

// iterations_done[b] = steps sample b took
__global__ void cg_report(const CgScalars* sc, int32_t* iterations_done, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) iterations_done[b] = sc[b].iters;
}

// Pinned host words the p update raises with the halt flag, one per CG call in flight. A
// word returns to the pool when its call's work is done (its event has fired), so a late
// write from an earlier call never stops a later one.
struct HostHalt {
  int device = -1;
  int32_t* word = nullptr;      // host address
  int32_t* dev_word = nullptr;  // the same word as the device addresses it
  hipEvent_t done = nullptr;    // recorded after the call's last kernel
  bool in_use = false;
};
std::mutex g_halt_mu;
std::vector<HostHalt*> g_halt_pool;

HostHalt* acquire_host_halt(int device) {
  std::lock_guard<std::mutex> lk(g_halt_mu);
  for (HostHalt* h : g_halt_pool)
    if (!h->in_use && h->device == device && hipEventQuery(h->done) == hipSuccess) {
      h->in_use = true;
      *h->word = 0;
      return h;
    }
  HostHalt* h = new HostHalt;
  h->device = device;
  void* w = nullptr;
  if (hipHostMalloc(&w, 64, hipHostMallocCoherent) != hipSuccess) {
    delete h;
    return nullptr;  // the call then runs without the host watch
  }
  h->word = static_cast<int32_t*>(w);
  void* dw = nullptr;
  if (hipHostGetDevicePointer(&dw, w, 0) != hipSuccess ||
      hipEventCreateWithFlags(&h->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(w);
    delete h;
    return nullptr;
  }
  h->dev_word = static_cast<int32_t*>(dw);
  *h->word = 0;
  h->in_use = true;
  g_halt_pool.push_back(h);
  return h;
}

void release_host_halt(HostHalt* h, hipStream_t st) {
  const bool recorded = hipEventRecord(h->done, st) == hipSuccess;
  std::lock_guard<std::mutex> lk(g_halt_mu);
  // reusable once the event fires; if it could not be recorded, never (a word whose
  // call may still be running must not be handed out)
  h->in_use = !recorded;
}

// Releases a call's host word on every return path.
struct HostHaltGuard {
  HostHalt* h;
  hipStream_t st;
  ~HostHaltGuard() {
    if (h) release_host_halt(h, st);
  }
};

template <typename T, int V>
hipError_t run_cg(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* bvec, void* x,
                  int32_t iterations, double absdelta, int32_t* iterations_done, double* norms, void* mws, T* r,
                  T* pv, T* q, double* pq_partial, double* rr_partial, double* lik_partial, double* pp_partial,
                  CgScalars* sc, int32_t* halt_flag, hipStream_t st, MetricFn metric) {
  const int64_t n = p->n_xi;
  const int blocks = dot_blocks(n, V);
  const dim3 grid(static_cast<unsigned>(blocks), static_cast<unsigned>(batch));
  const int stride = iterations + 1;
  const int nb = static_cast<int>(batch);
  // the halt flag only with early stopping: fixed-count runs pay nothing for it
  int32_t* halt = absdelta > 0.0 ? halt_flag : nullptr;
  int dev = 0;
  HostHalt* hh = halt && hipGetDevice(&dev) == hipSuccess ? acquire_host_halt(dev) : nullptr;
  const HostHaltGuard guard{hh, st};
  int32_t* host_halt = hh ? hh->dev_word : nullptr;
  T* xv = static_cast<T*>(x);
  cg_init<T, V><<<grid, kDotThreads, 0, st>>>(xv, r, pv, static_cast<const T*>(bvec), n, rr_partial, halt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  cg_start<<<static_cast<unsigned>(batch), kDotThreads, 0, st>>>(rr_partial, sc, norms, stride, blocks, halt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  bool pp_ready = true;  // p.p is known for the current p (r.r at the start)
  for (int it = 0; it < iterations; ++it) {
    // every sample has stopped: the remaining iterations would do nothing
    if (hh && __atomic_load_n(hh->word, __ATOMIC_ACQUIRE) != 0) break;
    const int par = it & 1;
    int nlik = 0;
    if ((e = metric(p, batch, w, w_bs, pv, q, mws, halt, st, lik_partial, kMetricDots, &nlik)) != hipSuccess)
      return e;
    const bool split = nlik > 0 && pp_ready;
    if (split) {
      update_xr<T, V, true><<<grid, kDotThreads, 0, st>>>(xv, r, pv, q, n, sc, lik_partial, nlik, pp_partial,
                                                          it == 0, rr_partial, par, halt);
    } else {
      dot_partial<T, V><<<grid, kDotThreads, 0, st>>>(pv, q, n, pq_partial, halt);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      update_xr<T, V, false><<<grid, kDotThreads, 0, st>>>(xv, r, pv, q, n, sc, pq_partial, 0, nullptr, 0,
                                                           rr_partial, par, halt);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the next iteration can split p.q only if this p update sums p.p
    if (nlik > 0)
      update_p<T, V, true><<<grid, kDotThreads, 0, st>>>(pv, r, n, sc, rr_partial, par, it, absdelta, norms, stride,
                                                         halt, host_halt, pp_partial);
    else
      update_p<T, V, false><<<grid, kDotThreads, 0, st>>>(pv, r, n, sc, rr_partial, par, it, absdelta, norms, stride,
                                                          halt, host_halt, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    pp_ready = nlik > 0;
  }
  if (halt && norms) {
    // the iterations after the halt wrote nothing: repeat each sample's last norm there
    cg_fill_norms<<<static_cast<unsigned>(batch), 64, 0, st>>>(sc, norms, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (iterations_done) {
    cg_report<<<static_cast<unsigned>((batch + 63) / 64), 64, 0, st>>>(sc, iterations_done, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; }


}  // namespace

int64_t cg_workspace_bytes(const icr_plan* p, int64_t batch) {
  const int el = p->elem_bytes;
  const int64_t vec = batch * p->n_xi * el;
  auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
  return up(batch * p->n_xi * el)          // metric workspace
         + 3 * up(vec)                     // r, p, q
         + 3 * up(batch * kDotBlocks * 8)  // partial sums of p.q, r.r and p.p
         + up(batch * kMetricDots * 8)     // partial sums of <L p, w * L p>
         + up(batch * int64_t(sizeof(CgScalars)))
         + 256;                            // halt flag and active count
}

hipError_t launch_cg(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* bvec,
                     void* x, int32_t iterations, double absdelta, int32_t* iterations_done, double* norms,
                     void* workspace, hipStream_t st, MetricFn metric) {
  const int el = p->elem_bytes;
  const int64_t n = p->n_xi;
  auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
  char* base = static_cast<char*>(workspace);
  void* mws = base;
  base += up(batch * n * el);
  void* r = base; base += up(batch * n * el);
  void* pv = base; base += up(batch * n * el);
  void* q = base; base += up(batch * n * el);
  double* pq_partial = reinterpret_cast<double*>(base); base += up(batch * kDotBlocks * 8);
  double* rr_partial = reinterpret_cast<double*>(base); base += up(batch * kDotBlocks * 8);
  double* pp_partial = reinterpret_cast<double*>(base); base += up(batch * kDotBlocks * 8);
  double* lik_partial = reinterpret_cast<double*>(base); base += up(batch * kMetricDots * 8);
  CgScalars* sc = reinterpret_cast<CgScalars*>(base);
  base += up(batch * int64_t(sizeof(CgScalars)));
  int32_t* halt = reinterpret_cast<int32_t*>(base);
  // 16-byte accesses when every sample's vector starts 16-byte aligned (the workspace
  // vectors are 256-byte aligned; x and b are the caller's)
  const int v16 = 16 / el;
  const bool vec = n % v16 == 0 && aligned16(x) && aligned16(bvec) && aligned16(workspace);
  if (p->precision == ICR_F64) {
    return vec ? run_cg<double, 2>(p, batch, w, w_bs, bvec, x, iterations, absdelta, iterations_done, norms, mws,
                                   static_cast<double*>(r), static_cast<double*>(pv), static_cast<double*>(q),
                                   pq_partial, rr_partial, lik_partial, pp_partial, sc, halt, st, metric)
               : run_cg<double, 1>(p, batch, w, w_bs, bvec, x, iterations, absdelta, iterations_done, norms, mws,
                                   static_cast<double*>(r), static_cast<double*>(pv), static_cast<double*>(q),
                                   pq_partial, rr_partial, lik_partial, pp_partial, sc, halt, st, metric);
  }
  return vec ? run_cg<float, 4>(p, batch, w, w_bs, bvec, x, iterations, absdelta, iterations_done, norms, mws,
                                static_cast<float*>(r), static_cast<float*>(pv), static_cast<float*>(q), pq_partial,
                                rr_partial, lik_partial, pp_partial, sc, halt, st, metric)
             : run_cg<float, 1>(p, batch, w, w_bs, bvec, x, iterations, absdelta, iterations_done, norms, mws,
                                static_cast<float*>(r), static_cast<float*>(pv), static_cast<float*>(q), pq_partial,
                                rr_partial, lik_partial, pp_partial, sc, halt, st, metric);
}

}  // namespace icr
