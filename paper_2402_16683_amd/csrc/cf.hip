// Correlated-field model on an n x n periodic grid and the Fisher metric of a Poisson
// likelihood (NIFTy.re, section "Gaussian Processes": s = FT(sqrt(P) xi); section
// "Performance of NIFTy.re compared to NIFTy": M_p = J^T N^-1 J + 1).
//
// The field is real, so FT is the 2-D Hartley transform, normalised to be its own
// inverse: T x = (Re - Im)(FFT2 x) / n. With lambda = exp(m + T(A xi)) the Jacobian is
// J = diag(lambda) T diag(A) and N^-1 = diag(1 / lambda), so
//   M_p v = v + A T(lambda(p) T(A v)).
// A transform is four passes over the grid, each a hand-written kernel, on real data
// (the separable Hartley transform S = H_rows H_cols and the identity cas(a + b) =
// (cas a cas b + cas(-a) cas b + cas a cas(-b) - cas(-a) cas(-b)) / 2 give T from S):
//   1. 1-D Hartley transforms of the (pre-multiplied) rows, two rows per workgroup as one
//      complex Stockham FFT (radix 4) in LDS;
//   2. a tiled transpose;
//   3. the same on the rows of the transpose (the column transforms), paired as (l, -l)
//      so each workgroup forms T for both from S[., l] and S[., -l];
//   4. a tiled transpose back with the post-operation (x lambda, exp(m + .), or v + A .),
//      so the elementwise work rides on the passes.
// FP32 throughout; twiddles from sincospif on the reduced angle.
#include <cmath>
#include <new>
#include <string>

#include "icr_cf.h"
#include "icr_internal.h"

struct icr_cf_plan {
  int n = 0;
  int logn = 0;
  double mean = 0.0;
  float* amp = nullptr;  // device [n][n] amplitude spectrum
};

namespace icr {
namespace {

constexpr int kTile = 32;

constexpr int kFftThreads = 512;
constexpr int kFftIt = 2;  // radix-4 butterflies per thread and stage: n / 4 <= kFftIt * kFftThreads

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place FFT of n complex values in LDS, Stockham autosort (natural order in and out):
// radix-4 stages, then one radix-2 stage when log2(n) is odd. A stage of span ns reads the
// r-th quarter at j + r n/4, twiddles it by exp(-2 pi i r (j mod ns) / (4 ns)), takes the
// 4-point DFT and writes it to (j / ns) 4 ns + (j mod ns) + r ns; all reads of a stage
// finish (barrier) before its writes. Called by the whole workgroup; ends with a barrier.
__device__ void lds_fft(float2* buf, int n, int logn) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int q4 = n >> 2;
  int ns = 1, lns = 0;
  for (; lns + 2 <= logn; ns <<= 2, lns += 2) {  // while 4 ns <= n
    float2 v[kFftIt][4];
#pragma unroll
    for (int it = 0; it < kFftIt; ++it) {
      const int j = tid + it * nt;
      if (j < q4) {
        const int k = j & (ns - 1);
        float sn, cs;
        sincospif(-2.0f * static_cast<float>(k) / static_cast<float>(4 * ns), &sn, &cs);
        const float2 w1 = make_float2(cs, sn), w2 = cmul(w1, w1), w3 = cmul(w2, w1);
        const float2 a = buf[j], b = cmul(buf[j + q4], w1), c = cmul(buf[j + 2 * q4], w2),
                     d = cmul(buf[j + 3 * q4], w3);
        const float2 t0 = make_float2(a.x + c.x, a.y + c.y), t1 = make_float2(a.x - c.x, a.y - c.y);
        const float2 t2 = make_float2(b.x + d.x, b.y + d.y), t3 = make_float2(b.x - d.x, b.y - d.y);
        v[it][0] = make_float2(t0.x + t2.x, t0.y + t2.y);
        v[it][1] = make_float2(t1.x + t3.y, t1.y - t3.x);  // t1 - i t3
        v[it][2] = make_float2(t0.x - t2.x, t0.y - t2.y);
        v[it][3] = make_float2(t1.x - t3.y, t1.y + t3.x);  // t1 + i t3
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kFftIt; ++it) {
      const int j = tid + it * nt;
      if (j < q4) {
        const int base = ((j >> lns) << (lns + 2)) + (j & (ns - 1));
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[base + r * ns] = v[it][r];
      }
    }
    __syncthreads();
  }
  if (ns < n) {  // the last stage is radix 2 (ns = n / 2)
    const int q2 = n >> 1;
    float2 v[2 * kFftIt][2];
#pragma unroll
    for (int it = 0; it < 2 * kFftIt; ++it) {
      const int j = tid + it * nt;
      if (j < q2) {
        float sn, cs;
        sincospif(-static_cast<float>(j & (ns - 1)) / static_cast<float>(ns), &sn, &cs);
        const float2 a = buf[j], b = cmul(buf[j + q2], make_float2(cs, sn));
        v[it][0] = make_float2(a.x + b.x, a.y + b.y);
        v[it][1] = make_float2(a.x - b.x, a.y - b.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2 * kFftIt; ++it) {
      const int j = tid + it * nt;
      if (j < q2) {
        const int base = ((j >> lns) << (lns + 1)) + (j & (ns - 1));
        buf[base] = v[it][0];
        buf[base + ns] = v[it][1];
      }
    }
    __syncthreads();
  }
}

constexpr int kDhtPer = 8;  // k values per thread in the post-processing (n / threads <= 8)

// 1-D Hartley transforms (unnormalised, (Re - Im) of the DFT) of two real rows a, b at
// once: the FFT of z = row_a + i row_b gives, with u = Z[-k], H_a[k] = (Z.x + u.x - Z.y +
// u.y) / 2 and H_b[k] = (Z.y + u.y + Z.x - u.x) / 2. Pass 1 (kCombine false) takes the
// row pairs (2w, 2w+1) of the pre-multiplied input and writes both transforms. Pass 3
// (kCombine true) takes the rows (w, n-w) (w = 0: rows 0 and n/2) of the transposed
// first-pass result, i.e. the column transforms S[., l] and S[., -l] of the separable
// transform, and writes the 2-D Hartley transform from them,
//   T[k][l] = (S[k][l] + S[-k][l] + S[k][-l] - S[-k][-l]) / 2   (cas(a + b) identity),
// scaled by 1/n, still transposed (out row l holds T[.][l]).
template <bool kCombine>
__global__ void __launch_bounds__(kFftThreads) cf_dht_rows(const float* __restrict__ in, const float* __restrict__ pre,
                                                           float* __restrict__ out, int n, int logn, float scale) {
  extern __shared__ float2 buf[];
  const int w = blockIdx.x;
  const int ra = kCombine ? w : 2 * w;
  const int rb = kCombine ? (w == 0 ? n / 2 : n - w) : 2 * w + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  const float* xa = in + int64_t(ra) * n;
  const float* xb = in + int64_t(rb) * n;
  for (int i = tid; i < n; i += nt) {
    float a = xa[i], b = xb[i];
    if (pre) {
      a *= pre[int64_t(ra) * n + i];
      b *= pre[int64_t(rb) * n + i];
    }
    buf[i] = make_float2(a, b);
  }
  __syncthreads();
  lds_fft(buf, n, logn);
  float ha[kDhtPer], hb[kDhtPer];
#pragma unroll
  for (int it = 0; it < kDhtPer; ++it) {
    const int k = tid + it * nt;
    if (k < n) {
      const float2 z = buf[k], u = buf[(n - k) & (n - 1)];
      ha[it] = 0.5f * (z.x + u.x - z.y + u.y);
      hb[it] = 0.5f * (z.y + u.y + z.x - u.x);
    }
  }
  float* oa = out + int64_t(ra) * n;
  float* ob = out + int64_t(rb) * n;
  if (!kCombine) {
#pragma unroll
    for (int it = 0; it < kDhtPer; ++it) {
      const int k = tid + it * nt;
      if (k < n) {
        oa[k] = ha[it];
        ob[k] = hb[it];
      }
    }
    return;
  }
  __syncthreads();  // every thread has read the spectrum: reuse the LDS for H_a, H_b
  float* hs = reinterpret_cast<float*>(buf);
#pragma unroll
  for (int it = 0; it < kDhtPer; ++it) {
    const int k = tid + it * nt;
    if (k < n) {
      hs[k] = ha[it];
      hs[n + k] = hb[it];
    }
  }
  __syncthreads();
  const float half = 0.5f * scale;
#pragma unroll
  for (int it = 0; it < kDhtPer; ++it) {
    const int k = tid + it * nt;
    if (k < n) {
      const int nk = (n - k) & (n - 1);
      if (w == 0) {  // rows 0 and n/2 are their own reflections
        oa[k] = ha[it] * scale;
        ob[k] = hb[it] * scale;
      } else {
        oa[k] = half * (ha[it] + hs[nk] + hb[it] - hs[n + nk]);
        ob[k] = half * (hb[it] + hs[n + nk] + ha[it] - hs[nk]);
      }
    }
  }
}

__global__ void __launch_bounds__(kTile * 8) cf_transpose(const float* __restrict__ in, float* __restrict__ out,
                                                          int n) {
  __shared__ float tile[kTile][kTile + 1];
  const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int k = 0; k < kTile; k += 8) tile[ty + k][tx] = in[int64_t(by + ty + k) * n + bx + tx];
  __syncthreads();
  for (int k = 0; k < kTile; k += 8) out[int64_t(bx + ty + k) * n + by + tx] = tile[tx][ty + k];
}

enum Post { kPostNone = 0, kPostMul = 1, kPostExp = 2, kPostMetric = 3 };

// out = post(Tt^T): the transpose back of pass 3's result with the operator's elementwise
// step (x lambda, exp(m + .), or v + A .).
template <int kPost>
__global__ void __launch_bounds__(kTile * 8) cf_finish(const float* __restrict__ tt, float* __restrict__ out,
                                                       const float* __restrict__ v1, const float* __restrict__ v2,
                                                       float mean, int n) {
  __shared__ float tile[kTile][kTile + 1];
  const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int k = 0; k < kTile; k += 8) tile[ty + k][tx] = tt[int64_t(by + ty + k) * n + bx + tx];
  __syncthreads();
  for (int k = 0; k < kTile; k += 8) {
    const int64_t idx = int64_t(bx + ty + k) * n + by + tx;
    const float t = tile[tx][ty + k];
    float r;
    if (kPost == kPostMul) r = t * v1[idx];
    else if (kPost == kPostExp) r = expf(mean + t);
    else if (kPost == kPostMetric) r = v1[idx] + v2[idx] * t;
    else r = t;
    out[idx] = r;
  }
}

__global__ void cf_amplitude_kernel(float* __restrict__ amp, int n, double a, double a0, double length, double slope) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(n) * n) return;
  const int i = static_cast<int>(t / n), j = static_cast<int>(t % n);
  const double ki = i < n - i ? i : n - i, kj = j < n - j ? j : n - j;
  const double k2 = (ki * ki + kj * kj) * length * length;
  amp[t] = t == 0 ? static_cast<float>(a0) : static_cast<float>(a * pow(1.0 + k2, -slope / 4.0));
}

// out = post(T(pre * x)); work: two real n x n buffers.
hipError_t transform(const icr_cf_plan* p, const float* x, const float* pre, float* out, int post, const float* v1,
                     const float* v2, float* work, hipStream_t st) {
  const int n = p->n;
  float* r1 = work;
  float* r2 = work + int64_t(n) * n;
  const unsigned pairs = static_cast<unsigned>(n / 2);
  // n / 4 radix-4 butterflies per stage over at most kFftIt per thread (n <= 4096)
  const unsigned threads = static_cast<unsigned>(n / 4 < kFftThreads ? (n / 4 < 64 ? 64 : n / 4) : kFftThreads);
  const size_t lds = sizeof(float2) * n;
  const dim3 tgrid(n / kTile, n / kTile), tblock(kTile, 8);
  cf_dht_rows<false><<<pairs, threads, lds, st>>>(x, pre, r1, n, p->logn, 1.0f);
  cf_transpose<<<tgrid, tblock, 0, st>>>(r1, r2, n);
  cf_dht_rows<true><<<pairs, threads, lds, st>>>(r2, nullptr, r1, n, p->logn, 1.0f / static_cast<float>(n));
  const float mean = static_cast<float>(p->mean);
  switch (post) {
    case kPostMul: cf_finish<kPostMul><<<tgrid, tblock, 0, st>>>(r1, out, v1, v2, mean, n); break;
    case kPostExp: cf_finish<kPostExp><<<tgrid, tblock, 0, st>>>(r1, out, v1, v2, mean, n); break;
    case kPostMetric: cf_finish<kPostMetric><<<tgrid, tblock, 0, st>>>(r1, out, v1, v2, mean, n); break;
    default: cf_finish<kPostNone><<<tgrid, tblock, 0, st>>>(r1, out, v1, v2, mean, n); break;
  }
  return hipGetLastError();
}

icr_status cf_fail(icr_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

bool cf_aligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) % 4) == 0; }

}  // namespace
}  // namespace icr

extern "C" {

icr_status icr_cf_create(int32_t n, double amplitude, double zero_mode, double length, double slope,
                         double offset_mean, void* hip_stream, icr_cf_plan** out_plan) {
  icr::clear_error();
  if (!out_plan) return icr::cf_fail(ICR_ERR_INVALID_ARG, "out_plan is NULL");
  *out_plan = nullptr;
  if (n < 32 || n > 4096 || (n & (n - 1)) != 0)
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "n must be a power of two in [32, 4096]");
  if (!(amplitude > 0.0) || !(zero_mode >= 0.0) || !(length >= 0.0) || !std::isfinite(slope) ||
      !std::isfinite(offset_mean) || !std::isfinite(amplitude) || !std::isfinite(zero_mode) || !std::isfinite(length))
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "amplitude > 0, zero_mode >= 0, length >= 0, finite slope and mean");
  icr_cf_plan* p = new (std::nothrow) icr_cf_plan;
  if (!p) return icr::cf_fail(ICR_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->n = n;
  while ((1 << p->logn) < n) ++p->logn;
  p->mean = offset_mean;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipMalloc(&p->amp, sizeof(float) * size_t(n) * n);
  if (e == hipSuccess) {
    const int64_t total = int64_t(n) * n;
    icr::cf_amplitude_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, st>>>(p->amp, n, amplitude,
                                                                                        zero_mode, length, slope);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) {
    if (p->amp) (void)hipFree(p->amp);
    delete p;
    return icr::cf_fail(e == hipErrorOutOfMemory ? ICR_ERR_OUT_OF_MEMORY : ICR_ERR_HIP,
                        std::string("correlated-field plan: ") + hipGetErrorString(e));
  }
  *out_plan = p;
  return ICR_OK;
}

icr_status icr_cf_workspace_bytes(const icr_cf_plan* p, int64_t* bytes) {
  icr::clear_error();
  if (!p || !bytes) return icr::cf_fail(ICR_ERR_INVALID_ARG, "plan or bytes is NULL");
  *bytes = int64_t(p->n) * p->n * 3 * int64_t(sizeof(float));
  return ICR_OK;
}

icr_status icr_cf_copy_amplitude(const icr_cf_plan* p, float* amp) {
  icr::clear_error();
  if (!p || !amp) return icr::cf_fail(ICR_ERR_INVALID_ARG, "plan or amp is NULL");
  const hipError_t e = hipMemcpy(amp, p->amp, sizeof(float) * size_t(p->n) * p->n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return icr::cf_fail(ICR_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  return ICR_OK;
}

icr_status icr_cf_transform(const icr_cf_plan* p, const float* x, float* y, void* workspace, void* hip_stream) {
  icr::clear_error();
  if (!p || !x || !y || !workspace) return icr::cf_fail(ICR_ERR_INVALID_ARG, "NULL argument");
  if (!icr::cf_aligned(x) || !icr::cf_aligned(y) || (reinterpret_cast<uintptr_t>(workspace) % 8) != 0)
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "buffer not aligned");
  const hipError_t e = icr::transform(p, x, nullptr, y, icr::kPostNone, nullptr, nullptr,
                                      static_cast<float*>(workspace), static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return icr::cf_fail(ICR_ERR_HIP, std::string("transform: ") + hipGetErrorString(e));
  return ICR_OK;
}

icr_status icr_cf_rate(const icr_cf_plan* p, const float* position, float* lambda, void* workspace,
                       void* hip_stream) {
  icr::clear_error();
  if (!p || !position || !lambda || !workspace) return icr::cf_fail(ICR_ERR_INVALID_ARG, "NULL argument");
  if (!icr::cf_aligned(position) || !icr::cf_aligned(lambda) || (reinterpret_cast<uintptr_t>(workspace) % 8) != 0)
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "buffer not aligned");
  const hipError_t e = icr::transform(p, position, p->amp, lambda, icr::kPostExp, nullptr, nullptr,
                                      static_cast<float*>(workspace), static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return icr::cf_fail(ICR_ERR_HIP, std::string("rate: ") + hipGetErrorString(e));
  return ICR_OK;
}

icr_status icr_cf_metric_apply(const icr_cf_plan* p, const float* lambda, const float* v, float* out,
                               void* workspace, void* hip_stream) {
  icr::clear_error();
  if (!p || !lambda || !v || !out || !workspace) return icr::cf_fail(ICR_ERR_INVALID_ARG, "NULL argument");
  if (!icr::cf_aligned(lambda) || !icr::cf_aligned(v) || !icr::cf_aligned(out) ||
      (reinterpret_cast<uintptr_t>(workspace) % 8) != 0)
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "buffer not aligned");
  if (v == out) return icr::cf_fail(ICR_ERR_INVALID_ARG, "v and out must differ");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  float* work = static_cast<float*>(workspace);
  float* u = work + 2 * int64_t(p->n) * p->n;
  // u = lambda * T(A v); out = v + A * T(u)
  hipError_t e = icr::transform(p, v, p->amp, u, icr::kPostMul, lambda, nullptr, work, st);
  if (e == hipSuccess) e = icr::transform(p, u, nullptr, out, icr::kPostMetric, v, p->amp, work, st);
  if (e != hipSuccess) return icr::cf_fail(ICR_ERR_HIP, std::string("metric: ") + hipGetErrorString(e));
  return ICR_OK;
}

icr_status icr_cf_destroy(icr_cf_plan* p) {
  icr::clear_error();
  if (!p) return ICR_OK;
  if (p->amp) (void)hipFree(p->amp);
  delete p;
  return ICR_OK;
}

}  // extern "C"
