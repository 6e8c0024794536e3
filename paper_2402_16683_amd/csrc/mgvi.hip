// Metric Gaussian Variational Inference around the ICR prior with a Gaussian
// likelihood (inverse noise variance w per final pixel), section "Variational
// Inference": MGVI draws antithetic samples mean +- delta with delta = M^-1 r,
// r = eta + L^T (sqrt(w) eta') (covariance M, so delta has covariance M^-1), and
// moves the expansion point by Newton-CG on the KL, whose gradient over antithetic
// pairs is M mean - L^T W d with the metric M = L^T W L + 1.
//
// Two device operations serve both, on top of the sweeps and CG:
//   weighted adjoint  out = L^T (w^p * y) + add   (p = 1/2: sample right-hand side,
//                                                   p = 1: the data term b = L^T W d)
//   Newton step       mean -= M^-1 (M mean - b)    (one metric product, CG, update)
#include "icr_internal.h"

namespace icr {
namespace {

constexpr int kVecThreads = 256;
constexpr int kVecBlocks = 1024;

// y = w^p * v over n elements per sample (w with stride w_bs, 0 = shared by the batch).
template <typename T, typename TA>
__global__ void __launch_bounds__(kVecThreads) weight_kernel(const TA* __restrict__ w, int64_t w_bs,
                                                            const T* __restrict__ v, int64_t v_bs,
                                                            T* __restrict__ y, int64_t y_bs, int64_t n, int half) {
  const int64_t b = blockIdx.y;
  w += b * w_bs;
  v += b * v_bs;
  y += b * y_bs;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const TA wk = w[k];
    store_acc(y + k, (half ? sqrt(wk) : wk) * load_acc(v + k));
  }
}

// a -= c elementwise over n elements per sample.
template <typename T>
__global__ void __launch_bounds__(kVecThreads) sub_kernel(T* __restrict__ a, const T* __restrict__ c, int64_t n) {
  const int64_t b = blockIdx.y;
  a += b * n;
  c += b * n;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x)
    store_acc(a + k, load_acc(a + k) - load_acc(c + k));
}

template <typename T>
hipError_t weight_t(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* v, int64_t v_bs,
                    void* y, int64_t y_bs, int64_t n, bool half, hipStream_t st) {
  using TA = typename Acc<T>::type;
  const dim3 grid(kVecBlocks, static_cast<unsigned>(batch));
  weight_kernel<T, TA><<<grid, kVecThreads, 0, st>>>(static_cast<const TA*>(w), w_bs, static_cast<const T*>(v),
                                                     v_bs, static_cast<T*>(y), y_bs, n, half ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t sub_t(int64_t batch, void* a, const void* c, int64_t n, hipStream_t st) {
  const dim3 grid(kVecBlocks, static_cast<unsigned>(batch));
  sub_kernel<T><<<grid, kVecThreads, 0, st>>>(static_cast<T*>(a), static_cast<const T*>(c), n);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_weight(const icr_plan* p, int64_t batch, const void* w, int64_t w_bs, const void* v, int64_t v_bs,
                         void* y, int64_t y_bs, int64_t n, bool half, hipStream_t st) {
  switch (p->precision) {
    case ICR_F64: return weight_t<double>(p, batch, w, w_bs, v, v_bs, y, y_bs, n, half, st);
    case ICR_F32: return weight_t<float>(p, batch, w, w_bs, v, v_bs, y, y_bs, n, half, st);
    default: return weight_t<bf16_t>(p, batch, w, w_bs, v, v_bs, y, y_bs, n, half, st);
  }
}

hipError_t launch_sub(const icr_plan* p, int64_t batch, void* a, const void* c, int64_t n, hipStream_t st) {
  switch (p->precision) {
    case ICR_F64: return sub_t<double>(batch, a, c, n, st);
    case ICR_F32: return sub_t<float>(batch, a, c, n, st);
    default: return sub_t<bf16_t>(batch, a, c, n, st);
  }
}

}  // namespace icr
