// Correlated-field model on an n x n periodic grid and the Fisher metric of a Poisson
// likelihood (NIFTy.re, section "Gaussian Processes": s = FT(sqrt(P) xi); section
// "Performance of NIFTy.re compared to NIFTy": M_p = J^T N^-1 J + 1).
//
// The field is real, so FT is the 2-D Hartley transform, normalised to be its own
// inverse: T x = (Re - Im)(FFT2 x) / n. With lambda = exp(m + T(A xi)) the Jacobian is
// J = diag(lambda) T diag(A) and N^-1 = diag(1 / lambda), so
//   M_p v = v + A T(lambda(p) T(A v)).
//
// T comes from the separable transform S = H_rows H_cols (1-D Hartley transforms along
// each axis, in either order) through the identity cas(a + b) = (cas a cas b + cas(-a) cas b
// + cas a cas(-b) - cas(-a) cas(-b)) / 2:
//   T[k][l] = (S[k][l] + S[-k][l] + S[k][-l] - S[-k][-l]) / 2.
// Two real sequences go through one complex FFT, z = a + i b. When b is the reflection
// partner of a (column -c of column c, or row -k of row k) of data already transformed
// along the other axis, the combine collapses: with Z = FFT(z), T at a is Re Z[k] and at
// the partner Im Z[-k]. The pair (0, n/2) (both their own partners) takes the plain split
// H_a = (Z[k] + conj Z[-k]) / 2, H_b = (Z[k] - conj Z[-k]) / 2i in Hartley form.
//
// Passes (hand-written kernels, FP32, Stockham FFTs in LDS, radix 4 up to n = 1024, else 16):
//   rows:  four real rows per workgroup (two complex FFTs); writes the row transforms to a
//          column-blocked layout: block b holds the columns c = 4b + j (j < 4) and their
//          partners m = n - c (n/2 for c = 0) as float2 (value at c, value at m), all rows
//          of the block contiguous, so the column pass reads one contiguous region;
//   cols:  one block (four complex FFTs of length n) per workgroup: the column transforms
//          and the combine give T for the block's eight columns. For T alone (and the rate
//          exp(m + T)) they are written out; for M_p they are multiplied by lambda and
//          transformed along the columns again (the second transform starts with the
//          column axis), written back in place with the rows ordered as partner pairs
//          (0, n/2), (1, n-1), ...;
//   final rows (M_p): two row pairs per workgroup, the row transforms and the combine,
//          and out = v + A T(u) in the same pass.
// M_p is three launches moving v, A, lambda, v, A, out and the blocked grid twice. Up to
// n = 64 each operator is one launch of a single workgroup that holds the grid in LDS and
// runs the same steps with the grid rearranged between the axes.
// Twiddles come from a 128-entry table (two factors per twiddle) staged in LDS.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "icr_cf.h"
#include "icr_internal.h"

struct icr_cf_plan {
  int n = 0;
  int logn = 0;
  double mean = 0.0;
  float* amp = nullptr;  // device [n][n] amplitude spectrum
  float2* tw = nullptr;  // device twiddle table (128 entries, see the kernels)
};

namespace icr {
namespace {

// LDS holds F sequences of N complex values. Inside a sequence one float2 of padding
// follows every 16, so the stride-16 writes of the first radix-16 stage spread over the
// banks; sequences are N + N/16 + 4 apart, so a walk across sequences at equal index does.
template <int N>
constexpr int seq_stride() {
  return N + N / 16 + 4;
}
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Largest radix of the FFT stages. Small grids are latency-bound: a smaller radix gives
// more threads per workgroup and shorter stages.
// Measured device time per M_p apply, radix 4 against 16: 11.4 against 16.3 us at 256^2,
// 14.6 against 21.8 at 512^2, 22.5 against 28.0 at 1024^2; radix 8 fell between.
template <int N>
constexpr int max_radix() {
  return N <= 1024 ? 4 : 16;
}

// Grids up to this size run each operator as one workgroup (n = 64: 8.4 us per M_p apply;
// at n = 128 the three-pass path is faster).
constexpr int kOneGroupLimit = 64;

// One butterfly of the largest radix per thread and stage (64 to 1024 threads).
template <int N, int F>
constexpr int fft_threads() {
  return F * N / max_radix<N>() < 64 ? 64 : (F * N / max_radix<N>() > 1024 ? 1024 : F * N / max_radix<N>());
}

// Per-thread trip count of a loop over `count` items with nt threads.
constexpr int trips(int count, int nt) { return (count + nt - 1) / nt; }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// cos(pi e / 8) for 0 <= e <= 4
constexpr float kCosPi8[5] = {1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f, 0.0f};
constexpr float cos_pi8(int e) {
  return e > 8 ? cos_pi8(16 - e) : (e > 4 ? -kCosPi8[8 - e] : kCosPi8[e]);
}
constexpr int high_bit(int r) { return r < 2 ? r : 2 * high_bit(r / 2); }

// x exp(-2 pi i E / R) for R dividing 16; the quarter turns are exact.
template <int R, int E>
__device__ __forceinline__ float2 rot(float2 x) {
  constexpr int e = (16 / R * E) & 15;  // the angle in units of pi / 8
  if constexpr (e == 0) return x;
  else if constexpr (e == 4) return make_float2(x.y, -x.x);
  else if constexpr (e == 8) return make_float2(-x.x, -x.y);
  else if constexpr (e == 12) return make_float2(-x.y, x.x);
  else {
    constexpr float c = cos_pi8(e), s = cos_pi8((e + 12) & 15);  // cos and sin of pi e / 8
    return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
  }
}

// In-register DFT of R points (R a power of two up to 16), forward sign, natural order in
// and out: radix-2 decimation in time, X[k] = E[k] + W^k O[k], X[k + R/2] = E[k] - W^k O[k].
template <int R>
struct Dft {
  template <int K>
  __device__ __forceinline__ static void combine(float2 (&x)[R], const float2 (&e)[R / 2], const float2 (&o)[R / 2]) {
    if constexpr (K < R / 2) {
      const float2 t = rot<R, K>(o[K]);
      x[K] = cadd(e[K], t);
      x[K + R / 2] = csub(e[K], t);
      combine<K + 1>(x, e, o);
    }
  }
  __device__ __forceinline__ static void run(float2 (&x)[R]) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft<R / 2>::run(e);
    Dft<R / 2>::run(o);
    combine<0>(x, e, o);
  }
};
template <>
struct Dft<1> {
  __device__ __forceinline__ static void run(float2 (&)[1]) {}
};

// Twiddles exp(-2 pi i t / n) (t < n <= 4096) as lo[t mod 64] * hi[t / 64], from a
// 128-entry table (lo then hi, computed by the plan in double precision) staged in LDS.
constexpr int kTwEntries = 128;
__device__ __forceinline__ float2 twiddle(const float2* tws, int t) { return cmul(tws[64 + (t >> 6)], tws[t & 63]); }
template <int NT>
__device__ __forceinline__ void load_twiddles(float2* tws, const float2* __restrict__ tw) {
#pragma unroll
  for (int it = 0; it < trips(kTwEntries, NT); ++it) {
    const int i = static_cast<int>(threadIdx.x) + it * NT;
    if (i < kTwEntries) tws[i] = tw[i];
  }
}

// W^r from W^1, W^2, W^4, W^8 (table lookups) as a product of at most four of them.
template <int r>
__device__ __forceinline__ float2 wpow(float2 w1, float2 w2, float2 w4, float2 w8) {
  if constexpr (r == 1) return w1;
  else if constexpr (r == 2) return w2;
  else if constexpr (r == 4) return w4;
  else if constexpr (r == 8) return w8;
  else return cmul(wpow<high_bit(r)>(w1, w2, w4, w8), wpow<r - high_bit(r)>(w1, w2, w4, w8));
}
// v[r] *= W^(r t1) for 0 < r < R
template <int R, int r = 1>
__device__ __forceinline__ void apply_twiddles(float2 (&v)[R], float2 w1, float2 w2, float2 w4, float2 w8) {
  if constexpr (r < R) {
    v[r] = cmul(v[r], wpow<r>(w1, w2, w4, w8));
    apply_twiddles<R, r + 1>(v, w1, w2, w4, w8);
  }
}

// One Stockham (self-sorting) stage of radix R and span NS over F sequences: butterfly j
// (< N/R) reads j + r N/R, twiddles by exp(-2 pi i r (j mod NS) / (R NS)), takes the DFT
// and writes (j / NS) R NS + (j mod NS) + q NS. All reads finish (barrier) before the writes.
template <int N, int F, int NT, int R, int NS>
__device__ __forceinline__ void fft_stage(float2* buf, const float2* tws) {
  constexpr int B = N / R, kTotal = F * B, kIt = trips(kTotal, NT), S = seq_stride<N>();
  float2 v[kIt][R];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int t = static_cast<int>(threadIdx.x) + it * NT;
    if (kTotal % NT == 0 || t < kTotal) {
      const int f = t / B, j = t % B;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = buf[f * S + pad16(j + r * B)];
      if constexpr (NS > 1) {
        const int t1 = (j % NS) * (N / (R * NS));
        const float2 w1 = twiddle(tws, t1);
        const float2 w2 = R > 2 ? twiddle(tws, 2 * t1) : w1;
        const float2 w4 = R > 4 ? twiddle(tws, 4 * t1) : w1;
        const float2 w8 = R > 8 ? twiddle(tws, 8 * t1) : w1;
        apply_twiddles<R>(v[it], w1, w2, w4, w8);
      }
      Dft<R>::run(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int t = static_cast<int>(threadIdx.x) + it * NT;
    if (kTotal % NT == 0 || t < kTotal) {
      const int f = t / B, j = t % B, k = j % NS;
      const int base = (j / NS) * R * NS + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[f * S + pad16(base + q * NS)] = v[it][q];
    }
  }
  __syncthreads();
}

// In-place FFT of the F sequences in LDS: stages of the largest radix, then one of radix
// N / NS. Called by the whole workgroup after a barrier (which also covers the twiddle
// table); ends with one.
template <int N, int F, int NT, int NS = 1>
__device__ __forceinline__ void fft_lds(float2* buf, const float2* tws) {
  if constexpr (NS < N) {
    constexpr int R = N / NS >= max_radix<N>() ? max_radix<N>() : N / NS;
    fft_stage<N, F, NT, R, NS>(buf, tws);
    fft_lds<N, F, NT, NS * R>(buf, tws);
  }
}

// Hartley transforms of the two real sequences in z = a + i b at index k from P = Z[k]
// and Q = Z[-k].
__device__ __forceinline__ float hartley_a(float2 P, float2 Q) { return 0.5f * (P.x + Q.x - P.y + Q.y); }
__device__ __forceinline__ float hartley_b(float2 P, float2 Q) { return 0.5f * (P.y + Q.y + P.x - Q.x); }

// partner of column (or row) c < n/2: its reflection n - c, and n/2 for c = 0
template <int N>
__device__ __forceinline__ int partner(int c) {
  return c == 0 ? N / 2 : N - c;
}
template <int N>
__device__ __forceinline__ int reflect(int k) {
  return (N - k) & (N - 1);
}

// The combine on a partner pair (column c with its partner m, or a row pair) from one
// complex FFT Z of z = (S at c) + i (S at m), where S is already transformed along the
// other axis, at index k (P = Z[k], Q = Z[-k]): T at c and at m. For c = 0 (partner n/2,
// both their own reflections) T is S itself.
__device__ __forceinline__ float combine_c(bool self, float2 P, float2 Q) { return self ? hartley_a(P, Q) : P.x; }
__device__ __forceinline__ float combine_m(bool self, float2 P, float2 Q) { return self ? hartley_b(P, Q) : Q.y; }

// Load rows 2s and 2s+1 of x (times pre, if given) of a run of `rows` rows into LDS as
// sequence s = row 2s + i row 2s+1, four columns per item.
template <int N, int NT, int kRows>
__device__ __forceinline__ void load_row_pairs(const float* __restrict__ x, const float* __restrict__ pre,
                                               float2* buf) {
  constexpr int kItems = kRows / 2 * N / 4, kIt = trips(kItems, NT), S = seq_stride<N>();
  float4 a[kIt], b[kIt];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kItems % NT == 0 || e < kItems) {
      const int s = e / (N / 4), i = 4 * (e % (N / 4));
      a[it] = *reinterpret_cast<const float4*>(x + int64_t(2 * s) * N + i);
      b[it] = *reinterpret_cast<const float4*>(x + int64_t(2 * s + 1) * N + i);
    }
  }
  if (pre) {
    float4 pa[kIt], pb[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kItems % NT == 0 || e < kItems) {
        const int s = e / (N / 4), i = 4 * (e % (N / 4));
        pa[it] = *reinterpret_cast<const float4*>(pre + int64_t(2 * s) * N + i);
        pb[it] = *reinterpret_cast<const float4*>(pre + int64_t(2 * s + 1) * N + i);
      }
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      a[it] = make_float4(a[it].x * pa[it].x, a[it].y * pa[it].y, a[it].z * pa[it].z, a[it].w * pa[it].w);
      b[it] = make_float4(b[it].x * pb[it].x, b[it].y * pb[it].y, b[it].z * pb[it].z, b[it].w * pb[it].w);
    }
  }
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kItems % NT == 0 || e < kItems) {
      const int s = e / (N / 4), i = 4 * (e % (N / 4));
      float2* d = buf + s * S + pad16(i);  // i is a multiple of 4: the four stay adjacent
      d[0] = make_float2(a[it].x, b[it].x);
      d[1] = make_float2(a[it].y, b[it].y);
      d[2] = make_float2(a[it].z, b[it].z);
      d[3] = make_float2(a[it].w, b[it].w);
    }
  }
}

// Output of a final row pass from the FFTs of the row-pair sequences s < kPairs (pair
// p0 + s: rows p and partner(p)): out = v + A T / n, or T / n, or exp(mean + T / n).
enum Post { kPostPlain = 0, kPostExp = 1, kPostMetric = 2 };
template <int N, int NT, int kPairs, int kPost>
__device__ __forceinline__ void store_row_pairs(const float2* buf, int p0, const float* __restrict__ v,
                                                const float* __restrict__ amp, float* __restrict__ out, float mean) {
  constexpr int kItems = kPairs * 2 * N / 4, kIt = trips(kItems, NT), S = seq_stride<N>();
  constexpr float inv = 1.0f / static_cast<float>(N);
  float4 vv[kIt], aa[kIt];
  if constexpr (kPost == kPostMetric) {
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kItems % NT == 0 || e < kItems) {
        const int s = e / (N / 2), h = (e / (N / 4)) & 1, l = 4 * (e % (N / 4));
        const int p = p0 + s;
        const int64_t idx = int64_t(h == 0 ? p : partner<N>(p)) * N + l;
        vv[it] = *reinterpret_cast<const float4*>(v + idx);
        aa[it] = *reinterpret_cast<const float4*>(amp + idx);
      }
    }
  }
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kItems % NT == 0 || e < kItems) {
      const int s = e / (N / 2), h = (e / (N / 4)) & 1, l = 4 * (e % (N / 4));
      const int p = p0 + s;
      const float2* z = buf + s * S;
      float t[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 P = z[pad16(l + i)], Q = z[pad16(reflect<N>(l + i))];
        t[i] = inv * (h ? combine_m(p == 0, P, Q) : combine_c(p == 0, P, Q));
      }
      const int64_t idx = int64_t(h == 0 ? p : partner<N>(p)) * N + l;
      float4 r;
      if constexpr (kPost == kPostMetric) {
        r = make_float4(vv[it].x + aa[it].x * t[0], vv[it].y + aa[it].y * t[1], vv[it].z + aa[it].z * t[2],
                        vv[it].w + aa[it].w * t[3]);
      } else if constexpr (kPost == kPostExp) {
        r = make_float4(expf(mean + t[0]), expf(mean + t[1]), expf(mean + t[2]), expf(mean + t[3]));
      } else {
        r = make_float4(t[0], t[1], t[2], t[3]);
      }
      *reinterpret_cast<float4*>(out + idx) = r;
    }
  }
}

// Row transforms: workgroup q takes rows 4q..4q+3 of x (times pre, if given), rows 4q + 2s
// and 4q + 2s + 1 as the real and imaginary parts of sequence s, and writes
// blk[(b n + row) 4 + j] = (H_row[c], H_row[partner(c)]) for c = 4b + j.
template <int N>
__global__ void __launch_bounds__((fft_threads<N, 2>())) cf_rows(const float* __restrict__ x,
                                                                 const float* __restrict__ pre,
                                                                 const float2* __restrict__ tw,
                                                                 float2* __restrict__ blk) {
  constexpr int F = 2, NT = fft_threads<N, 2>(), S = seq_stride<N>();
  __shared__ float2 buf[F * S];
  __shared__ float2 tws[kTwEntries];
  const int q = blockIdx.x;
  const int64_t row0 = int64_t(4) * q * N;
  load_twiddles<NT>(tws, tw);
  load_row_pairs<N, NT, 4>(x + row0, pre ? pre + row0 : nullptr, buf);
  __syncthreads();
  fft_lds<N, F, NT>(buf, tws);
  constexpr int kItems = 2 * N;  // (block, row, j): 16 float2 (128 bytes) per block
#pragma unroll
  for (int it = 0; it < trips(kItems, NT); ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kItems % NT == 0 || e < kItems) {
      const int b = e >> 4, r = (e >> 2) & 3, j = e & 3;
      const int c = 4 * b + j, m = partner<N>(c);
      const float2* z = buf + (r >> 1) * S;
      const float2 zc = z[pad16(c)], zcn = z[pad16(reflect<N>(c))];
      const float2 zm = z[pad16(m)], zmn = z[pad16(reflect<N>(m))];
      const float hc = (r & 1) ? hartley_b(zc, zcn) : hartley_a(zc, zcn);
      const float hm = (r & 1) ? hartley_b(zm, zmn) : hartley_a(zm, zmn);
      blk[(int64_t(b) * N + 4 * q + r) * 4 + j] = make_float2(hc, hm);
    }
  }
}

// Block of workgroup i. From n = 512 on, the eight blocks whose columns share 128-byte
// lines of lambda run together on one XCD (workgroup i runs on XCD i mod 8), so the
// column-wise reads of lambda hit in that XCD's L2.
template <int N>
__device__ __forceinline__ int col_block(int i) {
  if constexpr (N / 8 >= 64) {
    const int x = i & 7, t = i >> 3;
    return 8 * (x + 8 * (t >> 3)) + (t & 7);
  } else {
    return i;
  }
}

// u = lambda T / n in place on the F column-pair sequences (sequence f: column c0(f) and
// its partner) of FFTs Z, from the row pairs (k, -k): each item reads Z[k], Z[-k] and
// writes both, so items never overlap.
template <int N, int F, int NT, typename C0>
__device__ __forceinline__ void scale_by_rate(float2* buf, const float* __restrict__ lam, C0 c0_of) {
  constexpr int kItems = F * (N / 2 + 1), kIt = trips(kItems, NT), S = seq_stride<N>();
  constexpr float inv = 1.0f / static_cast<float>(N);
  float l4[kIt][4];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kItems % NT == 0 || e < kItems) {
      const int k = e / F, f = e % F, nk = reflect<N>(k);
      const int c = c0_of(f), m = partner<N>(c);
      l4[it][0] = lam[int64_t(k) * N + c];
      l4[it][1] = lam[int64_t(k) * N + m];
      l4[it][2] = lam[int64_t(nk) * N + c];
      l4[it][3] = lam[int64_t(nk) * N + m];
    }
  }
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kItems % NT == 0 || e < kItems) {
      const int k = e / F, f = e % F, nk = reflect<N>(k);
      const bool self = c0_of(f) == 0;
      float2* z = buf + f * S;
      const float2 P = z[pad16(k)], Q = z[pad16(nk)];
      z[pad16(k)] = make_float2(inv * l4[it][0] * combine_c(self, P, Q), inv * l4[it][1] * combine_m(self, P, Q));
      z[pad16(nk)] = make_float2(inv * l4[it][2] * combine_c(self, Q, P), inv * l4[it][3] * combine_m(self, Q, P));
    }
  }
}

// Column transforms of one block (four complex FFTs over the rows; sequence j is column
// c + i column partner(c), c = 4b + j) and the combine: T at column c is Re Z[k], at its
// partner Im Z[-k] (the block-0 pair (0, n/2) by the plain split).
//   kPostPlain / kPostExp: out = T / n (or exp(mean + T / n)), row-major.
//   kPostMetric: u = lambda T / n, then the column transforms of u, written back to the
//   block in place with row k at slot 0 (k = 0), 1 (k = n/2), 2k (k < n/2), 2(n-k)+1.
// (Half a block per workgroup, two per compute unit at n = 4096, measured slower.)
template <int N, int kPost>
__global__ void __launch_bounds__((fft_threads<N, 4>())) cf_cols(float2* __restrict__ blk,
                                                                 const float* __restrict__ lam,
                                                                 float* __restrict__ out,
                                                                 const float2* __restrict__ tw, float mean) {
  constexpr int F = 4, NT = fft_threads<N, F>(), S = seq_stride<N>();
  __shared__ float2 buf[F * S];
  __shared__ float2 tws[kTwEntries];
  const int b = col_block<N>(blockIdx.x);
  // a row of the block is two float4, each the pairs (2 jj, 2 jj + 1)
  float4* region = reinterpret_cast<float4*>(blk + int64_t(b) * N * 4);
  load_twiddles<NT>(tws, tw);
  constexpr int kLd = N * F / 2, kItL = trips(kLd, NT);
  {
    float4 r4[kItL];
#pragma unroll
    for (int it = 0; it < kItL; ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kLd % NT == 0 || e < kLd) r4[it] = region[e];
    }
#pragma unroll
    for (int it = 0; it < kItL; ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kLd % NT == 0 || e < kLd) {
        const int row = e >> 1, f = 2 * (e & 1);
        buf[f * S + pad16(row)] = make_float2(r4[it].x, r4[it].y);
        buf[(f + 1) * S + pad16(row)] = make_float2(r4[it].z, r4[it].w);
      }
    }
  }
  __syncthreads();
  fft_lds<N, F, NT>(buf, tws);
  constexpr float inv = 1.0f / static_cast<float>(N);
  if constexpr (kPost != kPostMetric) {
    constexpr int kItems = 2 * F * N;  // (row k, lower / partner, f)
#pragma unroll
    for (int it = 0; it < trips(kItems, NT); ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kItems % NT == 0 || e < kItems) {
        const int k = e / (2 * F), h = (e / F) & 1, f = e % F;
        const int c = 4 * b + f;
        const float2* z = buf + f * S;
        const float2 P = z[pad16(k)], Q = z[pad16(reflect<N>(k))];
        float t = inv * (h ? combine_m(c == 0, P, Q) : combine_c(c == 0, P, Q));
        if (kPost == kPostExp) t = expf(mean + t);
        out[int64_t(k) * N + (h ? partner<N>(c) : c)] = t;
      }
    }
  } else {
    scale_by_rate<N, F, NT>(buf, lam, [b](int f) { return 4 * b + f; });
    __syncthreads();
    fft_lds<N, F, NT>(buf, tws);
#pragma unroll
    for (int it = 0; it < kItL; ++it) {  // (slot, pair of sequences)
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kLd % NT == 0 || e < kLd) {
        const int slot = e >> 1, f = 2 * (e & 1);
        const int p = slot >> 1;
        const int k = (slot & 1) ? partner<N>(p) : p;
        const float2 P0 = buf[f * S + pad16(k)], Q0 = buf[f * S + pad16(reflect<N>(k))];
        const float2 P1 = buf[(f + 1) * S + pad16(k)], Q1 = buf[(f + 1) * S + pad16(reflect<N>(k))];
        region[e] = make_float4(hartley_a(P0, Q0), hartley_b(P0, Q0), hartley_a(P1, Q1), hartley_b(P1, Q1));
      }
    }
  }
}

// Final row pass of M_p: workgroup q takes the row pairs p = 2q + s (s = 0, 1), rows
// (p, partner(p)) from slots 4q + 2s and 4q + 2s + 1 of every block, as sequence
// s = row p + i row partner(p); the row transforms and the combine give T(u) on both
// rows, and out = v + A T(u) / n.
template <int N>
__global__ void __launch_bounds__((fft_threads<N, 2>())) cf_rows_final(const float2* __restrict__ blk,
                                                                       const float* __restrict__ v,
                                                                       const float* __restrict__ amp,
                                                                       float* __restrict__ out,
                                                                       const float2* __restrict__ tw) {
  constexpr int F = 2, NT = fft_threads<N, 2>(), S = seq_stride<N>();
  __shared__ float2 buf[F * S];
  __shared__ float2 tws[kTwEntries];
  const int q = blockIdx.x;
  load_twiddles<NT>(tws, tw);
  const float4* blk4 = reinterpret_cast<const float4*>(blk);
  constexpr int kLd = N, kIt = trips(kLd, NT);  // (block, slot, j pair): 8 float4 per block
  float4 d[kIt];
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kLd % NT == 0 || e < kLd) {
      const int b = e >> 3, slot = (e >> 1) & 3, jj = e & 1;
      d[it] = blk4[(int64_t(b) * N + 4 * q + slot) * 2 + jj];
    }
  }
  float* bf = reinterpret_cast<float*>(buf);
#pragma unroll
  for (int it = 0; it < kIt; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * NT;
    if (kLd % NT == 0 || e < kLd) {
      const int b = e >> 3, slot = (e >> 1) & 3, jj = e & 1;
      const int s = slot >> 1, h = slot & 1, c0 = 4 * b + 2 * jj, c1 = c0 + 1;
      bf[2 * (s * S + pad16(c0)) + h] = d[it].x;
      bf[2 * (s * S + pad16(partner<N>(c0))) + h] = d[it].y;
      bf[2 * (s * S + pad16(c1)) + h] = d[it].z;
      bf[2 * (s * S + pad16(partner<N>(c1))) + h] = d[it].w;
    }
  }
  __syncthreads();
  fft_lds<N, F, NT>(buf, tws);
  store_row_pairs<N, NT, 2, kPostMetric>(buf, 2 * q, v, amp, out, 0.0f);
}

// The whole operator in one workgroup for small n (the grid fits in LDS as n/2 complex
// sequences): rows as pairs (2s, 2s+1), then the same grid rearranged as column pairs
// (c, partner(c)), and for M_p once more as row pairs (p, partner(p)).
template <int N, int kPost>
__global__ void __launch_bounds__((fft_threads<N, N / 2>())) cf_small(const float* __restrict__ x,
                                                                      const float* __restrict__ pre,
                                                                      const float* __restrict__ lam,
                                                                      const float* __restrict__ v,
                                                                      float* __restrict__ out,
                                                                      const float2* __restrict__ tw, float mean) {
  constexpr int F = N / 2, NT = fft_threads<N, F>(), S = seq_stride<N>();
  __shared__ float2 buf[F * S];
  __shared__ float2 tws[kTwEntries];
  load_twiddles<NT>(tws, tw);
  load_row_pairs<N, NT, N>(x, pre, buf);
  __syncthreads();
  fft_lds<N, F, NT>(buf, tws);
  constexpr int kItems = F * F, kIt = trips(kItems, NT);  // (row pair s, column pair c)
  {
    // row transforms -> column-pair sequences: sequence c at row r = (H_row[r][c], H_row[r][m])
    float2 o0[kIt], o1[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kItems % NT == 0 || e < kItems) {
        const int s = e / F, c = e % F, m = partner<N>(c);
        const float2* z = buf + s * S;
        const float2 zc = z[pad16(c)], zcn = z[pad16(reflect<N>(c))];
        const float2 zm = z[pad16(m)], zmn = z[pad16(reflect<N>(m))];
        o0[it] = make_float2(hartley_a(zc, zcn), hartley_a(zm, zmn));
        o1[it] = make_float2(hartley_b(zc, zcn), hartley_b(zm, zmn));
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kItems % NT == 0 || e < kItems) {
        const int s = e / F, c = e % F;
        buf[c * S + pad16(2 * s)] = o0[it];
        buf[c * S + pad16(2 * s + 1)] = o1[it];
      }
    }
  }
  __syncthreads();
  fft_lds<N, F, NT>(buf, tws);
  constexpr float inv = 1.0f / static_cast<float>(N);
  if constexpr (kPost != kPostMetric) {
    constexpr int kOut = N * N;  // (row k, column c), both halves of every pair
#pragma unroll
    for (int it = 0; it < trips(kOut, NT); ++it) {
      const int e = static_cast<int>(threadIdx.x) + it * NT;
      if (kOut % NT == 0 || e < kOut) {
        const int k = e / N, col = e % N;
        const bool lower = col < N / 2;
        const int c = lower ? col : (col == N / 2 ? 0 : N - col);
        const float2* z = buf + c * S;
        const float2 P = z[pad16(k)], Q = z[pad16(reflect<N>(k))];
        float t = inv * (lower ? combine_c(c == 0, P, Q) : combine_m(c == 0, P, Q));
        if (kPost == kPostExp) t = expf(mean + t);
        out[e] = t;
      }
    }
  } else {
    scale_by_rate<N, F, NT>(buf, lam, [](int f) { return f; });
    __syncthreads();
    fft_lds<N, F, NT>(buf, tws);
    {
      // column transforms -> row-pair sequences: sequence p at column l = (S'[p][l], S'[partner(p)][l])
      float2 o0[kIt], o1[kIt];
#pragma unroll
      for (int it = 0; it < kIt; ++it) {
        const int e = static_cast<int>(threadIdx.x) + it * NT;
        if (kItems % NT == 0 || e < kItems) {
          const int p = e / F, c = e % F, pp = partner<N>(p);
          const float2* z = buf + c * S;
          const float2 P1 = z[pad16(p)], Q1 = z[pad16(reflect<N>(p))];
          const float2 P2 = z[pad16(pp)], Q2 = z[pad16(reflect<N>(pp))];
          o0[it] = make_float2(hartley_a(P1, Q1), hartley_a(P2, Q2));  // column c
          o1[it] = make_float2(hartley_b(P1, Q1), hartley_b(P2, Q2));  // column partner(c)
        }
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kIt; ++it) {
        const int e = static_cast<int>(threadIdx.x) + it * NT;
        if (kItems % NT == 0 || e < kItems) {
          const int p = e / F, c = e % F;
          buf[p * S + pad16(c)] = o0[it];
          buf[p * S + pad16(partner<N>(c))] = o1[it];
        }
      }
    }
    __syncthreads();
    fft_lds<N, F, NT>(buf, tws);
    store_row_pairs<N, NT, F, kPostMetric>(buf, 0, v, pre, out, 0.0f);
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

// out = T(pre * x) (kPostPlain) or exp(mean + T(pre * x)) (kPostExp); work: the blocked grid.
template <int N>
hipError_t transform_n(const icr_cf_plan* p, const float* x, const float* pre, float* out, int post, float2* work,
                       hipStream_t st) {
  const float mean = static_cast<float>(p->mean);
  if constexpr (N <= kOneGroupLimit) {
    constexpr unsigned nt = fft_threads<N, N / 2>();
    if (post == kPostExp) cf_small<N, kPostExp><<<1, nt, 0, st>>>(x, pre, nullptr, nullptr, out, p->tw, mean);
    else cf_small<N, kPostPlain><<<1, nt, 0, st>>>(x, pre, nullptr, nullptr, out, p->tw, mean);
  } else {
    cf_rows<N><<<N / 4, fft_threads<N, 2>(), 0, st>>>(x, pre, p->tw, work);
    constexpr unsigned wgs = N / 8, nt = fft_threads<N, 4>();
    if (post == kPostExp) cf_cols<N, kPostExp><<<wgs, nt, 0, st>>>(work, nullptr, out, p->tw, mean);
    else cf_cols<N, kPostPlain><<<wgs, nt, 0, st>>>(work, nullptr, out, p->tw, mean);
  }
  return hipGetLastError();
}

// out = v + A T(lambda T(A v))
template <int N>
hipError_t metric_n(const icr_cf_plan* p, const float* lam, const float* v, float* out, float2* work,
                    hipStream_t st) {
  if constexpr (N <= kOneGroupLimit) {
    cf_small<N, kPostMetric><<<1, fft_threads<N, N / 2>(), 0, st>>>(v, p->amp, lam, v, out, p->tw, 0.0f);
  } else {
    cf_rows<N><<<N / 4, fft_threads<N, 2>(), 0, st>>>(v, p->amp, p->tw, work);
    constexpr unsigned wgs = N / 8, nt = fft_threads<N, 4>();
    cf_cols<N, kPostMetric><<<wgs, nt, 0, st>>>(work, lam, nullptr, p->tw, 0.0f);
    cf_rows_final<N><<<N / 4, fft_threads<N, 2>(), 0, st>>>(work, v, p->amp, out, p->tw);
  }
  return hipGetLastError();
}

template <template <int> class Op, typename... Args>
hipError_t by_size(int logn, Args... args) {
  switch (logn) {
    case 5: return Op<32>::run(args...);
    case 6: return Op<64>::run(args...);
    case 7: return Op<128>::run(args...);
    case 8: return Op<256>::run(args...);
    case 9: return Op<512>::run(args...);
    case 10: return Op<1024>::run(args...);
    case 11: return Op<2048>::run(args...);
    case 12: return Op<4096>::run(args...);
    default: return hipErrorInvalidValue;
  }
}
template <int N>
struct TransformOp {
  static hipError_t run(const icr_cf_plan* p, const float* x, const float* pre, float* out, int mode, float2* work,
                        hipStream_t st) {
    return transform_n<N>(p, x, pre, out, mode, work, st);
  }
};
template <int N>
struct MetricOp {
  static hipError_t run(const icr_cf_plan* p, const float* lam, const float* v, float* out, float2* work,
                        hipStream_t st) {
    return metric_n<N>(p, lam, v, out, work, st);
  }
};

icr_status cf_fail(icr_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

// the passes move four floats at a time
bool cf_aligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) % 16) == 0; }

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
  // twiddle table: exp(-2 pi i l / n) for l < 64, then exp(-2 pi i 64 h / n) for h < 64,
  // from the double-precision angle
  std::vector<float2> tw(icr::kTwEntries);
  for (int t = 0; t < icr::kTwEntries; ++t) {
    const double turns = t < 64 ? t : 64.0 * (t - 64);
    const double a = -2.0 * M_PI * turns / static_cast<double>(n);
    tw[t] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a)));
  }
  hipError_t e = hipMalloc(&p->amp, sizeof(float) * size_t(n) * n);
  if (e == hipSuccess) e = hipMalloc(&p->tw, sizeof(float2) * tw.size());
  if (e == hipSuccess) e = hipMemcpy(p->tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const int64_t total = int64_t(n) * n;
    icr::cf_amplitude_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, st>>>(p->amp, n, amplitude,
                                                                                        zero_mode, length, slope);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) {
    if (p->amp) (void)hipFree(p->amp);
    if (p->tw) (void)hipFree(p->tw);
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
  *bytes = int64_t(p->n) * p->n * int64_t(sizeof(float));
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
  if (!icr::cf_aligned(x) || !icr::cf_aligned(y) || !icr::cf_aligned(workspace))
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "buffer not 16-byte aligned");
  const hipError_t e = icr::by_size<icr::TransformOp>(p->logn, p, x, static_cast<const float*>(nullptr), y,
                                                      static_cast<int>(icr::kPostPlain), static_cast<float2*>(workspace),
                                                      static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return icr::cf_fail(ICR_ERR_HIP, std::string("transform: ") + hipGetErrorString(e));
  return ICR_OK;
}

icr_status icr_cf_rate(const icr_cf_plan* p, const float* position, float* lambda, void* workspace,
                       void* hip_stream) {
  icr::clear_error();
  if (!p || !position || !lambda || !workspace) return icr::cf_fail(ICR_ERR_INVALID_ARG, "NULL argument");
  if (!icr::cf_aligned(position) || !icr::cf_aligned(lambda) || !icr::cf_aligned(workspace))
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "buffer not 16-byte aligned");
  const hipError_t e = icr::by_size<icr::TransformOp>(p->logn, p, position, static_cast<const float*>(p->amp), lambda,
                                                      static_cast<int>(icr::kPostExp), static_cast<float2*>(workspace),
                                                      static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return icr::cf_fail(ICR_ERR_HIP, std::string("rate: ") + hipGetErrorString(e));
  return ICR_OK;
}

icr_status icr_cf_metric_apply(const icr_cf_plan* p, const float* lambda, const float* v, float* out,
                               void* workspace, void* hip_stream) {
  icr::clear_error();
  if (!p || !lambda || !v || !out || !workspace) return icr::cf_fail(ICR_ERR_INVALID_ARG, "NULL argument");
  if (!icr::cf_aligned(lambda) || !icr::cf_aligned(v) || !icr::cf_aligned(out) || !icr::cf_aligned(workspace))
    return icr::cf_fail(ICR_ERR_INVALID_ARG, "buffer not 16-byte aligned");
  if (v == out) return icr::cf_fail(ICR_ERR_INVALID_ARG, "v and out must differ");
  const hipError_t e = icr::by_size<icr::MetricOp>(p->logn, p, lambda, v, out, static_cast<float2*>(workspace),
                                                   static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return icr::cf_fail(ICR_ERR_HIP, std::string("metric: ") + hipGetErrorString(e));
  return ICR_OK;
}

icr_status icr_cf_destroy(icr_cf_plan* p) {
  icr::clear_error();
  if (!p) return ICR_OK;
  if (p->amp) (void)hipFree(p->amp);
  if (p->tw) (void)hipFree(p->tw);
  delete p;
  return ICR_OK;
}

}  // extern "C"
