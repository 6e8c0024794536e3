// 2-D refinement level, forward and adjoint, with the dense 4 x 9 R and lower 4 x 4
// sqrtD of a stationary level, or of each coarse row of a shell-charted level (one set
// per radial index, the marching axis), FP32 arithmetic with FP32 or bfloat16 storage.
//
// Forward: a lane owns two neighbouring interior coarse pixels along x (x = 2P+1, 2P+2)
// and marches along y; the four coarse columns 2P .. 2P+3 of the rows y-1, y, y+1 slide
// in registers, so each coarse row is read once per lane, and the pair's four fine
// values per fine row are one 16-byte excitation load and one 16-byte store.
//
// The transpose of the forward block map s_{l+1}[2(c-1)+b] = sum_w R[b,w] s_l[c+w] +
// sum_{b'} sqrtD[b,b'] xi_{l+1}[2(c-1)+b'] is, per coarse pixel p (a gather, no atomics)
//   s_bar_l[p]            = sum_{w, c = p - w interior} sum_b R[b,w] y[2(c-1)+b],
//   xi_bar_{l+1}[2(p-1)+b'] = sum_{b >= b'} sqrtD[b,b'] y[2(p-1)+b]       (p interior).
// Each block c forms its nine window contributions u[w] = sum_b R[b,w] y_c[b] once.
// A lane owns two neighbouring blocks along x (so the four fine values of a pair's
// fine row are one 16-byte vector) and marches along y: the wy = -1, 0, +1 parts are
// accumulated in registers row by row, and the wx = -1, +1 parts of the neighbouring
// pairs come from the adjacent lanes through DPP wave shifts. A wavefront covers 62
// pairs; its first and last lanes recompute the neighbouring strips' edge pairs.
// There is no LDS and no barrier; each coarse cotangent is summed by one lane in a
// fixed order, so results are bitwise reproducible.
#include "icr_internal.h"
#include "sweep_io.h"

namespace icr {
namespace {

using namespace sweep;

struct Mat2 {
  float r[36];  // R[b][w], b = (by, bx), w = (wy, wx), lexicographic with the last axis fastest
  float s[10];  // lower sqrtD by rows: s[c (c + 1) / 2 + c']
};

// The matrices of a block row: a stationary level passes its set by value, a shell
// level a table with one row per coarse row (R, then sqrtD lower by rows, see
// shell2_table_kernel), read through the constant address space: every lane of a
// wavefront marches through the same rows, so the compiler uses scalar loads.
struct Stat2 {
  Mat2 m;
};
struct Shell2 {
  const float* tab;
  int nsets;
};
typedef const float __attribute__((address_space(4))) const_float2d;
template <typename M>
__device__ __forceinline__ const const_float2d* row_of(const M& m, int set) {
  return (const const_float2d*)(m.tab + static_cast<int64_t>(min(max(set, 0), m.nsets - 1)) * kShellStride);
}
template <typename M>
constexpr bool kShell2 = false;
template <>
constexpr bool kShell2<Shell2> = true;

// Shell levels: a wavefront's matrix rows for the block rows it marches, staged in its own
// LDS slice by one round of vector loads. Read with scalar loads instead, every block row
// waits for its own row (the scheduling barriers that keep the data prefetch ahead keep
// those loads in place), and a short march is a chain of such waits. Marches longer than
// kStagedRows block rows read the table directly.
constexpr int kStagedRows = 10;
constexpr int kRowFloats = 48;  // R (36) and the lower sqrtD (10), padded to whole 16-byte vectors
__device__ __forceinline__ void stage_rows(const Shell2& m, float* lds, int set0, int n, int lane) {
  constexpr int kVec = kRowFloats / 4;
  constexpr int kRounds = (kStagedRows * kVec + 63) / 64;
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    const int i = lane + k * 64;
    if (i < n * kVec) {
      const int r = i / kVec, q = i - r * kVec;
      const int set = min(max(set0 + r, 0), m.nsets - 1);
      reinterpret_cast<float4*>(lds + r * kRowFloats)[q] =
          reinterpret_cast<const float4*>(m.tab + static_cast<int64_t>(set) * kShellStride)[q];
    }
  }
}

struct Adj2Geom {
  int ny, nx;   // coarse shape
  int pairs;    // (nx - 2) / 2 block pairs per row
  int strips;   // wavefront strips along x
  int ychunk;   // coarse rows per wavefront
  int nfx;      // fine row length
  int waves;    // wavefronts per sample
};

constexpr int kLanes = 64;
constexpr int kOwnedPairs = kLanes - 2;  // the first and last lanes are halo
constexpr int kWavesPerGroup = 4;

__host__ __device__ __forceinline__ int sd2(int c, int cp) { return c * (c + 1) / 2 + cp; }

template <typename TS, bool kAdd, typename M>
__global__ void __launch_bounds__(kLanes * kWavesPerGroup) refine2_adj(Adj2Geom g, RefineAdjArgs a, M mats) {
  fetch_args(g.ny, g.nx, g.pairs, g.strips, g.ychunk, g.nfx, g.waves, a.y, a.y_bs, a.xi_bar, a.xi_bar_bs, a.s_bar,
             a.s_bar_bs);
  if (kAdd) fetch_args(a.add, a.add_bs);
  if (halted(a.halt)) return;
  const int lane = threadIdx.x % kLanes;
  // the wavefront index is uniform across its lanes; saying so lets every row-derived
  // address (and a shell level's matrix rows) go through scalar registers
  const int wave = blockIdx.x * kWavesPerGroup + __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
  if (wave >= g.waves) return;  // whole wavefronts leave; the kernel has no barrier
  const int strip = wave % g.strips, chunk = wave / g.strips;
  const int P = strip * kOwnedPairs + lane - 1;  // blocks x = 2P+1, 2P+2
  const bool pair_ok = P >= 0 && P < g.pairs;
  const bool owner = lane >= 1 && lane <= kOwnedPairs && pair_ok;
  const int y0 = chunk * g.ychunk;
  const int y1 = min(y0 + g.ychunk, g.ny);
  const int64_t b = blockIdx.y;
  const TS* y = static_cast<const TS*>(a.y) + b * a.y_bs;
  TS* xb = static_cast<TS*>(a.xi_bar) + b * a.xi_bar_bs;
  TS* sb = static_cast<TS*>(a.s_bar) + b * a.s_bar_bs;
  const TS* add = kAdd ? static_cast<const TS*>(a.add) + b * a.add_bs : nullptr;
  // loads use clamped (in-bounds) block coordinates; blocks outside the interior are
  // zeroed after the load, so no load sits under a branch
  const int Pc = min(max(P, 0), g.pairs - 1);
  auto fine_off = [&](int yb, int by) { return static_cast<int64_t>(2 * (yb - 1) + by) * g.nfx + 4 * Pc; };
  // shell levels: the matrix rows of block rows y0-1 .. y1 (sets yb - 1) in LDS
  __shared__ float staged_rows[kShell2<M> ? kWavesPerGroup : 1][kShell2<M> ? kStagedRows * kRowFloats : 1];
  float* my_rows = staged_rows[kShell2<M> ? threadIdx.x / kLanes : 0];
  const bool staged = kShell2<M> && y1 - y0 + 2 <= kStagedRows;  // uniform per wavefront
  if constexpr (kShell2<M>) {
    if (staged) stage_rows(mats, my_rows, y0 - 2, y1 - y0 + 2, lane);
  }

  struct Row {
    float4 r[2];  // cotangent of the pair's fine rows 2(yb-1) and 2(yb-1)+1
    float4 v[2];  // metric: values added to xi_bar (kAdd)
  };
  auto load_row = [&](int yb, Row& rw) {
    const int yc = min(max(yb, 1), g.ny - 2);
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      rw.r[by] = Io<TS>::ld4(y + fine_off(yc, by));
      if (kAdd) rw.v[by] = Io<TS>::ld4(add + fine_off(yc, by));
    }
  };

  float A0[2][3], A1[2][3];  // partial coarse cotangents of rows yb-1 and yb, per block and wx
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int x = 0; x < 3; ++x) { A0[p][x] = 0.0f; A1[p][x] = 0.0f; }

  auto process = [&](int yb, const Row& rw) {
    const bool ok = pair_ok && yb >= 1 && yb <= g.ny - 2;
    float R[36], S[10];  // this block row's matrices
    if constexpr (kShell2<M>) {
      if (staged) {
        const float* lr = my_rows + (yb - (y0 - 1)) * kRowFloats;
#pragma unroll
        for (int e = 0; e < 36; ++e) R[e] = lr[e];
#pragma unroll
        for (int e = 0; e < 10; ++e) S[e] = lr[36 + e];
      } else {
        const auto row = row_of(mats, yb - 1);
#pragma unroll
        for (int e = 0; e < 36; ++e) R[e] = row[e];
#pragma unroll
        for (int e = 0; e < 10; ++e) S[e] = row[36 + e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 36; ++e) R[e] = mats.m.r[e];
#pragma unroll
      for (int e = 0; e < 10; ++e) S[e] = mats.m.s[e];
    }
    float yv[2][4];  // [block of the pair][by * 2 + bx]
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      const float4 r = rw.r[by];
      yv[0][by * 2] = ok ? r.x : 0.0f;
      yv[0][by * 2 + 1] = ok ? r.y : 0.0f;
      yv[1][by * 2] = ok ? r.z : 0.0f;
      yv[1][by * 2 + 1] = ok ? r.w : 0.0f;
    }
    if (ok && owner && yb >= y0 && yb < y1) {
      float xo[2][4];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int cp = 0; cp < 4; ++cp) {
          float v = 0.0f;
#pragma unroll
          for (int c = cp; c < 4; ++c) v = fmaf(S[sd2(c, cp)], yv[p][c], v);
          xo[p][cp] = v;
        }
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        float4 v = make_float4(xo[0][by * 2], xo[0][by * 2 + 1], xo[1][by * 2], xo[1][by * 2 + 1]);
        if (kAdd) {
          const float4 av = rw.v[by];
          v.x += av.x; v.y += av.y; v.z += av.z; v.w += av.w;
        }
        st4_stream<TS>(xb + fine_off(yb, by), v);  // nontemporal: measured 79 vs 87 us (plain) at 1540^2 x 16
      }
    }
    // window contributions, then the y march: row yb-1 is complete after this block row
    float G[2][3];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      float u[9];
#pragma unroll
      for (int w = 0; w < 9; ++w) {
        float v = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) v = fmaf(R[c * 9 + w], yv[p][c], v);
        u[w] = v;
      }
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        G[p][x] = A0[p][x] + u[x];       // wy = -1: coarse row yb - 1
        A0[p][x] = A1[p][x] + u[3 + x];  // wy =  0: coarse row yb
        A1[p][x] = u[6 + x];             // wy = +1: coarse row yb + 1
      }
    }
    if (yb >= y0 + 1) {  // uniform over the wavefront
      // column 2P+1 takes block 2P+1 at wx = 0, block 2P+2 at wx = -1 and block 2P (the
      // left lane's second block) at wx = +1; column 2P+2 symmetrically
      const float from_left = dpp_from_left(G[1][2]);
      const float from_right = dpp_from_right(G[0][0]);
      if (owner) {
        TS* row = sb + static_cast<int64_t>(yb - 1) * g.nx;
        Io<TS>::st1(row + 2 * P + 1, from_left + G[0][1] + G[1][0]);
        Io<TS>::st1(row + 2 * P + 2, G[0][2] + G[1][1] + from_right);
        if (P == 0) Io<TS>::st1(row, G[0][0]);
        if (P == g.pairs - 1) Io<TS>::st1(row + g.nx - 1, G[1][2]);
      }
    }
  };

  // block rows y0-1 .. y1, two rows in flight: a ring of three buffers, unrolled so no
  // buffer is copied
  Row ra, rb, rc;
  load_row(y0 - 1, ra);
  load_row(y0, rb);
  // the scheduling barriers keep each prefetch ahead of the next row's first wait (with
  // the prefetch sunk below it, the loop entry and the back edge merge into a wait for
  // every outstanding access, loads and stores sharing one counter)
  for (int yb = y0 - 1; yb <= y1; yb += 3) {
    load_row(yb + 2, rc);
    __builtin_amdgcn_sched_barrier(0);
    process(yb, ra);
    if (yb + 1 > y1) break;
    load_row(yb + 3, ra);
    __builtin_amdgcn_sched_barrier(0);
    process(yb + 1, rb);
    if (yb + 2 > y1) break;
    load_row(yb + 4, rb);
    __builtin_amdgcn_sched_barrier(0);
    process(yb + 2, rc);
  }
}

struct Fwd2Geom {
  int ny, nx;   // coarse shape
  int pairs;    // (nx - 2) / 2 pixel pairs per interior row
  int strips;   // wavefront strips along x (64 pairs each)
  int ychunk;   // interior coarse rows per wavefront
  int nfx;      // fine row length
  int waves;    // wavefronts per sample
};

template <typename TS, bool kW, typename M>
__global__ void __launch_bounds__(kLanes * kWavesPerGroup) refine2_fwd(Fwd2Geom g, RefineFwdArgs a, M mats) {
  fetch_args(g.ny, g.nx, g.pairs, g.strips, g.ychunk, g.nfx, g.waves, a.s_in, a.s_in_bs, a.xi, a.xi_bs, a.s_out,
             a.s_out_bs);
  if (kW) fetch_args(a.w, a.w_bs);
  if (halted(a.halt)) return;
  const int lane = threadIdx.x % kLanes;
  // the wavefront index is uniform across its lanes; saying so lets every row-derived
  // address (and a shell level's matrix rows) go through scalar registers
  const int wave = blockIdx.x * kWavesPerGroup + __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
  if (wave >= g.waves) return;  // whole wavefronts leave; the kernel has no barrier
  const int strip = wave % g.strips, chunk = wave / g.strips;
  const int P = strip * kLanes + lane;
  const bool valid = P < g.pairs;
  const int Pc = valid ? P : g.pairs - 1;  // lanes past the row end load the last pair, store nothing
  const int y0 = 1 + chunk * g.ychunk;     // interior coarse rows y0 .. y1-1
  const int y1 = min(y0 + g.ychunk, g.ny - 1);
  const int64_t b = blockIdx.y;
  const TS* sc = static_cast<const TS*>(a.s_in) + b * a.s_in_bs;
  const TS* xi = static_cast<const TS*>(a.xi) + b * a.xi_bs;
  TS* so = static_cast<TS*>(a.s_out) + b * a.s_out_bs;
  const float* w = kW ? static_cast<const float*>(a.w) + b * a.w_bs : nullptr;
  auto fine_off = [&](int y, int by) { return static_cast<int64_t>(2 * (y - 1) + by) * g.nfx + 4 * Pc; };
  auto coarse_row = [&](int y, float (&r)[4]) {
    const TS* row = sc + static_cast<int64_t>(y) * g.nx + 2 * Pc;
    const float2 u = Io<TS>::ld2(row), v = Io<TS>::ld2(row + 2);
    r[0] = u.x; r[1] = u.y; r[2] = v.x; r[3] = v.y;
  };
  // shell levels: the matrix rows of coarse rows y0 .. y1-1 (sets y - 1) in LDS
  __shared__ float staged_rows[kShell2<M> ? kWavesPerGroup : 1][kShell2<M> ? kStagedRows * kRowFloats : 1];
  float* my_rows = staged_rows[kShell2<M> ? threadIdx.x / kLanes : 0];
  const bool staged = kShell2<M> && y1 - y0 <= kStagedRows;  // uniform per wavefront
  if constexpr (kShell2<M>) {
    if (staged) stage_rows(mats, my_rows, y0 - 1, y1 - y0, lane);
  }

  struct Step {
    float c[4];    // coarse row y + 1, columns 2P .. 2P+3
    float4 x[2];   // excitations of the pair's fine rows 2(y-1), 2(y-1)+1
    float4 wr[2];  // metric weights (kW)
  };
  auto load_step = [&](int y, Step& st) {
    const int yc = min(y, y1 - 1);  // past the chunk: reload its last row (in bounds, unused)
    coarse_row(yc + 1, st.c);
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      st.x[by] = Io<TS>::ld4(xi + fine_off(yc, by));
      if (kW) st.wr[by] = *reinterpret_cast<const float4*>(w + fine_off(yc, by));
    }
  };
  float rm[4], r0[4];  // coarse rows y-1 and y
  auto compute_step = [&](int y, const Step& st) {
    float o[2][4];
    float R[36], S[10];  // this coarse row's matrices
    if constexpr (kShell2<M>) {
      if (staged) {
        const float* lr = my_rows + (y - y0) * kRowFloats;
#pragma unroll
        for (int e = 0; e < 36; ++e) R[e] = lr[e];
#pragma unroll
        for (int e = 0; e < 10; ++e) S[e] = lr[36 + e];
      } else {
        const auto row = row_of(mats, y - 1);
#pragma unroll
        for (int e = 0; e < 36; ++e) R[e] = row[e];
#pragma unroll
        for (int e = 0; e < 10; ++e) S[e] = row[36 + e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 36; ++e) R[e] = mats.m.r[e];
#pragma unroll
      for (int e = 0; e < 10; ++e) S[e] = mats.m.s[e];
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      float win[9];  // window of block 2P+1+p: columns 2P+p .. 2P+p+2 of rows y-1, y, y+1
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        win[x] = rm[p + x];
        win[3 + x] = r0[p + x];
        win[6 + x] = st.c[p + x];
      }
      float xv[4];
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        xv[by * 2] = p == 0 ? st.x[by].x : st.x[by].z;
        xv[by * 2 + 1] = p == 0 ? st.x[by].y : st.x[by].w;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float v = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) v = fmaf(R[c * 9 + k], win[k], v);
#pragma unroll
        for (int cp = 0; cp <= c; ++cp) v = fmaf(S[sd2(c, cp)], xv[cp], v);
        o[p][c] = v;
      }
    }
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      float4 v = make_float4(o[0][by * 2], o[0][by * 2 + 1], o[1][by * 2], o[1][by * 2 + 1]);
      if (kW) {
        const float4 ww = st.wr[by];
        v.x *= ww.x; v.y *= ww.y; v.z *= ww.z; v.w *= ww.w;
      }
      if (valid) st4_stream<TS>(so + fine_off(y, by), v);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) { rm[k] = r0[k]; r0[k] = st.c[k]; }
  };

  coarse_row(y0 - 1, rm);
  coarse_row(y0, r0);
  // two rows in flight: a ring of three buffers, unrolled so no buffer is copied; the
  // scheduling barriers keep each prefetch ahead of the next row's first wait
  Step sa, sb, sc2;
  load_step(y0, sa);
  load_step(y0 + 1, sb);
  for (int y = y0; y < y1; y += 3) {
    load_step(y + 2, sc2);
    __builtin_amdgcn_sched_barrier(0);
    compute_step(y, sa);
    if (y + 1 >= y1) break;
    load_step(y + 3, sa);
    __builtin_amdgcn_sched_barrier(0);
    compute_step(y + 1, sb);
    if (y + 2 >= y1) break;
    load_step(y + 4, sb);
    __builtin_amdgcn_sched_barrier(0);
    compute_step(y + 2, sc2);
  }
}

// The metric's last level both ways in one pass: M v = L^T (w * L v) + v needs, at the
// finest level, the forward block s_c = R window_c + sqrtD v_c, the weighted block
// y_c = w_c * s_c and then the adjoint of y_c, which is a function of y_c alone (plus
// the neighbouring blocks' window contributions). A lane that computes s_c can hand
// y_c straight to the adjoint arithmetic, so the weighted fine field is never stored
// and read back. The layout is the adjoint's (strips of kOwnedPairs pairs whose first
// and last lanes recompute the neighbouring strips' edge pairs, a wavefront marching
// block rows y0-1 .. y1); each block row also runs the forward: its three coarse rows
// slide in registers (one new row per block row), and the excitations of the level are
// the values v the metric adds to the excitation cotangent, loaded once for both.
// kDot: the kernel also sums <s, w * s> over the fine blocks it stores (per lane in its
// march order, a fixed butterfly over each wavefront's lanes, then the workgroup's
// wavefronts in order), the likelihood part of <v, M v> = <L v, w * L v> + <v, v>, which
// CG needs as p.q: one partial sum per workgroup.
template <typename TS, typename M, bool kDot>
__global__ void __launch_bounds__(kLanes * kWavesPerGroup) refine2_metric(Adj2Geom g, RefineMetricArgs a, M mats) {
  fetch_args(g.ny, g.nx, g.pairs, g.strips, g.ychunk, g.nfx, g.waves, a.s_in, a.s_in_bs, a.v, a.v_bs, a.w, a.w_bs,
             a.out, a.out_bs, a.s_bar, a.s_bar_bs);
  if (kDot) fetch_args(a.dot, a.dot_bs);
  if (halted(a.halt)) return;
  const int lane = threadIdx.x % kLanes;
  const int wave = blockIdx.x * kWavesPerGroup + __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
  const bool live = wave < g.waves;  // uniform per wavefront
  if (!kDot && !live) return;        // whole wavefronts leave; without kDot there is no barrier
  const int strip = wave % g.strips, chunk = wave / g.strips;
  const int P = strip * kOwnedPairs + lane - 1;  // blocks x = 2P+1, 2P+2
  const bool pair_ok = P >= 0 && P < g.pairs;
  const bool owner = lane >= 1 && lane <= kOwnedPairs && pair_ok;
  const int y0 = chunk * g.ychunk;
  const int y1 = min(y0 + g.ychunk, g.ny);
  const int64_t b = blockIdx.y;
  const TS* sc = static_cast<const TS*>(a.s_in) + b * a.s_in_bs;
  const TS* v = static_cast<const TS*>(a.v) + b * a.v_bs;
  const float* w = static_cast<const float*>(a.w) + b * a.w_bs;
  TS* out = static_cast<TS*>(a.out) + b * a.out_bs;
  TS* sb = static_cast<TS*>(a.s_bar) + b * a.s_bar_bs;
  // every load goes to an in-bounds address (clamped pair, row and block row); blocks
  // outside the interior are zeroed after the forward
  const int Pc = min(max(P, 0), g.pairs - 1);
  auto fine_off = [&](int yb, int by) { return static_cast<int64_t>(2 * (yb - 1) + by) * g.nfx + 4 * Pc; };
  auto coarse_row = [&](int y, float (&r)[4]) {
    const TS* row = sc + static_cast<int64_t>(min(max(y, 0), g.ny - 1)) * g.nx + 2 * Pc;
    const float2 u = Io<TS>::ld2(row), t = Io<TS>::ld2(row + 2);
    r[0] = u.x; r[1] = u.y; r[2] = t.x; r[3] = t.y;
  };
  // shell levels: the matrix rows of block rows y0-1 .. y1 (sets yb - 1) in LDS
  __shared__ float staged_rows[kShell2<M> ? kWavesPerGroup : 1][kShell2<M> ? kStagedRows * kRowFloats : 1];
  float* my_rows = staged_rows[kShell2<M> ? threadIdx.x / kLanes : 0];
  const bool staged = kShell2<M> && live && y1 - y0 + 2 <= kStagedRows;  // uniform per wavefront
  if constexpr (kShell2<M>) {
    if (staged) stage_rows(mats, my_rows, y0 - 2, y1 - y0 + 2, lane);
  }

  struct Step {
    float c[4];    // coarse row yb + 1, columns 2P .. 2P+3
    float4 x[2];   // v on the pair's fine rows 2(yb-1), 2(yb-1)+1
    float4 wr[2];  // w on the same rows
  };
  auto load_step = [&](int yb, Step& st) {
    coarse_row(yb + 1, st.c);
    const int yc = min(max(yb, 1), g.ny - 2);
#pragma unroll
    for (int by = 0; by < 2; ++by) {
      st.x[by] = Io<TS>::ld4(v + fine_off(yc, by));
      st.wr[by] = *reinterpret_cast<const float4*>(w + fine_off(yc, by));
    }
  };

  float rm[4], r0[4];        // coarse rows yb-1 and yb
  double dot_acc = 0.0;      // kDot
  float A0[2][3], A1[2][3];  // partial coarse cotangents of rows yb-1 and yb, per block and wx
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int x = 0; x < 3; ++x) { A0[p][x] = 0.0f; A1[p][x] = 0.0f; }

  auto process = [&](int yb, const Step& st) {
    const bool ok = pair_ok && yb >= 1 && yb <= g.ny - 2;
    float R[36], S[10];  // this block row's matrices
    if constexpr (kShell2<M>) {
      if (staged) {
        const float* lr = my_rows + (yb - (y0 - 1)) * kRowFloats;
#pragma unroll
        for (int e = 0; e < 36; ++e) R[e] = lr[e];
#pragma unroll
        for (int e = 0; e < 10; ++e) S[e] = lr[36 + e];
      } else {
        const auto row = row_of(mats, yb - 1);
#pragma unroll
        for (int e = 0; e < 36; ++e) R[e] = row[e];
#pragma unroll
        for (int e = 0; e < 10; ++e) S[e] = row[36 + e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 36; ++e) R[e] = mats.m.r[e];
#pragma unroll
      for (int e = 0; e < 10; ++e) S[e] = mats.m.s[e];
    }
    // forward and weight: yv[p][by * 2 + bx] of block 2P+1+p
    float yv[2][4], sv[2][4];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      float win[9];  // columns 2P+p .. 2P+p+2 of rows yb-1, yb, yb+1
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        win[x] = rm[p + x];
        win[3 + x] = r0[p + x];
        win[6 + x] = st.c[p + x];
      }
      float xv[4], wv[4];
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        xv[by * 2] = p == 0 ? st.x[by].x : st.x[by].z;
        xv[by * 2 + 1] = p == 0 ? st.x[by].y : st.x[by].w;
        wv[by * 2] = p == 0 ? st.wr[by].x : st.wr[by].z;
        wv[by * 2 + 1] = p == 0 ? st.wr[by].y : st.wr[by].w;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) s = fmaf(R[c * 9 + k], win[k], s);
#pragma unroll
        for (int cp = 0; cp <= c; ++cp) s = fmaf(S[sd2(c, cp)], xv[cp], s);
        sv[p][c] = s;
        yv[p][c] = ok ? s * wv[c] : 0.0f;
      }
    }
    // adjoint: excitation cotangent plus v
    if (ok && owner && yb >= y0 && yb < y1) {
      float xo[2][4];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int cp = 0; cp < 4; ++cp) {
          float t = 0.0f;
#pragma unroll
          for (int c = cp; c < 4; ++c) t = fmaf(S[sd2(c, cp)], yv[p][c], t);
          xo[p][cp] = t;
        }
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        const float4 av = st.x[by];
        const float4 o = make_float4(xo[0][by * 2] + av.x, xo[0][by * 2 + 1] + av.y, xo[1][by * 2] + av.z,
                                     xo[1][by * 2 + 1] + av.w);
        st4_stream<TS>(out + fine_off(yb, by), o);
      }
      if constexpr (kDot) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int c = 0; c < 4; ++c) dot_acc += static_cast<double>(sv[p][c]) * static_cast<double>(yv[p][c]);
      }
    }
    // window contributions, then the y march: row yb-1 is complete after this block row
    float G[2][3];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      float u[9];
#pragma unroll
      for (int wi = 0; wi < 9; ++wi) {
        float t = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) t = fmaf(R[c * 9 + wi], yv[p][c], t);
        u[wi] = t;
      }
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        G[p][x] = A0[p][x] + u[x];       // wy = -1: coarse row yb - 1
        A0[p][x] = A1[p][x] + u[3 + x];  // wy =  0: coarse row yb
        A1[p][x] = u[6 + x];             // wy = +1: coarse row yb + 1
      }
    }
    if (yb >= y0 + 1) {  // uniform over the wavefront
      const float from_left = dpp_from_left(G[1][2]);
      const float from_right = dpp_from_right(G[0][0]);
      if (owner) {
        TS* row = sb + static_cast<int64_t>(yb - 1) * g.nx;
        Io<TS>::st1(row + 2 * P + 1, from_left + G[0][1] + G[1][0]);
        Io<TS>::st1(row + 2 * P + 2, G[0][2] + G[1][1] + from_right);
        if (P == 0) Io<TS>::st1(row, G[0][0]);
        if (P == g.pairs - 1) Io<TS>::st1(row + g.nx - 1, G[1][2]);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) { rm[k] = r0[k]; r0[k] = st.c[k]; }
  };

  // block rows y0-1 .. y1; the window of block row yb is coarse rows yb-1 .. yb+1
  if (live) {
    coarse_row(y0 - 2, rm);
    coarse_row(y0 - 1, r0);
    Step sa, sb2, sc2;
    load_step(y0 - 1, sa);
    load_step(y0, sb2);
    for (int yb = y0 - 1; yb <= y1; yb += 3) {  // scheduling barriers: as in the adjoint
      load_step(yb + 2, sc2);
      __builtin_amdgcn_sched_barrier(0);
      process(yb, sa);
      if (yb + 1 > y1) break;
      load_step(yb + 3, sa);
      __builtin_amdgcn_sched_barrier(0);
      process(yb + 1, sb2);
      if (yb + 2 > y1) break;
      load_step(yb + 4, sb2);
      __builtin_amdgcn_sched_barrier(0);
      process(yb + 2, sc2);
    }
  }
  if constexpr (kDot) {
    __shared__ double red[kWavesPerGroup];
#pragma unroll
    for (int off = kLanes / 2; off > 0; off >>= 1) dot_acc += __shfl_xor(dot_acc, off, kLanes);
    if (lane == 0) red[threadIdx.x / kLanes] = dot_acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kWavesPerGroup; ++k) s += red[k];
      a.dot[b * a.dot_bs + blockIdx.x] = s;
    }
  }
}

bool aligned2(const void* p, int bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

Mat2 mat2_of(const icr_plan* p, int level) {
  const LevelMats& lm = p->lev[level];
  Mat2 m;
  for (int t = 0; t < 36; ++t) m.r[t] = lm.h_r[t];
  for (int c = 0; c < 4; ++c)
    for (int cp = 0; cp <= c; ++cp) m.s[sd2(c, cp)] = lm.h_s[c * 4 + cp];
  return m;
}

// rows per wavefront for a sweep of `rows` rows in `strips` strips. A wavefront that
// marches one row per chunk also recomputes the two halo rows (the adjoint) or loads the
// two window rows (the forward) for it, so long marches save work, while short ones
// spread the level over more SIMDs. The wavefront budget grows with the batch up to
// 16384 (16 per SIMD over 1024 SIMDs: 2-D step 0.2447 ms at 8, 0.2405 at 16, 0.252 at
// 32, 0.265 at 64 per SIMD for 1540^2 x 16); one sample gets 2048 (charted 1284^2
// metric 57.6 us against 62.0 at 16384 and 57.1 at 1024), three get 4096 (76.2 us
// against 93.7 at 16384). Levels of at most 400 rows get at most 2048 wavefronts, since
// their short marches spent much of each chunk on its two halo rows: steps of the 2-D SE
// prior at 1540^2 x 16 0.2307 ms against 0.2392 (the 388^2 -> 772^2 adjoint 19.1 against
// 27.2 us; 3072, 4096 and 6144 in between), 196^2 x 1024 407 against 428 us, x 256 116
// against 125 us, 388^2 x 64 84.5 against 91 us, 772^2 x 4 55.2 against 54.0 us; the
// charted CG step at three right-hand sides 110.0 against 112.2 us.
int pick_ychunk(int rows, int strips, int64_t batch) {
  const int64_t budget = std::min<int64_t>(rows <= 400 ? 2048 : 16384, 1024 * (batch + 1));
  int64_t chunks = budget / (int64_t(strips) * batch);
  chunks = std::max<int64_t>(1, std::min<int64_t>(chunks, rows));
  return static_cast<int>((rows + chunks - 1) / chunks);
}

template <typename TS, typename M>
hipError_t fwd2_launch(const icr_plan* p, int level, const M& m, const RefineFwdArgs& a, hipStream_t st) {
  Fwd2Geom g;
  g.ny = p->shapes[level][1];
  g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.strips = (g.pairs + kLanes - 1) / kLanes;
  g.nfx = p->shapes[level + 1][2];
  const int64_t batch = a.batch < 65535 ? a.batch : 65535;
  g.ychunk = pick_ychunk(g.ny - 2, g.strips, batch);
  const int nchunks = (g.ny - 2 + g.ychunk - 1) / g.ychunk;
  g.waves = g.strips * nchunks;
  const unsigned groups = static_cast<unsigned>((g.waves + kWavesPerGroup - 1) / kWavesPerGroup);
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineFwdArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.s_in = static_cast<const TS*>(a.s_in) + b0 * a.s_in_bs;
    c.xi = static_cast<const TS*>(a.xi) + b0 * a.xi_bs;
    c.s_out = static_cast<TS*>(a.s_out) + b0 * a.s_out_bs;
    if (a.w) c.w = static_cast<const float*>(a.w) + b0 * a.w_bs;
    const dim3 grid(groups, static_cast<unsigned>(c.batch));
    if (a.w) refine2_fwd<TS, true, M><<<grid, kLanes * kWavesPerGroup, 0, st>>>(g, c, m);
    else refine2_fwd<TS, false, M><<<grid, kLanes * kWavesPerGroup, 0, st>>>(g, c, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TS, typename M>
hipError_t adj2_launch(const icr_plan* p, int level, const M& m, const RefineAdjArgs& a, hipStream_t st) {
  Adj2Geom g;
  g.ny = p->shapes[level][1];
  g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.strips = (g.pairs + kOwnedPairs - 1) / kOwnedPairs;
  g.nfx = p->shapes[level + 1][2];
  const int64_t batch = a.batch < 65535 ? a.batch : 65535;
  g.ychunk = pick_ychunk(g.ny, g.strips, batch);
  const int nchunks = (g.ny + g.ychunk - 1) / g.ychunk;
  g.waves = g.strips * nchunks;
  const unsigned groups = static_cast<unsigned>((g.waves + kWavesPerGroup - 1) / kWavesPerGroup);
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineAdjArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.y = static_cast<const TS*>(a.y) + b0 * a.y_bs;
    c.xi_bar = static_cast<TS*>(a.xi_bar) + b0 * a.xi_bar_bs;
    c.s_bar = static_cast<TS*>(a.s_bar) + b0 * a.s_bar_bs;
    if (a.add) c.add = static_cast<const TS*>(a.add) + b0 * a.add_bs;
    const dim3 grid(groups, static_cast<unsigned>(c.batch));
    if (a.add) refine2_adj<TS, true, M><<<grid, kLanes * kWavesPerGroup, 0, st>>>(g, c, m);
    else refine2_adj<TS, false, M><<<grid, kLanes * kWavesPerGroup, 0, st>>>(g, c, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// the metric kernel's layout (the adjoint's) for `batch` samples per launch
Adj2Geom metric2_geom(const icr_plan* p, int level, int64_t batch) {
  Adj2Geom g;
  g.ny = p->shapes[level][1];
  g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.strips = (g.pairs + kOwnedPairs - 1) / kOwnedPairs;
  g.nfx = p->shapes[level + 1][2];
  g.ychunk = pick_ychunk(g.ny, g.strips, batch < 65535 ? batch : 65535);
  const int nchunks = (g.ny + g.ychunk - 1) / g.ychunk;
  g.waves = g.strips * nchunks;
  return g;
}

template <typename TS, typename M>
hipError_t metric2_launch(const icr_plan* p, int level, const M& m, const RefineMetricArgs& a, hipStream_t st) {
  const Adj2Geom g = metric2_geom(p, level, a.batch);
  const unsigned groups = static_cast<unsigned>((g.waves + kWavesPerGroup - 1) / kWavesPerGroup);
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineMetricArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.s_in = static_cast<const TS*>(a.s_in) + b0 * a.s_in_bs;
    c.v = static_cast<const TS*>(a.v) + b0 * a.v_bs;
    c.w = static_cast<const float*>(a.w) + b0 * a.w_bs;
    c.out = static_cast<TS*>(a.out) + b0 * a.out_bs;
    c.s_bar = static_cast<TS*>(a.s_bar) + b0 * a.s_bar_bs;
    if (a.dot) c.dot = a.dot + b0 * a.dot_bs;
    const dim3 grid(groups, static_cast<unsigned>(c.batch));
    if (a.dot) refine2_metric<TS, M, true><<<grid, kLanes * kWavesPerGroup, 0, st>>>(g, c, m);
    else refine2_metric<TS, M, false><<<grid, kLanes * kWavesPerGroup, 0, st>>>(g, c, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TS>
hipError_t metric2_any(const icr_plan* p, int level, const RefineMetricArgs& a, hipStream_t st) {
  if (p->shell)
    return metric2_launch<TS>(p, level, Shell2{p->lev[level].shell_tab, static_cast<int>(p->lev[level].nsets)}, a, st);
  return metric2_launch<TS>(p, level, Stat2{mat2_of(p, level)}, a, st);
}

template <typename TS>
hipError_t fwd2_any(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st) {
  if (p->shell) return fwd2_launch<TS>(p, level, Shell2{p->lev[level].shell_tab, static_cast<int>(p->lev[level].nsets)}, a, st);
  return fwd2_launch<TS>(p, level, Stat2{mat2_of(p, level)}, a, st);
}
template <typename TS>
hipError_t adj2_any(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st) {
  if (p->shell) return adj2_launch<TS>(p, level, Shell2{p->lev[level].shell_tab, static_cast<int>(p->lev[level].nsets)}, a, st);
  return adj2_launch<TS>(p, level, Stat2{mat2_of(p, level)}, a, st);
}

// Stationary or shell-charted 2-D levels in FP32 arithmetic with an even coarse row
// length; everything else takes the generic kernels. Slices off a vector boundary (a
// level-0 size that is not a multiple of 4) run the same kernels with element accesses.
bool eligible2(const icr_plan* p, int level) {
  if (p->ndim != 2 || p->precision == ICR_F64) return false;
  if (p->charted && !(p->shell && p->lev[level].shell_tab)) return false;
  const int nx = p->shapes[level][2];
  if (nx % 2 != 0 || nx < 4) return false;
  const int64_t nf = int64_t(p->shapes[level + 1][1]) * p->shapes[level + 1][2];
  return nf < (int64_t(1) << 31);
}

}  // namespace

bool try_refine2_fwd(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st, hipError_t* err) {
  if (!eligible2(p, level)) return false;
  const int el = p->elem_bytes;
  if (!aligned2(a.xi, el) || !aligned2(a.s_out, el) || !aligned2(a.s_in, el)) return false;
  if (a.w && (!aligned2(a.w, 16) || a.w_bs % 4)) return false;
  const bool vec_ok = aligned2(a.xi, 4 * el) && aligned2(a.s_out, 4 * el) && aligned2(a.s_in, 2 * el) &&
                      a.xi_bs % 4 == 0 && a.s_out_bs % 4 == 0 && a.s_in_bs % 2 == 0;
  if (p->precision == ICR_F32)
    *err = vec_ok ? fwd2_any<float>(p, level, a, st) : fwd2_any<f32u>(p, level, a, st);
  else
    *err = vec_ok ? fwd2_any<bf16_t>(p, level, a, st) : fwd2_any<bf16u>(p, level, a, st);
  return true;
}

bool try_refine2_adj(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st, hipError_t* err) {
  if (!eligible2(p, level)) return false;
  const int el = p->elem_bytes;
  const int vec = 4 * el;
  if (!aligned2(a.y, el) || !aligned2(a.xi_bar, el) || !aligned2(a.s_bar, el) || (a.add && !aligned2(a.add, el)))
    return false;
  const bool vec_ok = aligned2(a.y, vec) && aligned2(a.xi_bar, vec) && (!a.add || aligned2(a.add, vec)) &&
                      a.y_bs % 4 == 0 && a.xi_bar_bs % 4 == 0 && (!a.add || a.add_bs % 4 == 0);
  if (p->precision == ICR_F32)
    *err = vec_ok ? adj2_any<float>(p, level, a, st) : adj2_any<f32u>(p, level, a, st);
  else
    *err = vec_ok ? adj2_any<bf16_t>(p, level, a, st) : adj2_any<bf16u>(p, level, a, st);
  return true;
}

// the metric level's vector accesses are aligned (else it runs with element accesses)
static bool metric2_vec_ok(const icr_plan* p, const RefineMetricArgs& a) {
  const int el = p->elem_bytes;
  return aligned2(a.v, 4 * el) && aligned2(a.out, 4 * el) && aligned2(a.s_in, 2 * el) && a.v_bs % 4 == 0 &&
         a.out_bs % 4 == 0 && a.s_in_bs % 2 == 0;
}

bool refine2_metric_ok(const icr_plan* p, int level, const RefineMetricArgs& a) {
  if (!eligible2(p, level)) return false;
  const int el = p->elem_bytes;
  if (!aligned2(a.v, el) || !aligned2(a.out, el) || !aligned2(a.s_in, el) || !aligned2(a.s_bar, el)) return false;
  return aligned2(a.w, 16) && a.w_bs % 4 == 0;
}

int64_t refine2_metric_partials(const icr_plan* p, int level, int64_t batch) {
  return (metric2_geom(p, level, batch).waves + kWavesPerGroup - 1) / kWavesPerGroup;
}

hipError_t launch_refine2_metric(const icr_plan* p, int level, const RefineMetricArgs& a, hipStream_t st) {
  const bool vec_ok = metric2_vec_ok(p, a);
  if (p->precision == ICR_F32) return vec_ok ? metric2_any<float>(p, level, a, st) : metric2_any<f32u>(p, level, a, st);
  return vec_ok ? metric2_any<bf16_t>(p, level, a, st) : metric2_any<bf16u>(p, level, a, st);
}

}  // namespace icr
