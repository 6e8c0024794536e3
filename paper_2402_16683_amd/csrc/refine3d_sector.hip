// 3-D refinement level in the reflection-sector basis, FP32 arithmetic with FP32 or
// bfloat16 storage, for stationary levels whose R is reflection-symmetric, and for
// shell-charted levels (one R per coarse plane along z) whose R is symmetric under
// reflecting y and x: there z stays dense and each plane reads its own coefficients.
//
// R = B C P (see sector_kernel in build_f64.hip): P takes each axis of the 3x3x3
// window to even/odd channels (e, m, o) = (s_-1 + s_+1, s_0, s_+1 - s_-1), C has
// one coefficient per channel t = (tz, ty, tx) feeding sector sigma(t) (S on axes
// where t is e or m, D where t is o), and B is the per-axis butterfly
// o_0 = S - D, o_1 = S + D. A block costs 27 multiplies plus butterflies instead of
// the 216 multiply-adds of the dense 8 x 27 R. The transpose is R^T = P^T C^T Q
// with Q the per-axis (S, D) = (y_0 + y_1, y_1 - y_0) and P^T sending
// (e, m, o) to the window slots (-1, 0, +1) as (e - o, m, e + o).
//
// Forward: one thread per pair of neighbouring interior coarse pixels along x
// (x = 2q+1, 2q+2), marching along z. The 2 x 2 x 2 children of the pair fill four
// 16-byte fine rows, so excitations and outputs stream as full vectors. Coarse
// windows come through the cache (the coarse level is 1/8 of the fine one); the x
// and y even/odd stages of each coarse plane are computed once and slide along z.
//
// Adjoint (a gather, no atomics): each block's cotangent y is mapped to sectors
// (Q), scaled per channel (C^T) and sent back through P^T one axis at a time. The
// z stage accumulates in registers while marching along z; the x stage takes the
// neighbouring pairs' contributions from the adjacent lanes (DPP), the y stage from
// the neighbouring rows through LDS, inside a tile of block pairs whose outer ring
// (halo) is recomputed by each tile.
// Every coarse cotangent is summed by one thread in a fixed order.
#include <algorithm>
#include <type_traits>

#include "icr_internal.h"
#include "sweep_io.h"

namespace icr {
namespace {

using namespace sweep;

// sector coefficients C (27, already divided by 8) and the lower sqrtD packed by rows
struct Sector3 {
  float c[27];
  float s[36];
};

__device__ __forceinline__ int sd(int b, int bp) { return b * (b + 1) / 2 + bp; }

// The matrices the kernels apply to the blocks of a coarse plane. A stationary level
// passes its one sector set by value. A shell-charted level (one set per coarse plane
// along z, where R keeps the reflection symmetry of y and x only) passes a table with
// one row per plane: C[ty tx][bz][wz] (z dense, y and x in sector form) and sqrtD.
struct StationaryMats {
  Sector3 k;
};
struct ShellMats {
  const float* tab;  // [nz - 2][kShellStride]: C[ty tx][bz][wz] (54), sqrtD lower by rows (36), padding
  int nsets;
};
// A plane's row is the same for every lane of a workgroup (all lanes march through
// the same planes): read it through the constant address space, which lets the
// compiler use scalar loads (the table is never written while a sweep runs).
typedef const float __attribute__((address_space(4))) const_float;
template <typename M>
__device__ __forceinline__ const const_float* shell_row(const M& m, int set) {
  return (const const_float*)(m.tab + static_cast<int64_t>(set) * kShellStride);
}
// The gradient contraction's matrices: the length derivatives of the level in the same
// form, plus the value sqrtD (its product with the excitations gives the scale term).
struct DotStationary {
  Sector3 k;      // derivative: sector coefficients of dR, dsqrtD
  float sv[36];   // value sqrtD, lower by rows
};
struct DotShell {
  const float* tab;   // derivative table (rows as in ShellMats)
  int nsets;
  const float* vtab;  // value table
};
template <typename M>
constexpr bool kIsShell = false;
template <>
constexpr bool kIsShell<ShellMats> = true;
template <>
constexpr bool kIsShell<DotShell> = true;

// The four coarse values x = 2q .. 2q+3 of rows y-1, y, y+1 of one plane.
struct Raw3 {
  float2 a[3], b[3];
};
template <typename TS>
__device__ __forceinline__ Raw3 plane_load(const TS* __restrict__ plane, int y, int nx, int q) {
  Raw3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const TS* row = plane + static_cast<int64_t>(y - 1 + i) * nx + 2 * q;
    r.a[i] = Io<TS>::ld2(row);
    r.b[i] = Io<TS>::ld2(row + 2);
  }
  return r;
}

// x and y even/odd stages of one coarse plane for the pixel pair (2q+1, 2q+2):
// T[k][ty * 3 + tx], channels e, m, o = 0, 1, 2.
__device__ __forceinline__ void plane_stage(const Raw3& raw, float (&T)[2][9]) {
  float X[3][2][3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float2 a = raw.a[r], b = raw.b[r];
    X[r][0][0] = a.x + b.x; X[r][0][1] = a.y; X[r][0][2] = b.x - a.x;
    X[r][1][0] = a.y + b.y; X[r][1][1] = b.x; X[r][1][2] = b.y - a.y;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int tx = 0; tx < 3; ++tx) {
      T[k][tx] = X[0][k][tx] + X[2][k][tx];
      T[k][3 + tx] = X[1][k][tx];
      T[k][6 + tx] = X[2][k][tx] - X[0][k][tx];
    }
}

// z stage, sector sums and butterflies of one block: out[bz*4 + by*2 + bx]
__device__ __forceinline__ void sector_forward(const float (&T0)[9], const float (&T1)[9],
                                               const float (&T2)[9], const Sector3& k, float (&out)[8]) {
  float Y[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) Y[s] = 0.0f;
#pragma unroll
  for (int tz = 0; tz < 3; ++tz)
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const float v = tz == 0 ? T0[j] + T2[j] : (tz == 1 ? T1[j] : T2[j] - T0[j]);
      const int sg = ((tz == 2) << 2) | ((j / 3 == 2) << 1) | (j % 3 == 2);
      Y[sg] = fmaf(k.c[tz * 9 + j], v, Y[sg]);
    }
  float A[8], Bv[8];
#pragma unroll
  for (int h = 0; h < 4; ++h) {  // x: (sz, sy, sx) -> (sz, sy, bx)
    A[2 * h] = Y[2 * h] - Y[2 * h + 1];
    A[2 * h + 1] = Y[2 * h] + Y[2 * h + 1];
  }
#pragma unroll
  for (int sz = 0; sz < 2; ++sz)  // y: (sz, sy, bx) -> (sz, by, bx)
#pragma unroll
    for (int bx = 0; bx < 2; ++bx) {
      Bv[sz * 4 + bx] = A[sz * 4 + bx] - A[sz * 4 + 2 + bx];
      Bv[sz * 4 + 2 + bx] = A[sz * 4 + bx] + A[sz * 4 + 2 + bx];
    }
#pragma unroll
  for (int h = 0; h < 4; ++h) {  // z: (sz, by, bx) -> (bz, by, bx)
    out[h] = Bv[h] - Bv[4 + h];
    out[4 + h] = Bv[h] + Bv[4 + h];
  }
}

// Shell-charted block: y and x in sector form, z dense. Y[bz][sy sx] collects, per
// window channel (ty, tx), the three window planes with that plane's coefficients;
// the y and x butterflies then give out[bz*4 + by*2 + bx].
template <typename P>
__device__ __forceinline__ void shell_forward(const float (&T0)[9], const float (&T1)[9],
                                              const float (&T2)[9], P c, float (&out)[8]) {
  float Y[2][4];
#pragma unroll
  for (int bz = 0; bz < 2; ++bz)
#pragma unroll
    for (int s = 0; s < 4; ++s) Y[bz][s] = 0.0f;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const int sg = ((j / 3 == 2) << 1) | (j % 3 == 2);
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
      Y[bz][sg] = fmaf(c[j * 6 + bz * 3], T0[j],
                       fmaf(c[j * 6 + bz * 3 + 1], T1[j], fmaf(c[j * 6 + bz * 3 + 2], T2[j], Y[bz][sg])));
  }
#pragma unroll
  for (int bz = 0; bz < 2; ++bz) {
    float A[2][2];
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {  // x: (sy, sx) -> (sy, bx)
      A[sy][0] = Y[bz][sy * 2] - Y[bz][sy * 2 + 1];
      A[sy][1] = Y[bz][sy * 2] + Y[bz][sy * 2 + 1];
    }
#pragma unroll
    for (int bx = 0; bx < 2; ++bx) {  // y: (sy, bx) -> (by, bx)
      out[bz * 4 + bx] = A[0][bx] - A[1][bx];
      out[bz * 4 + 2 + bx] = A[0][bx] + A[1][bx];
    }
  }
}

struct Fwd3Geom {
  int nz, ny, nx;  // coarse shape
  int pairs;       // (nx - 2) / 2 pixel pairs per interior row
  int rows;        // ny - 2 interior rows
  int zchunk;      // interior coarse planes per workgroup
  int nfy, nfx;    // fine rows per plane, fine row length
  int xy_blocks;   // workgroups per chunk of planes
  int nwg;         // workgroups per sample
};

// The z loop is unrolled by two with ping-pong load buffers, and every load goes to a
// clamped in-bounds address: loaded registers are never copied or loaded under a
// branch, so the next step's loads stay in flight while the current step computes.
// kDot: the gradient contraction. The kernel applies the level's derivative matrices
// and, instead of storing the fine block, adds <cotangent block, block> to an FP64 sum
// per lane (in z order), and <cotangent block, value sqrtD xi block> to a second one;
// both are reduced over the workgroup by a fixed tree.
template <typename TS, bool kW, typename M, bool kDot = false>
__global__ void __launch_bounds__(256) refine3_fwd_sector(Fwd3Geom g, RefineFwdArgs a, M m) {
  fetch_args(g.nz, g.ny, g.nx, g.pairs, g.rows, g.zchunk, g.nfy, g.nfx, g.xy_blocks, a.s_in, a.s_in_bs, a.xi,
             a.xi_bs, a.s_out, a.s_out_bs);
  if (kW) fetch_args(a.w, a.w_bs);
  if (kDot) fetch_args(a.dot, a.dot_bs, a.partial, a.partial_bs, a.partial_sig);
  if constexpr (kIsShell<M>) fetch_args(m.tab);
  if (halted(a.halt)) return;
  const int tile = static_cast<int>(blockIdx.x);
  // Within each chunk of planes the 8 XCDs (workgroups go to them round-robin) each take
  // a contiguous band of xy blocks, so the coarse rows that neighbouring blocks share are
  // read into one L2; all XCDs still work on the same chunk, keeping DRAM accesses close.
  const int chunk = tile / g.xy_blocks;
  int xy;
  {
    const int r = tile - chunk * g.xy_blocks;
    const int xcd = tile & (kXcds - 1);
    const int shift = (chunk * g.xy_blocks) & (kXcds - 1);  // xcd of the chunk's block r is (shift + r) mod 8
    int start = 0;
    for (int x = 0; x < xcd; ++x) {
      const int r0 = (x - shift) & (kXcds - 1);
      start += r0 < g.xy_blocks ? (g.xy_blocks - r0 + kXcds - 1) / kXcds : 0;
    }
    const int r0 = (xcd - shift) & (kXcds - 1);
    xy = start + (r - r0) / kXcds;
  }
  // no early exit: threads past the last pair work on the last pair and store nothing,
  // so every kernel argument can be fetched in one round at the start (an exit branch
  // made the pointer loads wait for the geometry loads)
  const int tid_raw = xy * 256 + threadIdx.x;
  const bool valid = tid_raw < g.rows * g.pairs;
  const int tid = valid ? tid_raw : g.rows * g.pairs - 1;
  const int yi = tid / g.pairs;
  const int q = tid - yi * g.pairs;
  const int y = yi + 1;
  const int zb = 1 + chunk * g.zchunk;
  const int ze = min(zb + g.zchunk, g.nz - 1);
  const int64_t b = blockIdx.y;
  const TS* sc = static_cast<const TS*>(a.s_in) + b * a.s_in_bs;
  const TS* xi = static_cast<const TS*>(a.xi) + b * a.xi_bs;
  TS* so = static_cast<TS*>(a.s_out) + b * a.s_out_bs;
  const float* w = kW ? static_cast<const float*>(a.w) + b * a.w_bs : nullptr;
  const TS* cot = kDot ? static_cast<const TS*>(a.dot) + b * a.dot_bs : nullptr;
  double dot_acc = 0.0, sig_acc = 0.0;
  const int64_t cplane = static_cast<int64_t>(g.ny) * g.nx;
  const int64_t fplane = static_cast<int64_t>(g.nfy) * g.nfx;
  const int64_t frow = static_cast<int64_t>(2 * (y - 1)) * g.nfx + 4 * q;

  struct Step {
    Raw3 raw;            // coarse plane z + 1
    float4 xr[2][2];     // excitations of the pair's children in plane z
    float4 wr[2][2];     // metric weights (kW) or the cotangent rows (kDot)
  };
  auto fine_off = [&](int z, int bz, int by) {
    return (2 * (z - 1) + bz) * fplane + frow + by * g.nfx;
  };
  auto load_step = [&](int z, Step& st) {
    const int zc = min(z, ze - 1);
    st.raw = plane_load<TS>(sc + (zc + 1) * cplane, y, g.nx, q);
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        st.xr[bz][by] = ld4_stream<TS>(xi + fine_off(zc, bz, by));
        if (kW) st.wr[bz][by] = *reinterpret_cast<const float4*>(w + fine_off(zc, bz, by));
        if (kDot) st.wr[bz][by] = ld4_stream<TS>(cot + fine_off(zc, bz, by));
      }
  };
  float T0[2][9], T1[2][9], T2[2][9];
  auto compute_step = [&](int z, const Step& st) {
    plane_stage(st.raw, T2);
    float o[2][8];
    float u[2][8];  // kDot: value sqrtD times the excitations
    float S[36];
    if constexpr (kIsShell<M>) {
      const auto c = shell_row(m, z - 1);
      shell_forward(T0[0], T1[0], T2[0], c, o[0]);
      shell_forward(T0[1], T1[1], T2[1], c, o[1]);
#pragma unroll
      for (int e = 0; e < 36; ++e) S[e] = c[54 + e];
    } else {
      sector_forward(T0[0], T1[0], T2[0], m.k, o[0]);
      sector_forward(T0[1], T1[1], T2[1], m.k, o[1]);
#pragma unroll
      for (int e = 0; e < 36; ++e) S[e] = m.k.s[e];
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      float x[8];
#pragma unroll
      for (int bz = 0; bz < 2; ++bz)
#pragma unroll
        for (int by = 0; by < 2; ++by) {
          x[bz * 4 + by * 2] = p == 0 ? st.xr[bz][by].x : st.xr[bz][by].z;
          x[bz * 4 + by * 2 + 1] = p == 0 ? st.xr[bz][by].y : st.xr[bz][by].w;
        }
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int cp = 0; cp <= c; ++cp) o[p][c] = fmaf(S[sd(c, cp)], x[cp], o[p][c]);
      if constexpr (kDot) {
        float Sv[36];
        if constexpr (kIsShell<M>) {
          const const_float* vr = (const const_float*)(m.vtab + static_cast<int64_t>(z - 1) * kShellStride);
#pragma unroll
          for (int e = 0; e < 36; ++e) Sv[e] = vr[54 + e];
        } else {
#pragma unroll
          for (int e = 0; e < 36; ++e) Sv[e] = m.sv[e];
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          float v = 0.0f;
#pragma unroll
          for (int cp = 0; cp <= c; ++cp) v = fmaf(Sv[sd(c, cp)], x[cp], v);
          u[p][c] = v;
        }
      }
    }
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        const int h = bz * 4 + by * 2;
        float4 v = make_float4(o[0][h], o[0][h + 1], o[1][h], o[1][h + 1]);
        if (kW) {
          const float4 ww = st.wr[bz][by];
          v.x *= ww.x; v.y *= ww.y; v.z *= ww.z; v.w *= ww.w;
        }
        if (kDot) {
          const float4 cv = st.wr[bz][by];
          if (valid) {
            dot_acc += (double(cv.x) * v.x + double(cv.y) * v.y) + (double(cv.z) * v.z + double(cv.w) * v.w);
            sig_acc += (double(cv.x) * u[0][h] + double(cv.y) * u[0][h + 1]) +
                       (double(cv.z) * u[1][h] + double(cv.w) * u[1][h + 1]);
          }
        } else if (valid) {
          st4_stream<TS>(so + fine_off(z, bz, by), v);
        }
      }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int j = 0; j < 9; ++j) { T0[p][j] = T1[p][j]; T1[p][j] = T2[p][j]; }
  };

  plane_stage(plane_load<TS>(sc + (zb - 1) * cplane, y, g.nx, q), T0);
  plane_stage(plane_load<TS>(sc + zb * cplane, y, g.nx, q), T1);
  // two steps in flight: a ring of three buffers, unrolled so no buffer is copied
  Step sa, sb2, sc2;
  load_step(zb, sa);
  load_step(zb + 1, sb2);
  // The scheduling barriers keep each prefetch ahead of the next step's first wait: the
  // loop header is also entered from the prologue, and with the prefetch sunk below the
  // wait the two paths merge into a wait for every outstanding access (loads and stores
  // share one counter), which drains the pipeline once per unrolled body.
  for (int z = zb; z < ze; z += 3) {
    load_step(z + 2, sc2);
    __builtin_amdgcn_sched_barrier(0);
    compute_step(z, sa);
    if (z + 1 >= ze) break;
    load_step(z + 3, sa);
    __builtin_amdgcn_sched_barrier(0);
    compute_step(z + 1, sb2);
    if (z + 2 >= ze) break;
    load_step(z + 4, sb2);
    __builtin_amdgcn_sched_barrier(0);
    compute_step(z + 2, sc2);
  }
  if constexpr (kDot) {  // fixed-order trees over the workgroup
    __shared__ double red[2][256];
    red[0][threadIdx.x] = dot_acc;
    red[1][threadIdx.x] = sig_acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (static_cast<int>(threadIdx.x) < s) {
        red[0][threadIdx.x] += red[0][threadIdx.x + s];
        red[1][threadIdx.x] += red[1][threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      a.partial[b * a.partial_bs + blockIdx.x] = red[0][0];
      a.partial_sig[b * a.partial_bs + blockIdx.x] = red[1][0];
    }
  }
}

// ----------------------------------------------------------------------------- adjoint


struct Adj3Geom {
  int nz, ny, nx;   // coarse shape
  int pairs;        // (nx - 2) / 2 block pairs per row
  int xtiles;       // tiles along x
  int zchunk;       // coarse planes per workgroup
  int nfy, nfx;
  int xy_tiles;     // tiles per chunk of planes
  int nwg;          // workgroups per sample
};

// Tile: kTP block pairs (x) by kTR block rows (y), halo ring included.
template <typename TS, bool kAdd, int kTP, int kTR, typename M>
__global__ void __launch_bounds__(kTP * kTR) refine3_adj_sector(Adj3Geom g, RefineAdjArgs a, M m) {
  constexpr int kOP = kTP - 2;     // owned pairs per tile (first and last lane of a row are halo)
  constexpr int kOR = kTR - 2;     // owned rows per tile
  constexpr int kAdjThreads = kTP * kTR;
  static_assert(64 % kTP == 0, "tile rows of lanes must not straddle wavefronts");
  // stationary levels: two coarse planes per barrier, sets alternating by plane pair;
  // shell levels: one plane per barrier (their coefficient ring refills behind each)
  constexpr int kPair = kIsShell<M> ? 1 : 2;
  __shared__ float ldy[2][kPair][8][kAdjThreads];
  // shell levels: the coefficient rows of block planes zb .. zb+3 in a ring (slot zb & 3);
  // read from LDS, the rows do not compete for the scalar registers
  __shared__ float coef_ring[kIsShell<M> ? 4 : 1][kShellStride];
  fetch_args(g.nz, g.ny, g.nx, g.pairs, g.xtiles, g.zchunk, g.nfy, g.nfx, g.xy_tiles, g.nwg, a.y, a.y_bs, a.xi_bar,
             a.xi_bar_bs, a.s_bar, a.s_bar_bs);
  if (halted(a.halt)) return;  // uniform over the workgroup: no barrier is left waiting
  if (kAdd) fetch_args(a.add, a.add_bs);
  if constexpr (kIsShell<M>) fetch_args(m.tab, m.nsets);
  const int t = threadIdx.x;
  const int i = t % kTP, j = t / kTP;
  const int tile = xcd_tile(blockIdx.x, g.nwg);
  const int xy = tile % g.xy_tiles;
  const int xt = xy % g.xtiles, yt = xy / g.xtiles;
  const int P = xt * kOP + i - 1;      // block pair: blocks x = 2P+1, 2P+2
  const int yb = yt * kOR + j - 1;     // block row = coarse row
  const int z0 = (tile / g.xy_tiles) * g.zchunk;
  const int z1 = min(z0 + g.zchunk, g.nz);
  const int64_t b = blockIdx.y;
  const bool pair_ok = P >= 0 && P < g.pairs;
  const bool blocks_ok = pair_ok && yb >= 1 && yb <= g.ny - 2;
  const bool owner = i >= 1 && i <= kOP && j >= 1 && j <= kOR && pair_ok && yb >= 0 && yb < g.ny;
  const TS* y = static_cast<const TS*>(a.y) + b * a.y_bs;
  TS* xb = static_cast<TS*>(a.xi_bar) + b * a.xi_bar_bs;
  TS* sb = static_cast<TS*>(a.s_bar) + b * a.s_bar_bs;
  const TS* add = kAdd ? static_cast<const TS*>(a.add) + b * a.add_bs : nullptr;
  // loads always use an in-bounds address (clamped block coordinates); blocks outside
  // the interior are zeroed after the load
  const int Pc = min(max(P, 0), g.pairs - 1);
  const int ybc = min(max(yb, 1), g.ny - 2);
  const int64_t fplane = static_cast<int64_t>(g.nfy) * g.nfx;
  const int64_t frow = static_cast<int64_t>(2 * (ybc - 1)) * g.nfx + 4 * Pc;
  auto fine_off = [&](int zc, int bz, int by) { return (2 * (zc - 1) + bz) * fplane + frow + by * g.nfx; };

  struct Plane {
    float4 r[2][2];   // cotangent rows of the pair's blocks
    float4 v[2][2];   // metric: values added to xi_bar (kAdd)
  };
  auto load_plane_y = [&](int zb, Plane& pl) {
    const int zc = min(max(zb, 1), g.nz - 2);
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        pl.r[bz][by] = Io<TS>::ld4(y + fine_off(zc, bz, by));
        if (kAdd) pl.v[bz][by] = Io<TS>::ld4(add + fine_off(zc, bz, by));
      }
  };

  float A0[2][9], A1[2][9];
  float pCy[4], pUp[4], pDn[4];  // pair mode: the y-stage values of the pending even plane
  auto store_row = [&](int zc, const float (&cy)[4], int set, int q) {
    if (owner) {  // owner rows have both neighbour rows inside the tile
      float sv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) sv[c] = cy[c] + ldy[set][q][c][t - kTP] + ldy[set][q][4 + c][t + kTP];
      TS* row = sb + (static_cast<int64_t>(zc) * g.ny + yb) * g.nx;
      Io<TS>::st1(row + 2 * P + 1, sv[0]);
      Io<TS>::st1(row + 2 * P + 2, sv[1]);
      if (P == 0) Io<TS>::st1(row, sv[2]);
      if (P == g.pairs - 1) Io<TS>::st1(row + g.nx - 1, sv[3]);
    }
  };
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int h = 0; h < 9; ++h) { A0[p][h] = 0.0f; A1[p][h] = 0.0f; }

  auto process = [&](int zb, const Plane& pl) {
    const bool ok = blocks_ok && zb >= 1 && zb <= g.nz - 2;
    float S[36];
    const float* cz = nullptr;  // shell: this block plane's row in the LDS ring
    float pre = 0.0f;           // shell: a value of the row for block plane zb + 2
    if constexpr (kIsShell<M>) {
      if (t < kShellStride) pre = m.tab[static_cast<int64_t>(min(max(zb + 1, 0), m.nsets - 1)) * kShellStride + t];
      cz = coef_ring[zb & 3];
#pragma unroll
      for (int e = 0; e < 36; ++e) S[e] = cz[54 + e];
    } else {
#pragma unroll
      for (int e = 0; e < 36; ++e) S[e] = m.k.s[e];
    }
    float yv[2][8];
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        const float4 r = pl.r[bz][by];
        yv[0][bz * 4 + by * 2] = ok ? r.x : 0.0f;
        yv[0][bz * 4 + by * 2 + 1] = ok ? r.y : 0.0f;
        yv[1][bz * 4 + by * 2] = ok ? r.z : 0.0f;
        yv[1][bz * 4 + by * 2 + 1] = ok ? r.w : 0.0f;
      }
    if (ok && owner && zb >= z0 && zb < z1) {
      float xo[2][8];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int cp = 0; cp < 8; ++cp) {
          float v = 0.0f;
#pragma unroll
          for (int c = cp; c < 8; ++c) v = fmaf(S[sd(c, cp)], yv[p][c], v);
          xo[p][cp] = v;
        }
#pragma unroll
      for (int bz = 0; bz < 2; ++bz)
#pragma unroll
        for (int by = 0; by < 2; ++by) {
          const int h = bz * 4 + by * 2;
          float4 v = make_float4(xo[0][h], xo[0][h + 1], xo[1][h], xo[1][h + 1]);
          if (kAdd) {
            const float4 av = pl.v[bz][by];
            v.x += av.x; v.y += av.y; v.z += av.z; v.w += av.w;
          }
          Io<TS>::st4(xb + fine_off(zb, bz, by), v);
        }
    }
    // sectors (Q), channels (C^T) and the z stage of P^T
    float G[2][9];
    if constexpr (kIsShell<M>) {
      // y and x sectors per z child, then per channel (ty, tx) the three window planes
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        float Ys[2][4];
#pragma unroll
        for (int bz = 0; bz < 2; ++bz) {
          const float* y = yv[p] + bz * 4;
          const float sx0 = y[0] + y[1], dx0 = y[1] - y[0], sx1 = y[2] + y[3], dx1 = y[3] - y[2];
          Ys[bz][0] = sx0 + sx1;
          Ys[bz][1] = dx0 + dx1;
          Ys[bz][2] = sx1 - sx0;
          Ys[bz][3] = dx1 - dx0;
        }
#pragma unroll
        for (int jj = 0; jj < 9; ++jj) {
          const int sg = ((jj / 3 == 2) << 1) | (jj % 3 == 2);
          const float u0 = fmaf(cz[jj * 6], Ys[0][sg], cz[jj * 6 + 3] * Ys[1][sg]);      // slot z-1
          const float u1 = fmaf(cz[jj * 6 + 1], Ys[0][sg], cz[jj * 6 + 4] * Ys[1][sg]);  // slot 0
          const float u2 = fmaf(cz[jj * 6 + 2], Ys[0][sg], cz[jj * 6 + 5] * Ys[1][sg]);  // slot z+1
          G[p][jj] = A0[p][jj] + u0;
          A0[p][jj] = A1[p][jj] + u1;
          A1[p][jj] = u2;
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        float A[8], Bv[8], Ys[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {  // z: (bz, by, bx) -> (sz, by, bx)
          A[h] = yv[p][h] + yv[p][4 + h];
          A[4 + h] = yv[p][4 + h] - yv[p][h];
        }
#pragma unroll
        for (int sz = 0; sz < 2; ++sz)  // y
#pragma unroll
          for (int bx = 0; bx < 2; ++bx) {
            Bv[sz * 4 + bx] = A[sz * 4 + bx] + A[sz * 4 + 2 + bx];
            Bv[sz * 4 + 2 + bx] = A[sz * 4 + 2 + bx] - A[sz * 4 + bx];
          }
#pragma unroll
        for (int h = 0; h < 4; ++h) {  // x
          Ys[2 * h] = Bv[2 * h] + Bv[2 * h + 1];
          Ys[2 * h + 1] = Bv[2 * h + 1] - Bv[2 * h];
        }
#pragma unroll
        for (int jj = 0; jj < 9; ++jj) {
          const int sy = jj / 3 == 2, sx = jj % 3 == 2;
          const float ue = m.k.c[jj] * Ys[(sy << 1) | sx];
          const float um = m.k.c[9 + jj] * Ys[(sy << 1) | sx];
          const float uo = m.k.c[18 + jj] * Ys[4 | (sy << 1) | sx];
          G[p][jj] = A0[p][jj] + (ue - uo);   // window slot z-1 of this block: coarse zb-1
          A0[p][jj] = A1[p][jj] + um;          // slot 0: coarse zb
          A1[p][jj] = ue + uo;                 // slot z+1: coarse zb+1
        }
      }
    }
    if (zb >= z0 + 1) {  // coarse plane zb - 1 is complete in G (uniform branch)
      const int zc = zb - 1;
      const int buf = zc & 1;  // one-plane mode
      // x stage: the pair sums its coarse columns x = 2P+1, 2P+2 from its own blocks and
      // the outer column of each neighbouring pair (the adjacent lanes, read with DPP
      // wave shifts); the first and last pairs also sum the edge columns x = 0 and nx-1.
      float H[4][3];
#pragma unroll
      for (int ty = 0; ty < 3; ++ty) {
        const float e0 = G[0][ty * 3], m0 = G[0][ty * 3 + 1], o0 = G[0][ty * 3 + 2];
        const float e1 = G[1][ty * 3], m1 = G[1][ty * 3 + 1], o1 = G[1][ty * 3 + 2];
        const float l0 = e0 - o0, r0 = e0 + o0;   // to the columns left / right of block 0
        const float l1 = e1 - o1, r1 = e1 + o1;   // and of block 1
        const float from_left = dpp_from_left(r1);    // x = 2P+1 from block 2P (left pair)
        const float from_right = dpp_from_right(l0);  // x = 2P+2 from block 2P+3 (right pair)
        H[0][ty] = from_left + m0 + l1;              // x = 2P+1
        H[1][ty] = r0 + m1 + from_right;             // x = 2P+2
        H[2][ty] = P == 0 ? l0 : 0.0f;               // x = 0
        H[3][ty] = P == g.pairs - 1 ? r1 : 0.0f;     // x = nx-1
      }
      // y stage through LDS
      float Cy[4], up[4], dn[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Cy[c] = H[c][1];
        up[c] = H[c][0] + H[c][2];  // to row yb + 1
        dn[c] = H[c][0] - H[c][2];  // to row yb - 1
      }
      if constexpr (kPair == 1) {
        // the buffer alternates with the plane, so one barrier per plane separates this
        // plane's writes from its reads and from the next plane's writes
#pragma unroll
        for (int c = 0; c < 4; ++c) { ldy[buf][0][c][t] = up[c]; ldy[buf][0][4 + c][t] = dn[c]; }
        __syncthreads();
        // every wave is past its reads of block plane zb - 2's slot: refill it with zb + 2's
        if constexpr (kIsShell<M>) {
          if (t < kShellStride) coef_ring[(zb + 2) & 3][t] = pre;
        }
        store_row(zc, Cy, buf, 0);
      } else {
        // two planes per barrier: an even plane (counted from z0) waits in registers, an
        // odd one writes both to the set of its pair (sets alternate by pair, so a pair's
        // writes never meet the previous pair's reads)
        const int idx = zc - z0;
        if ((idx & 1) == 0) {
#pragma unroll
          for (int c = 0; c < 4; ++c) { pCy[c] = Cy[c]; pUp[c] = up[c]; pDn[c] = dn[c]; }
        } else {
          const int set = (idx >> 1) & 1;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            ldy[set][0][c][t] = pUp[c]; ldy[set][0][4 + c][t] = pDn[c];
            ldy[set][1][c][t] = up[c];  ldy[set][1][4 + c][t] = dn[c];
          }
          __syncthreads();
          store_row(zc - 1, pCy, set, 0);
          store_row(zc, Cy, set, 1);
        }
      }
    }
  };

  // Block planes z0-1 .. z1 (coarse plane zb - 1 is finished while plane zb is read),
  // three planes in flight: a ring of three buffers, unrolled so no buffer is copied
  // (measured faster than deeper rings or an indexed ring array).
  if constexpr (kIsShell<M>) {  // rows of block planes z0-1 .. z0+2; later ones refill in process
    for (int e = t; e < 4 * kShellStride; e += kAdjThreads) {
      const int plane = z0 - 1 + e / kShellStride;
      coef_ring[plane & 3][e % kShellStride] =
          m.tab[static_cast<int64_t>(min(max(plane - 1, 0), m.nsets - 1)) * kShellStride + e % kShellStride];
    }
    __syncthreads();
  }
  Plane pa, pb, pc;
  load_plane_y(z0 - 1, pa);
  load_plane_y(z0, pb);
  for (int zb = z0 - 1; zb <= z1; zb += 3) {  // scheduling barriers: as in the forward
    load_plane_y(zb + 2, pc);
    __builtin_amdgcn_sched_barrier(0);
    process(zb, pa);
    if (zb + 1 > z1) break;
    load_plane_y(zb + 3, pa);
    __builtin_amdgcn_sched_barrier(0);
    process(zb + 1, pb);
    if (zb + 2 > z1) break;
    load_plane_y(zb + 4, pb);
    __builtin_amdgcn_sched_barrier(0);
    process(zb + 2, pc);
  }
  if constexpr (kPair == 2) {  // an odd number of planes leaves the last one pending
    const int idx = z1 - 1 - z0;
    if (idx >= 0 && (idx & 1) == 0) {
      const int set = (idx >> 1) & 1;
#pragma unroll
      for (int c = 0; c < 4; ++c) { ldy[set][0][c][t] = pUp[c]; ldy[set][0][4 + c][t] = pDn[c]; }
      __syncthreads();
      store_row(z1 - 1, pCy, set, 0);
    }
  }
}

bool aligned_to(const void* p, int bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

// Can this level run in the sector kernels? (3-D, FP32 arithmetic, stationary and
// reflection-symmetric, an even coarse x extent; slices off a vector boundary take the
// element-access storage forms.)
bool sector_eligible(const icr_plan* p, int level) {
  if (p->ndim != 3 || p->precision == ICR_F64) return false;
  const bool stationary = !p->charted && p->lev[level].sector_ok;
  const bool shell = p->shell && p->lev[level].shell_ok;
  if (!stationary && !shell) return false;
  const int* nc = p->shapes[level];
  if (nc[2] % 2 != 0 || nc[2] < 4) return false;
  const int64_t nf = int64_t(p->shapes[level + 1][0]) * p->shapes[level + 1][1] * p->shapes[level + 1][2];
  return nf < (int64_t(1) << 31);
}

// Compute units of the current device (256 on MI355X).
int64_t compute_units() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 256;
  return cus;
}

// Workgroups of `kernel` that the device holds at once (occupancy x compute units).
int64_t resident_workgroups(const void* kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1 || cus < 1)
    return 1024;
  return int64_t(per_cu) * cus;
}

// Split `planes` into chunks so that all workgroups of a launch (xy tiles x chunks x
// batch) fit in one resident round: a partial second round would run almost alone
// and double the time of the launch, and fewer, longer chunks recompute fewer halo
// planes. Beyond one round (huge levels or batches) each workgroup takes one chunk.
int64_t pick_chunks(int64_t xy_blocks, int planes, int64_t batch, int64_t slots) {
  int64_t n = slots / (xy_blocks * batch);
  if (n < 1) n = 1;
  if (n > planes) n = planes;
  return n;
}

StationaryMats stationary_mats(const LevelMats& m) {
  StationaryMats s;
  for (int t = 0; t < 27; ++t) s.k.c[t] = m.h_sector[t];
  for (int c = 0; c < 8; ++c)
    for (int cp = 0; cp <= c; ++cp) s.k.s[c * (c + 1) / 2 + cp] = m.h_s[c * 8 + cp];
  return s;
}
ShellMats shell_mats(const LevelMats& m) { return ShellMats{m.shell_tab, static_cast<int>(m.nsets)}; }

template <typename TS, typename M>
hipError_t fwd_launch(const icr_plan* p, int level, const M& k, const RefineFwdArgs& a, hipStream_t st) {
  Fwd3Geom g;
  g.nz = p->shapes[level][0]; g.ny = p->shapes[level][1]; g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.rows = g.ny - 2;
  g.nfy = p->shapes[level + 1][1];
  g.nfx = p->shapes[level + 1][2];
  const int64_t xy_blocks = (int64_t(g.rows) * g.pairs + 255) / 256;
  // one workgroup per compute unit, each marching as many planes as that takes: the
  // 196^3 -> 388^3 forward runs in 94 us as 3 chunks of 65 planes (222 workgroups),
  // against 103 us in 10 chunks (four workgroups per compute unit), 111 us in 2 and
  // 125 us in 4 (296 workgroups: a second, partial round); the 100^3 -> 196^3 forward
  // is as fast in 12 or 13 chunks and slower below 8 planes per chunk
  static const int64_t slots = compute_units();
  int64_t chunks = pick_chunks(xy_blocks, g.nz - 2, a.batch < 65535 ? a.batch : 65535, slots);
  g.zchunk = static_cast<int>((g.nz - 2 + chunks - 1) / chunks);
  const int64_t nchunks = (g.nz - 2 + g.zchunk - 1) / g.zchunk;
  g.xy_blocks = static_cast<int>(xy_blocks);
  g.nwg = static_cast<int>(xy_blocks * nchunks);
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineFwdArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.s_in = static_cast<const TS*>(a.s_in) + b0 * a.s_in_bs;
    c.xi = static_cast<const TS*>(a.xi) + b0 * a.xi_bs;
    c.s_out = static_cast<TS*>(a.s_out) + b0 * a.s_out_bs;
    if (a.w) c.w = static_cast<const float*>(a.w) + b0 * a.w_bs;
    const dim3 grid(static_cast<unsigned>(g.nwg), static_cast<unsigned>(c.batch));
    if (a.w) refine3_fwd_sector<TS, true, M><<<grid, 256, 0, st>>>(g, c, k);
    else refine3_fwd_sector<TS, false, M><<<grid, 256, 0, st>>>(g, c, k);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TS, int kTP, int kTR, typename M>
hipError_t adj_launch_tile(const icr_plan* p, int level, const M& k, const RefineAdjArgs& a,
                           hipStream_t st) {
  constexpr int kOP = kTP - 2, kOR = kTR - 2;  // as in the kernel
  Adj3Geom g;
  g.nz = p->shapes[level][0]; g.ny = p->shapes[level][1]; g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.xtiles = (g.pairs + kOP - 1) / kOP;
  const int ytiles = (g.ny + kOR - 1) / kOR;
  g.nfy = p->shapes[level + 1][1];
  g.nfx = p->shapes[level + 1][2];
  const int64_t xy_blocks = int64_t(g.xtiles) * ytiles;
  static const int64_t slots =
      resident_workgroups(reinterpret_cast<const void*>(refine3_adj_sector<TS, false, kTP, kTR, M>), kTP * kTR);
  const int64_t chunks = pick_chunks(xy_blocks, g.nz, a.batch < 65535 ? a.batch : 65535, slots);
  g.zchunk = static_cast<int>((g.nz + chunks - 1) / chunks);
  const int64_t nchunks = (g.nz + g.zchunk - 1) / g.zchunk;
  g.xy_tiles = static_cast<int>(xy_blocks);
  g.nwg = static_cast<int>(xy_blocks * nchunks);
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineAdjArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.y = static_cast<const TS*>(a.y) + b0 * a.y_bs;
    c.xi_bar = static_cast<TS*>(a.xi_bar) + b0 * a.xi_bar_bs;
    c.s_bar = static_cast<TS*>(a.s_bar) + b0 * a.s_bar_bs;
    if (a.add) c.add = static_cast<const TS*>(a.add) + b0 * a.add_bs;
    const dim3 grid(static_cast<unsigned>(g.nwg), static_cast<unsigned>(c.batch));
    if (a.add) refine3_adj_sector<TS, true, kTP, kTR, M><<<grid, kTP * kTR, 0, st>>>(g, c, k);
    else refine3_adj_sector<TS, false, kTP, kTR, M><<<grid, kTP * kTR, 0, st>>>(g, c, k);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// 16 block pairs (x) by 32 block rows (y): one 512-thread workgroup per CU at this
// register budget; measured fastest of 16x16, 32x8, 64x4, 32x16, 16x32 and 64x8 on
// the 388^3 level. With FP32 storage 16 x 24 tiles (one 384-thread workgroup per CU:
// about 200 registers per lane leave room for two wavefronts per SIMD) do better there
// (110-114 us against 115-118 us over repeated sweeps; 16 x 20, 26, 28, 48 and 32 x 32
// were slower, and so was capping the registers for two workgroups per CU, which
// spilled), with BF16 storage they do not (80-88 us against 76-80).
// Levels of at most 100 rows take 16x16 tiles (two workgroups per CU; the step 1.7 us
// shorter, the shell-charted step 1 us); 16x8 tiles on the smallest levels changed nothing.
template <typename TS>
hipError_t adj_launch(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st) {
  const LevelMats& m = p->lev[level];
  if (p->shell && p->shapes[level][1] <= 100) return adj_launch_tile<TS, 16, 16>(p, level, shell_mats(m), a, st);
  if (p->shell) return adj_launch_tile<TS, 16, 32>(p, level, shell_mats(m), a, st);
  if (p->shapes[level][1] <= 100) return adj_launch_tile<TS, 16, 16>(p, level, stationary_mats(m), a, st);
  if (IsF32Storage<TS>::value) return adj_launch_tile<TS, 16, 24>(p, level, stationary_mats(m), a, st);
  return adj_launch_tile<TS, 16, 32>(p, level, stationary_mats(m), a, st);
}
template <typename TS>
hipError_t fwd_launch(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st) {
  const LevelMats& m = p->lev[level];
  if (p->shell) return fwd_launch<TS>(p, level, shell_mats(m), a, st);
  return fwd_launch<TS>(p, level, stationary_mats(m), a, st);
}

// The derivative matrices of a level (plans built for hyperparameter gradients) and its
// value sqrtD.
DotStationary dstationary_mats(const LevelMats& m) {
  DotStationary s;
  for (int t = 0; t < 27; ++t) s.k.c[t] = m.h_dsector[t];
  for (int c = 0; c < 8; ++c)
    for (int cp = 0; cp <= c; ++cp) {
      s.k.s[c * (c + 1) / 2 + cp] = m.h_ds[c * 8 + cp];
      s.sv[c * (c + 1) / 2 + cp] = m.h_s[c * 8 + cp];
    }
  return s;
}
DotShell dshell_mats(const LevelMats& m) { return DotShell{m.dshell_tab, static_cast<int>(m.nsets), m.shell_tab}; }

template <typename TS, typename M>
hipError_t fwd_dot_launch(const icr_plan* p, int level, const M& k, const RefineFwdArgs& a, int64_t max_wgs,
                          hipStream_t st, int64_t* wgs) {
  Fwd3Geom g;
  g.nz = p->shapes[level][0]; g.ny = p->shapes[level][1]; g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.rows = g.ny - 2;
  g.nfy = p->shapes[level + 1][1];
  g.nfx = p->shapes[level + 1][2];
  const int64_t xy_blocks = (int64_t(g.rows) * g.pairs + 255) / 256;
  static const int64_t slots =
      resident_workgroups(reinterpret_cast<const void*>(refine3_fwd_sector<TS, false, M, true>), 256);
  int64_t chunks = pick_chunks(xy_blocks, g.nz - 2, a.batch < 65535 ? a.batch : 65535, slots);
  chunks = std::min<int64_t>(chunks, max_wgs / xy_blocks);  // caller checked max_wgs >= xy_blocks
  g.zchunk = static_cast<int>((g.nz - 2 + chunks - 1) / chunks);
  const int64_t nchunks = (g.nz - 2 + g.zchunk - 1) / g.zchunk;
  g.xy_blocks = static_cast<int>(xy_blocks);
  g.nwg = static_cast<int>(xy_blocks * nchunks);
  *wgs = g.nwg;
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineFwdArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.s_in = static_cast<const TS*>(a.s_in) + b0 * a.s_in_bs;
    c.xi = static_cast<const TS*>(a.xi) + b0 * a.xi_bs;
    c.dot = static_cast<const TS*>(a.dot) + b0 * a.dot_bs;
    c.partial = a.partial + b0 * a.partial_bs;
    c.partial_sig = a.partial_sig + b0 * a.partial_bs;
    const dim3 grid(static_cast<unsigned>(g.nwg), static_cast<unsigned>(c.batch));
    refine3_fwd_sector<TS, false, M, true><<<grid, 256, 0, st>>>(g, c, k);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TS>
hipError_t dot_launch(const icr_plan* p, int level, const RefineFwdArgs& a, int64_t max_wgs, hipStream_t st,
                      int64_t* wgs) {
  const LevelMats& m = p->lev[level];
  if (p->shell) return fwd_dot_launch<TS>(p, level, dshell_mats(m), a, max_wgs, st, wgs);
  return fwd_dot_launch<TS>(p, level, dstationary_mats(m), a, max_wgs, st, wgs);
}

}  // namespace

bool try_refine3_dot_sector(const icr_plan* p, int level, const RefineFwdArgs& a, int64_t max_wgs,
                            hipStream_t st, hipError_t* err, int64_t* wgs) {
  if (p->ndim != 3 || p->precision == ICR_F64) return false;
  const LevelMats& m = p->lev[level];
  const bool stationary = !p->charted && m.dsector_ok;
  const bool shell = p->shell && m.dshell_ok;
  if (!stationary && !shell) return false;
  const int* nc = p->shapes[level];
  if (nc[2] % 2 != 0 || nc[2] < 4) return false;
  const int64_t nf = int64_t(p->shapes[level + 1][0]) * p->shapes[level + 1][1] * p->shapes[level + 1][2];
  if (nf >= (int64_t(1) << 31)) return false;
  const int64_t xy_blocks = (int64_t(nc[1] - 2) * ((nc[2] - 2) / 2) + 255) / 256;
  if (xy_blocks > max_wgs) return false;
  const int el = p->elem_bytes;
  if (!aligned_to(a.xi, 4 * el) || !aligned_to(a.dot, 4 * el) || !aligned_to(a.s_in, 2 * el)) return false;
  if (a.xi_bs % 4 || a.dot_bs % 4 || a.s_in_bs % 2) return false;
  *err = p->precision == ICR_F32 ? dot_launch<float>(p, level, a, max_wgs, st, wgs)
                                 : dot_launch<bf16_t>(p, level, a, max_wgs, st, wgs);
  return true;
}

bool try_refine3_fwd_sector(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st,
                            hipError_t* err) {
  if (!sector_eligible(p, level)) return false;
  const int el = p->elem_bytes;
  const int vec = 4 * el;  // four fine values per vector access
  if (!aligned_to(a.xi, el) || !aligned_to(a.s_out, el) || !aligned_to(a.s_in, el)) return false;
  if (a.w && (!aligned_to(a.w, 16) || a.w_bs % 4)) return false;
  // slices off a vector boundary (a level-0 size that is not a multiple of 4) run the same
  // kernels with element accesses
  const bool vec_ok = aligned_to(a.xi, vec) && aligned_to(a.s_out, vec) && aligned_to(a.s_in, 2 * el) &&
                      a.xi_bs % 4 == 0 && a.s_out_bs % 4 == 0 && a.s_in_bs % 2 == 0;
  if (p->precision == ICR_F32)
    *err = vec_ok ? fwd_launch<float>(p, level, a, st) : fwd_launch<f32u>(p, level, a, st);
  else
    *err = vec_ok ? fwd_launch<bf16_t>(p, level, a, st) : fwd_launch<bf16u>(p, level, a, st);
  return true;
}

bool try_refine3_adj_sector(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st,
                            hipError_t* err) {
  if (!sector_eligible(p, level)) return false;
  const int el = p->elem_bytes;
  const int vec = 4 * el;
  if (!aligned_to(a.y, el) || !aligned_to(a.xi_bar, el) || !aligned_to(a.s_bar, el) ||
      (a.add && !aligned_to(a.add, el)))
    return false;
  const bool vec_ok = aligned_to(a.y, vec) && aligned_to(a.xi_bar, vec) && (!a.add || aligned_to(a.add, vec)) &&
                      a.y_bs % 4 == 0 && a.xi_bar_bs % 4 == 0 && (!a.add || a.add_bs % 4 == 0);
  if (p->precision == ICR_F32)
    *err = vec_ok ? adj_launch<float>(p, level, a, st) : adj_launch<f32u>(p, level, a, st);
  else
    *err = vec_ok ? adj_launch<bf16_t>(p, level, a, st) : adj_launch<bf16u>(p, level, a, st);
  return true;
}

}  // namespace icr
