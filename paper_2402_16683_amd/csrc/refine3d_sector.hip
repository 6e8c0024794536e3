// 3-D refinement level in the reflection-sector basis, FP32 arithmetic with FP32 or
// bfloat16 storage, for stationary levels whose R is reflection-symmetric.
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
// z stage accumulates in registers while marching along z; the y and x stages need
// the neighbouring blocks' contributions, which are exchanged through LDS inside a
// 16 x 16 tile of block pairs whose outer ring (halo) is recomputed by each tile.
// Every coarse cotangent is summed by one thread in a fixed order.
#include "icr_internal.h"

namespace icr {
namespace {

template <typename TS> struct Io;
template <> struct Io<float> {
  static __device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
  static __device__ __forceinline__ float2 ld2(const float* p) { return *reinterpret_cast<const float2*>(p); }
  static __device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
  static __device__ __forceinline__ void st1(float* p, float v) { *p = v; }
};
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  return static_cast<uint32_t>(f32_to_bf16(a)) | (static_cast<uint32_t>(f32_to_bf16(b)) << 16);
}
template <> struct Io<bf16_t> {
  static __device__ __forceinline__ float4 ld4(const bf16_t* p) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  }
  static __device__ __forceinline__ float2 ld2(const bf16_t* p) {
    const uint32_t u = *reinterpret_cast<const uint32_t*>(p);
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
  }
  static __device__ __forceinline__ void st4(bf16_t* p, float4 v) {
    *reinterpret_cast<uint2*>(p) = make_uint2(pack_bf16(v.x, v.y), pack_bf16(v.z, v.w));
  }
  static __device__ __forceinline__ void st1(bf16_t* p, float v) { *p = f32_to_bf16(v); }
};

// sector coefficients C (27, already divided by 8) and the lower sqrtD packed by rows
struct Sector3 {
  float c[27];
  float s[36];
};

__device__ __forceinline__ int sd(int b, int bp) { return b * (b + 1) / 2 + bp; }

// x and y even/odd stages of one coarse plane for the pixel pair (2q+1, 2q+2) of
// row y: T[k][ty * 3 + tx], channels e, m, o = 0, 1, 2.
template <typename TS>
__device__ __forceinline__ void plane_stage(const TS* __restrict__ plane, int y, int nx, int q,
                                            float (&T)[2][9]) {
  float X[3][2][3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const TS* row = plane + static_cast<int64_t>(y - 1 + r) * nx + 2 * q;
    const float2 a = Io<TS>::ld2(row);
    const float2 b = Io<TS>::ld2(row + 2);
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

struct Fwd3Geom {
  int nz, ny, nx;  // coarse shape
  int pairs;       // (nx - 2) / 2 pixel pairs per interior row
  int rows;        // ny - 2 interior rows
  int zchunk;      // interior coarse planes per workgroup
  int nfy, nfx;    // fine rows per plane, fine row length
};

template <typename TS>
__global__ void __launch_bounds__(256) refine3_fwd_sector(Fwd3Geom g, RefineFwdArgs a, Sector3 k) {
  const int tid = blockIdx.x * 256 + threadIdx.x;
  if (tid >= g.rows * g.pairs) return;
  const int yi = tid / g.pairs;
  const int q = tid - yi * g.pairs;
  const int y = yi + 1;
  const int zb = 1 + blockIdx.y * g.zchunk;
  const int ze = min(zb + g.zchunk, g.nz - 1);
  const int64_t b = blockIdx.z;
  const TS* sc = static_cast<const TS*>(a.s_in) + b * a.s_in_bs;
  const TS* xi = static_cast<const TS*>(a.xi) + b * a.xi_bs;
  TS* so = static_cast<TS*>(a.s_out) + b * a.s_out_bs;
  const float* w = a.w ? static_cast<const float*>(a.w) + b * a.w_bs : nullptr;
  const int64_t cplane = static_cast<int64_t>(g.ny) * g.nx;

  float T0[2][9], T1[2][9], T2[2][9];
  plane_stage<TS>(sc + (zb - 1) * cplane, y, g.nx, q, T0);
  plane_stage<TS>(sc + zb * cplane, y, g.nx, q, T1);
  for (int z = zb; z < ze; ++z) {
    plane_stage<TS>(sc + (z + 1) * cplane, y, g.nx, q, T2);
    int64_t off[2][2];
    float4 xr[2][2];
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        off[bz][by] = (static_cast<int64_t>(2 * (z - 1) + bz) * g.nfy + 2 * (y - 1) + by) * g.nfx + 4 * q;
        xr[bz][by] = Io<TS>::ld4(xi + off[bz][by]);
      }
    float o[2][8];
    sector_forward(T0[0], T1[0], T2[0], k, o[0]);
    sector_forward(T0[1], T1[1], T2[1], k, o[1]);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      float x[8];
#pragma unroll
      for (int bz = 0; bz < 2; ++bz)
#pragma unroll
        for (int by = 0; by < 2; ++by) {
          x[bz * 4 + by * 2] = p == 0 ? xr[bz][by].x : xr[bz][by].z;
          x[bz * 4 + by * 2 + 1] = p == 0 ? xr[bz][by].y : xr[bz][by].w;
        }
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int cp = 0; cp <= c; ++cp) o[p][c] = fmaf(k.s[sd(c, cp)], x[cp], o[p][c]);
    }
#pragma unroll
    for (int bz = 0; bz < 2; ++bz)
#pragma unroll
      for (int by = 0; by < 2; ++by) {
        const int h = bz * 4 + by * 2;
        float4 v = make_float4(o[0][h], o[0][h + 1], o[1][h], o[1][h + 1]);
        if (w) {
          const float4 ww = *reinterpret_cast<const float4*>(w + off[bz][by]);
          v.x *= ww.x; v.y *= ww.y; v.z *= ww.z; v.w *= ww.w;
        }
        Io<TS>::st4(so + off[bz][by], v);
      }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int j = 0; j < 9; ++j) { T0[p][j] = T1[p][j]; T1[p][j] = T2[p][j]; }
  }
}

// ----------------------------------------------------------------------------- adjoint

constexpr int kTP = 16;          // tile width in block pairs, halo included
constexpr int kTR = 16;          // tile height in block rows, halo included
constexpr int kOP = kTP - 2;     // owned pairs per tile
constexpr int kOR = kTR - 2;     // owned rows per tile
constexpr int kAdjThreads = kTP * kTR;

struct Adj3Geom {
  int nz, ny, nx;   // coarse shape
  int pairs;        // (nx - 2) / 2 block pairs per row
  int xtiles;       // tiles along x
  int zchunk;       // coarse planes per workgroup
  int nfy, nfx;
};

template <typename TS>
__global__ void __launch_bounds__(kAdjThreads) refine3_adj_sector(Adj3Geom g, RefineAdjArgs a, Sector3 k) {
  __shared__ float ldy[12][kAdjThreads];
  __shared__ float ldx[2][kAdjThreads];
  const int t = threadIdx.x;
  const int i = t % kTP, j = t / kTP;
  const int xt = blockIdx.x % g.xtiles, yt = blockIdx.x / g.xtiles;
  const int P = xt * kOP + i - 1;      // block pair: blocks x = 2P+1, 2P+2
  const int yb = yt * kOR + j - 1;     // block row = coarse row
  const int z0 = blockIdx.y * g.zchunk;
  const int z1 = min(z0 + g.zchunk, g.nz);
  const int64_t b = blockIdx.z;
  const bool pair_ok = P >= 0 && P < g.pairs;
  const bool blocks_ok = pair_ok && yb >= 1 && yb <= g.ny - 2;
  const bool owner = i >= 1 && i <= kOP && j >= 1 && j <= kOR && pair_ok && yb >= 0 && yb < g.ny;
  const TS* y = static_cast<const TS*>(a.y) + b * a.y_bs;
  TS* xb = static_cast<TS*>(a.xi_bar) + b * a.xi_bar_bs;
  TS* sb = static_cast<TS*>(a.s_bar) + b * a.s_bar_bs;
  const TS* add = a.add ? static_cast<const TS*>(a.add) + b * a.add_bs : nullptr;

  float A0[2][9], A1[2][9];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int h = 0; h < 9; ++h) { A0[p][h] = 0.0f; A1[p][h] = 0.0f; }

  for (int zb = z0 - 1; zb <= z1; ++zb) {
    float yv[2][8];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int c = 0; c < 8; ++c) yv[p][c] = 0.0f;
    if (blocks_ok && zb >= 1 && zb <= g.nz - 2) {
      int64_t off[2][2];
      float4 r[2][2];
#pragma unroll
      for (int bz = 0; bz < 2; ++bz)
#pragma unroll
        for (int by = 0; by < 2; ++by) {
          off[bz][by] = (static_cast<int64_t>(2 * (zb - 1) + bz) * g.nfy + 2 * (yb - 1) + by) * g.nfx + 4 * P;
          r[bz][by] = Io<TS>::ld4(y + off[bz][by]);
          yv[0][bz * 4 + by * 2] = r[bz][by].x;
          yv[0][bz * 4 + by * 2 + 1] = r[bz][by].y;
          yv[1][bz * 4 + by * 2] = r[bz][by].z;
          yv[1][bz * 4 + by * 2 + 1] = r[bz][by].w;
        }
      if (owner && zb >= z0 && zb < z1) {
        float xo[2][8];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int cp = 0; cp < 8; ++cp) {
            float v = 0.0f;
#pragma unroll
            for (int c = cp; c < 8; ++c) v = fmaf(k.s[sd(c, cp)], yv[p][c], v);
            xo[p][cp] = v;
          }
#pragma unroll
        for (int bz = 0; bz < 2; ++bz)
#pragma unroll
          for (int by = 0; by < 2; ++by) {
            const int h = bz * 4 + by * 2;
            float4 v = make_float4(xo[0][h], xo[0][h + 1], xo[1][h], xo[1][h + 1]);
            if (add) {
              const float4 av = Io<TS>::ld4(add + off[bz][by]);
              v.x += av.x; v.y += av.y; v.z += av.z; v.w += av.w;
            }
            Io<TS>::st4(xb + off[bz][by], v);
          }
      }
    }
    // sectors (Q), channels (C^T) and the z stage of P^T
    float G[2][9];
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
        const float ue = k.c[jj] * Ys[(sy << 1) | sx];
        const float um = k.c[9 + jj] * Ys[(sy << 1) | sx];
        const float uo = k.c[18 + jj] * Ys[4 | (sy << 1) | sx];
        G[p][jj] = A0[p][jj] + (ue - uo);   // window slot z-1 of this block: coarse zb-1
        A0[p][jj] = A1[p][jj] + um;          // slot 0: coarse zb
        A1[p][jj] = ue + uo;                 // slot z+1: coarse zb+1
      }
    }
    if (zb >= z0 + 1) {  // coarse plane zb - 1 is complete in G (uniform branch)
      const int zc = zb - 1;
      float Cy[2][3];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int tx = 0; tx < 3; ++tx) {
          Cy[p][tx] = G[p][3 + tx];
          ldy[p * 6 + tx][t] = G[p][tx] + G[p][6 + tx];      // to row yb + 1
          ldy[p * 6 + 3 + tx][t] = G[p][tx] - G[p][6 + tx];  // to row yb - 1
        }
      __syncthreads();
      float Hy[2][3];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int tx = 0; tx < 3; ++tx) {
          const float up = j > 0 ? ldy[p * 6 + tx][t - kTP] : 0.0f;
          const float dn = j < kTR - 1 ? ldy[p * 6 + 3 + tx][t + kTP] : 0.0f;
          Hy[p][tx] = Cy[p][tx] + up + dn;
        }
      const float lx0 = Hy[0][0] + Hy[0][2], rx0 = Hy[0][0] - Hy[0][2];
      const float lx1 = Hy[1][0] + Hy[1][2], rx1 = Hy[1][0] - Hy[1][2];
      ldx[0][t] = lx1;  // to the pair on the right (its first block's left neighbour)
      ldx[1][t] = rx0;  // to the pair on the left
      __syncthreads();
      if (owner) {
        const float left = i > 0 ? ldx[0][t - 1] : 0.0f;
        const float right = i < kTP - 1 ? ldx[1][t + 1] : 0.0f;
        TS* row = sb + (static_cast<int64_t>(zc) * g.ny + yb) * g.nx;
        Io<TS>::st1(row + 2 * P + 1, left + Hy[0][1] + rx1);
        Io<TS>::st1(row + 2 * P + 2, lx0 + Hy[1][1] + right);
        if (P == 0) Io<TS>::st1(row, rx0);
        if (P == g.pairs - 1) Io<TS>::st1(row + g.nx - 1, lx1);
      }
    }
  }
}

bool aligned_to(const void* p, int bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

// Can this level run in the sector kernels? (3-D, FP32 arithmetic, stationary and
// reflection-symmetric, an even coarse x extent, vector-aligned rows and batches.)
bool sector_eligible(const icr_plan* p, int level) {
  if (p->ndim != 3 || p->charted || p->precision == ICR_F64) return false;
  if (!p->lev[level].sector_ok) return false;
  const int* nc = p->shapes[level];
  if (nc[2] % 2 != 0 || nc[2] < 4) return false;
  const int64_t nf = int64_t(p->shapes[level + 1][0]) * p->shapes[level + 1][1] * p->shapes[level + 1][2];
  return nf < (int64_t(1) << 31);
}

int64_t pick_chunks(int64_t xy_blocks, int planes, int64_t target) {
  int64_t n = (target + xy_blocks - 1) / xy_blocks;
  if (n < 1) n = 1;
  if (n > planes) n = planes;
  return n;
}

template <typename TS>
hipError_t fwd_launch(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st) {
  const LevelMats& m = p->lev[level];
  Sector3 k;
  for (int t = 0; t < 27; ++t) k.c[t] = m.h_sector[t];
  for (int c = 0; c < 8; ++c)
    for (int cp = 0; cp <= c; ++cp) k.s[c * (c + 1) / 2 + cp] = m.h_s[c * 8 + cp];
  Fwd3Geom g;
  g.nz = p->shapes[level][0]; g.ny = p->shapes[level][1]; g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.rows = g.ny - 2;
  g.nfy = p->shapes[level + 1][1];
  g.nfx = p->shapes[level + 1][2];
  const int64_t xy_blocks = (int64_t(g.rows) * g.pairs + 255) / 256;
  const int64_t chunks = pick_chunks(xy_blocks, g.nz - 2, 2048);
  g.zchunk = static_cast<int>((g.nz - 2 + chunks - 1) / chunks);
  const int64_t nchunks = (g.nz - 2 + g.zchunk - 1) / g.zchunk;
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineFwdArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.s_in = static_cast<const TS*>(a.s_in) + b0 * a.s_in_bs;
    c.xi = static_cast<const TS*>(a.xi) + b0 * a.xi_bs;
    c.s_out = static_cast<TS*>(a.s_out) + b0 * a.s_out_bs;
    if (a.w) c.w = static_cast<const float*>(a.w) + b0 * a.w_bs;
    const dim3 grid(static_cast<unsigned>(xy_blocks), static_cast<unsigned>(nchunks),
                    static_cast<unsigned>(c.batch));
    refine3_fwd_sector<TS><<<grid, 256, 0, st>>>(g, c, k);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename TS>
hipError_t adj_launch(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st) {
  const LevelMats& m = p->lev[level];
  Sector3 k;
  for (int t = 0; t < 27; ++t) k.c[t] = m.h_sector[t];
  for (int c = 0; c < 8; ++c)
    for (int cp = 0; cp <= c; ++cp) k.s[c * (c + 1) / 2 + cp] = m.h_s[c * 8 + cp];
  Adj3Geom g;
  g.nz = p->shapes[level][0]; g.ny = p->shapes[level][1]; g.nx = p->shapes[level][2];
  g.pairs = (g.nx - 2) / 2;
  g.xtiles = (g.pairs + kOP - 1) / kOP;
  const int ytiles = (g.ny + kOR - 1) / kOR;
  g.nfy = p->shapes[level + 1][1];
  g.nfx = p->shapes[level + 1][2];
  const int64_t xy_blocks = int64_t(g.xtiles) * ytiles;
  const int64_t chunks = pick_chunks(xy_blocks, g.nz, 1024);
  g.zchunk = static_cast<int>((g.nz + chunks - 1) / chunks);
  const int64_t nchunks = (g.nz + g.zchunk - 1) / g.zchunk;
  for (int64_t b0 = 0; b0 < a.batch; b0 += 65535) {
    RefineAdjArgs c = a;
    c.batch = a.batch - b0 < 65535 ? a.batch - b0 : 65535;
    c.y = static_cast<const TS*>(a.y) + b0 * a.y_bs;
    c.xi_bar = static_cast<TS*>(a.xi_bar) + b0 * a.xi_bar_bs;
    c.s_bar = static_cast<TS*>(a.s_bar) + b0 * a.s_bar_bs;
    if (a.add) c.add = static_cast<const TS*>(a.add) + b0 * a.add_bs;
    const dim3 grid(static_cast<unsigned>(xy_blocks), static_cast<unsigned>(nchunks),
                    static_cast<unsigned>(c.batch));
    refine3_adj_sector<TS><<<grid, kAdjThreads, 0, st>>>(g, c, k);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

bool try_refine3_fwd_sector(const icr_plan* p, int level, const RefineFwdArgs& a, hipStream_t st,
                            hipError_t* err) {
  if (!sector_eligible(p, level)) return false;
  const int el = p->elem_bytes;
  const int vec = 4 * el;  // four fine values per vector access
  if (!aligned_to(a.xi, vec) || !aligned_to(a.s_out, vec) || !aligned_to(a.s_in, 2 * el)) return false;
  if (a.xi_bs % 4 || a.s_out_bs % 4 || a.s_in_bs % 2) return false;
  if (a.w && (!aligned_to(a.w, 16) || a.w_bs % 4)) return false;
  *err = p->precision == ICR_F32 ? fwd_launch<float>(p, level, a, st) : fwd_launch<bf16_t>(p, level, a, st);
  return true;
}

bool try_refine3_adj_sector(const icr_plan* p, int level, const RefineAdjArgs& a, hipStream_t st,
                            hipError_t* err) {
  if (!sector_eligible(p, level)) return false;
  const int el = p->elem_bytes;
  const int vec = 4 * el;
  if (!aligned_to(a.y, vec) || !aligned_to(a.xi_bar, vec) || (a.add && !aligned_to(a.add, vec))) return false;
  if (a.y_bs % 4 || a.xi_bar_bs % 4 || (a.add && a.add_bs % 4)) return false;
  *err = p->precision == ICR_F32 ? adj_launch<float>(p, level, a, st) : adj_launch<bf16_t>(p, level, a, st);
  return true;
}

}  // namespace icr
