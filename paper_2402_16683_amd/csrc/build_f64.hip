// FP64 device build of the ICR matrices.
//
//  * K_00 over all level-0 pixels and its lower Cholesky factor (one workgroup,
//    right-looking, pivots at or below tau clamped to a zero column);
//  * per level (stationary grid) or per interior coarse pixel (chart): the window
//    covariance K_cc, the cross covariance K_fc and the child covariance K_ff,
//    R = K_fc K_cc^-1 through the Cholesky factor of K_cc, D = K_ff - R K_cf
//    (symmetrised) and its clamped lower Cholesky factor sqrtD.
// This is GP conditioning on the 3^d window (Rasmussen & Williams 2006, eq. 2.19),
// the construction NIFTy.re's ICR model refines with (section "Gaussian Processes").
#include "icr_internal.h"

namespace icr {
namespace {

struct KernelSpec {
  int kind;
  double sigma2;
  double length;
};

struct ChartSpec {
  int chart;
  double p0, p1, p2, p3;
};

__device__ double kernel_value(const KernelSpec& k, double r) {
  const double t = r / k.length;
  double v;
  switch (k.kind) {
    case ICR_MATERN12: v = exp(-t); break;
    case ICR_MATERN32: { const double a = 1.7320508075688772 * t; v = (1.0 + a) * exp(-a); break; }
    case ICR_MATERN52: { const double a = 2.23606797749979 * t; v = (1.0 + a + a * a / 3.0) * exp(-a); break; }
    default: v = exp(-0.5 * t * t); break;
  }
  return k.sigma2 * v;
}

// d k(r) / d length of the kernels above (closed forms; the scale only multiplies)
__device__ double kernel_dlength(const KernelSpec& k, double r) {
  const double t = r / k.length;
  double v;
  switch (k.kind) {
    case ICR_MATERN12: v = t * exp(-t); break;
    case ICR_MATERN32: { const double a = 1.7320508075688772 * t; v = a * a * exp(-a); break; }
    case ICR_MATERN52: { const double a = 2.23606797749979 * t; v = a * a * (1.0 + a) / 3.0 * exp(-a); break; }
    default: v = t * t * exp(-0.5 * t * t); break;
  }
  return k.sigma2 * v / k.length;
}

// index-space point -> physical point (D = 2 for the log-radial chart, D = 3 for the
// log-radial cylinder: the same map of the first two axes plus a scaled third axis)
template <int D>
__device__ void chart_map(const ChartSpec& c, const double* x, double* y) {
  if (D == 2 && c.chart == ICR_CHART_LOGRADIAL_2D) {
    const double r = c.p0 * exp(c.p1 * x[0]);
    const double th = c.p2 * x[1];
    y[0] = r * cos(th);
    y[1] = r * sin(th);
  } else if (D == 3 && c.chart == ICR_CHART_LOGRADIAL_CYL_3D) {
    const double r = c.p0 * exp(c.p1 * x[0]);
    const double th = c.p2 * x[1];
    y[0] = r * cos(th);
    y[1] = r * sin(th);
    y[D - 1] = c.p3 * x[D - 1];
  } else {
    for (int a = 0; a < D; ++a) y[a] = x[a];
  }
}

template <int D>
__device__ double distance(const double* a, const double* b) {
  double s = 0.0;
  for (int k = 0; k < D; ++k) { const double d = a[k] - b[k]; s += d * d; }
  return sqrt(s);
}

// Conditioning matrices of one window, computed by one 64-lane workgroup with the
// matrices in LDS. win: [NW][D], kid: [NC][D] physical positions. Writes R [NC][NW] and
// sqrtD [NC][NC] (lower) and returns, uniformly, the number of clamped pivots, or -1 if
// K_cc is not positive definite or a pivot of D needed clamping with clamping disabled.
//   K_cc = L L^T (right-looking, column by column; lanes share each column's scaling and
//   the trailing update), R^T = K_cc^-1 K_cf by forward and backward substitution with
//   the eight right-hand sides side by side, D = K_ff - R K_cf (symmetrised) one entry
//   per lane, sqrtD = the clamped lower Cholesky factor of D (lane 0: 8 x 8).
// Derivatives with respect to the length scale (dr_out, ds_out; skipped when null) are
// computed by lane 0 afterwards from the same LDS matrices (condition_derivatives).
template <int D>
struct WindowLds {
  static constexpr int NW = pow3(D);
  static constexpr int NC = 1 << D;
  double lc[NW * NW];   // K_cc, then its lower factor (full rows)
  double kfc[NC * NW];
  double r[NC * NW];
  double dm[NC * NC];
  double s[NC * NC];
  double win[NW * D];
  double kid[NC * D];
  int result;
};

template <int D>
__device__ int condition_derivatives(const KernelSpec& ks, const double* win, const double* kid, double* lc,
                                     double* kfc, double* r_out, double* s_out, double* dm, int clamped,
                                     double* dr_out, double* ds_out) {
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  if (clamped > 0) return -2;
  // dR rows: K_cc dR[b,:]^T = dK_fc[b,:]^T - dK_cc R[b,:]^T, solved with the factor of K_cc
  for (int b = 0; b < NC; ++b) {
    double* x = dr_out + b * NW;
    for (int i = 0; i < NW; ++i) {
      double v = kernel_dlength(ks, distance<D>(kid + b * D, win + i * D));
      for (int j = 0; j < NW; ++j) v -= kernel_dlength(ks, distance<D>(win + i * D, win + j * D)) * r_out[b * NW + j];
      x[i] = v;
    }
    for (int i = 0; i < NW; ++i) {
      double v = x[i];
      for (int k = 0; k < i; ++k) v -= lc[i * NW + k] * x[k];
      x[i] = v / lc[i * NW + i];
    }
    for (int i = NW - 1; i >= 0; --i) {
      double v = x[i];
      for (int k = i + 1; k < NW; ++k) v -= lc[k * NW + i] * x[k];
      x[i] = v / lc[i * NW + i];
    }
  }
  // dD (symmetrised) into dm
  for (int b = 0; b < NC; ++b)
    for (int c = 0; c < NC; ++c) {
      double v = kernel_dlength(ks, distance<D>(kid + b * D, kid + c * D));
      for (int w = 0; w < NW; ++w)
        v -= dr_out[b * NW + w] * kfc[c * NW + w] +
             r_out[b * NW + w] * kernel_dlength(ks, distance<D>(kid + c * D, win + w * D));
      dm[b * NC + c] = v;
    }
  for (int b = 0; b < NC; ++b)
    for (int c = 0; c < b; ++c) {
      const double m = 0.5 * (dm[b * NC + c] + dm[c * NC + b]);
      dm[b * NC + c] = m;
      dm[c * NC + b] = m;
    }
  // X = S^-1 dD (columns), then Y = S^-1 X^T = S^-1 dD S^-T (symmetric)
  double x[NC * NC];
  for (int c = 0; c < NC; ++c)
    for (int i = 0; i < NC; ++i) {
      double v = dm[i * NC + c];
      for (int k = 0; k < i; ++k) v -= s_out[i * NC + k] * x[k * NC + c];
      x[i * NC + c] = v / s_out[i * NC + i];
    }
  for (int c = 0; c < NC; ++c)
    for (int i = 0; i < NC; ++i) {
      double v = x[c * NC + i];
      for (int k = 0; k < i; ++k) v -= s_out[i * NC + k] * dm[k * NC + c];
      dm[i * NC + c] = v / s_out[i * NC + i];
    }
  // dS = S Phi(Y)
  for (int i = 0; i < NC; ++i)
    for (int j = 0; j < NC; ++j) {
      double v = 0.0;
      if (j <= i) {
        for (int k = j; k <= i; ++k) {
          const double y = 0.5 * (dm[k * NC + j] + dm[j * NC + k]);
          v += s_out[i * NC + k] * (k == j ? 0.5 * y : y);
        }
      }
      ds_out[i * NC + j] = v;
    }
  return 0;
}

template <int D>
__device__ int condition_window(const KernelSpec& ks, WindowLds<D>& w, double tau, bool clamp, double* r_out,
                                double* s_out, double* dr_out, double* ds_out) {
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  const int lane = threadIdx.x;
  constexpr int kLanes = 64;
  for (int e = lane; e < NW * NW; e += kLanes) {
    const int i = e / NW, j = e % NW;
    w.lc[e] = kernel_value(ks, distance<D>(w.win + i * D, w.win + j * D));
  }
  for (int e = lane; e < NC * NW; e += kLanes) {
    const int b = e / NW, c = e % NW;
    w.kfc[e] = kernel_value(ks, distance<D>(w.kid + b * D, w.win + c * D));
    w.r[e] = w.kfc[e];
  }
  if (lane == 0) w.result = 0;
  __syncthreads();
  // Cholesky of K_cc, no clamping (R needs its inverse)
  for (int j = 0; j < NW; ++j) {
    const double piv = w.lc[j * NW + j];
    if (!(piv > 0.0)) return -1;  // uniform: every lane read the same pivot
    const double root = sqrt(piv);
    __syncthreads();
    for (int i = j + 1 + lane; i < NW; i += kLanes) w.lc[i * NW + j] /= root;
    if (lane == 0) w.lc[j * NW + j] = root;
    __syncthreads();
    const int m = NW - j - 1;
    for (int e = lane; e < m * m; e += kLanes) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) w.lc[i * NW + k] -= w.lc[i * NW + j] * w.lc[k * NW + j];
    }
    __syncthreads();
  }
  // R rows: L y = K_cf[:, b], then L^T x = y, all eight right-hand sides at once
  for (int i = 0; i < NW; ++i) {
    if (lane < NC) w.r[lane * NW + i] /= w.lc[i * NW + i];
    __syncthreads();
    const int m = NW - i - 1;
    for (int e = lane; e < NC * m; e += kLanes) {
      const int b = e / m, k = i + 1 + e % m;
      w.r[b * NW + k] -= w.lc[k * NW + i] * w.r[b * NW + i];
    }
    __syncthreads();
  }
  for (int i = NW - 1; i >= 0; --i) {
    if (lane < NC) w.r[lane * NW + i] /= w.lc[i * NW + i];
    __syncthreads();
    for (int e = lane; e < NC * i; e += kLanes) {
      const int b = e / i, k = e % i;
      w.r[b * NW + k] -= w.lc[i * NW + k] * w.r[b * NW + i];
    }
    __syncthreads();
  }
  // D = K_ff - R K_cf, symmetrised
  double dv = 0.0;
  if (lane < NC * NC) {
    const int b = lane / NC, c = lane % NC;
    dv = kernel_value(ks, distance<D>(w.kid + b * D, w.kid + c * D));
    for (int k = 0; k < NW; ++k) dv -= w.r[b * NW + k] * w.kfc[c * NW + k];
    w.dm[lane] = dv;
  }
  __syncthreads();
  if (lane < NC * NC) {
    const int b = lane / NC, c = lane % NC;
    dv = b == c ? w.dm[lane] : 0.5 * (w.dm[b * NC + c] + w.dm[c * NC + b]);
  }
  __syncthreads();
  if (lane < NC * NC) w.dm[lane] = dv;
  for (int e = lane; e < NC * NW; e += kLanes) r_out[e] = w.r[e];
  __syncthreads();
  // clamped lower Cholesky of D, column by column (lane 0)
  if (lane == 0) {
    int clamped = 0;
    for (int i = 0; i < NC * NC; ++i) w.s[i] = 0.0;
    for (int j = 0; j < NC && clamped >= 0; ++j) {
      double piv = w.dm[j * NC + j];
      for (int k = 0; k < j; ++k) piv -= w.s[j * NC + k] * w.s[j * NC + k];
      if (!(piv > tau)) {
        if (!clamp) {
          clamped = -1;
          break;
        }
        ++clamped;  // column j stays zero
        continue;
      }
      const double root = sqrt(piv);
      w.s[j * NC + j] = root;
      for (int i = j + 1; i < NC; ++i) {
        double v = w.dm[i * NC + j];
        for (int k = 0; k < j; ++k) v -= w.s[i * NC + k] * w.s[j * NC + k];
        w.s[i * NC + j] = v / root;
      }
    }
    for (int i = 0; i < NC * NC; ++i) s_out[i] = w.s[i];
    if (clamped >= 0 && dr_out)
      clamped = condition_derivatives<D>(ks, w.win, w.kid, w.lc, w.kfc, r_out, s_out, w.dm, clamped, dr_out, ds_out);
    w.result = clamped;
  }
  __syncthreads();
  return w.result;
}

struct LevelGeom {
  double origin[3];   // index-space origin o_l per axis (natural axis order)
  double spacing[3];  // delta_l per axis
  int interior[3];    // interior coarse pixels per axis (natural order)
  int64_t nsets;
  int shell;          // one set per interior index of the first axis, at pixel (c, 1, 1)
};

// One 64-lane workgroup per set: a stationary level has one set, a charted level one per
// interior coarse pixel (C order) or one per radial shell.
template <int D>
__global__ void __launch_bounds__(64) build_level_kernel(KernelSpec ks, ChartSpec cs, LevelGeom g, double tau,
                                                         int clamp, double* __restrict__ r64, double* __restrict__ s64,
                                                         double* __restrict__ dr64, double* __restrict__ ds64,
                                                         int32_t* __restrict__ count, int32_t* __restrict__ status) {
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  __shared__ WindowLds<D> w;
  const int64_t set = blockIdx.x;
  const int lane = threadIdx.x;
  double centre[D];
  if (cs.chart == ICR_CHART_REGULAR) {
    for (int a = 0; a < D; ++a) centre[a] = 0.0;  // only relative positions matter
  } else if (g.shell) {
    for (int a = 0; a < D; ++a) centre[a] = g.origin[a] + (a == 0 ? set + 1 : 1) * g.spacing[a];
  } else {
    int64_t rem = set;
    for (int a = D - 1; a >= 0; --a) {
      const int ca = static_cast<int>(rem % g.interior[a]) + 1;
      rem /= g.interior[a];
      centre[a] = g.origin[a] + ca * g.spacing[a];
    }
  }
  double pt[D];
  if (lane < NW) {
    int rem = lane;
    for (int a = D - 1; a >= 0; --a) {
      pt[a] = centre[a] + ((rem % 3) - 1) * g.spacing[a];
      rem /= 3;
    }
    chart_map<D>(cs, pt, w.win + lane * D);
  }
  if (lane < NC) {
    for (int a = 0; a < D; ++a) {
      const int ba = (lane >> (D - 1 - a)) & 1;
      pt[a] = centre[a] + (ba - 0.5) * 0.5 * g.spacing[a];
    }
    chart_map<D>(cs, pt, w.kid + lane * D);
  }
  __syncthreads();
  const int n = condition_window<D>(ks, w, tau, clamp != 0, r64 + set * NC * NW, s64 + set * NC * NC,
                                    dr64 ? dr64 + set * NC * NW : nullptr, ds64 ? ds64 + set * NC * NC : nullptr);
  if (lane != 0) return;
  if (n == -2) atomicOr(status, 4);
  else if (n < 0) atomicOr(status, 1);
  else if (n > 0) atomicAdd(count, n);
}

// K_00[i][j] = k(|x_i - x_j|) over the level-0 pixels in C order (kDeriv: d k / d length).
template <int D, bool kDeriv = false>
__global__ void build_k00_kernel(KernelSpec ks, ChartSpec cs, int n0a, int n0b, int n0c,
                                 double d0, double d1, double d2, int64_t n, double* __restrict__ a) {
  const int64_t i = static_cast<int64_t>(blockIdx.y);
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int shp[3] = {n0a, n0b, n0c};
  const double sp[3] = {d0, d1, d2};
  double xi[D], xj[D], pi[D], pj[D];
  int64_t ri = i, rj = j;
  for (int ax = D - 1; ax >= 0; --ax) {
    xi[ax] = static_cast<double>(ri % shp[ax]) * sp[ax];
    xj[ax] = static_cast<double>(rj % shp[ax]) * sp[ax];
    ri /= shp[ax];
    rj /= shp[ax];
  }
  chart_map<D>(cs, xi, pi);
  chart_map<D>(cs, xj, pj);
  a[i * n + j] = kDeriv ? kernel_dlength(ks, distance<D>(pi, pj)) : kernel_value(ks, distance<D>(pi, pj));
}

// Derivative of the level-0 factor along dK_00 (dL = L Phi(L^-1 dK L^-T), as for sqrtD),
// in three passes over n x n FP64 matrices. 1: X = L^-1 dK by forward substitution,
// column j by one wavefront that keeps the column in LDS (the lanes split each row's dot
// product, a butterfly sums it); dK is overwritten by X. 2: Y = L^-1 X^T the same way,
// the right-hand side of column j being row j of X. 3: one thread per element (i, j <= i)
// of dL = L Phi(Y).
template <bool kTransposedRhs>
__global__ void __launch_bounds__(64) dl00_solve_kernel(const double* __restrict__ low,
                                                        const double* __restrict__ rhs, double* __restrict__ out,
                                                        int64_t n) {
  extern __shared__ double col[];
  const int64_t j = blockIdx.x;
  const int lane = threadIdx.x;
  for (int64_t i = 0; i < n; ++i) {
    double v = 0.0;
    for (int64_t k = lane; k < i; k += 64) v += low[i * n + k] * col[k];
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) {
      const double b = kTransposedRhs ? rhs[j * n + i] : rhs[i * n + j];
      col[i] = (b - v) / low[i * n + i];
    }
    __syncthreads();  // one wavefront: makes col[i] visible to every lane
  }
  for (int64_t i = lane; i < n; i += 64) out[i * n + j] = col[i];
}
__global__ void dl00_product_kernel(const double* __restrict__ low, const double* __restrict__ y,
                                    double* __restrict__ dl, int64_t n) {
  const int64_t i = blockIdx.y;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double v = 0.0;
  for (int64_t k = j; k <= i; ++k) {
    const double s = 0.5 * (y[k * n + j] + y[j * n + k]);
    v += low[i * n + k] * (k == j ? 0.5 * s : s);
  }
  dl[i * n + j] = v;  // zero above the diagonal (empty sum)
}

// Blocked right-looking Cholesky of the n x n matrix a (row-major, in place, lower) in
// panels of kPanel columns. A pivot at or below tau makes its column zero and is
// counted; a zero column leaves the rest of the matrix unchanged. The blocked order only
// regroups the same updates: each panel's diagonal block is factored column by column in
// LDS by one workgroup and the rows below it solved against that factor, then one
// workgroup per 32 x 32 tile of the trailing lower triangle subtracts the panel's
// contribution.
constexpr int kPanel = 32;

__global__ void __launch_bounds__(1024) chol_panel_kernel(double* __restrict__ a, int64_t n, int64_t j0, double tau,
                                                          int clamp, int32_t* __restrict__ count,
                                                          int32_t* __restrict__ status) {
  // the diagonal block A11 (rows and columns j0 .. j1-1) is factored in LDS by the
  // workgroup, column by column (the rows below it are solved by chol_solve_kernel)
  __shared__ double l11[kPanel][kPanel + 1];
  __shared__ int zero_col[kPanel];
  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;
  const int64_t j1 = j0 + kPanel < n ? j0 + kPanel : n;
  const int nb = static_cast<int>(j1 - j0);
  for (int e = tid; e < kPanel * kPanel; e += nthreads) {
    const int r = e / kPanel, c = e % kPanel;
    l11[r][c] = (r < nb && c <= r) ? a[(j0 + r) * n + j0 + c] : 0.0;
  }
  if (tid >= nb && tid < kPanel) zero_col[tid] = 1;  // columns past the matrix (last panel)
  __syncthreads();
  int clamped = 0;
  for (int j = 0; j < nb; ++j) {
    const double piv = l11[j][j];
    __syncthreads();  // every thread holds the pivot before column j is written
    const bool bad = !(piv > tau);  // uniform across the workgroup
    if (tid == 0) zero_col[j] = bad ? 1 : 0;
    if (bad) {
      ++clamped;
      if (tid > j && tid < nb) l11[tid][j] = 0.0;
      if (tid == 0) l11[j][j] = 0.0;
      __syncthreads();
      continue;
    }
    const double root = sqrt(piv);
    if (tid > j && tid < nb) l11[tid][j] /= root;
    if (tid == 0) l11[j][j] = root;
    __syncthreads();
    // trailing update inside the block: one thread per (row, column) pair
    const int i = tid / kPanel, k = tid % kPanel;
    if (tid < kPanel * kPanel && i > j && k > j && k <= i && i < nb) l11[i][k] -= l11[i][j] * l11[k][j];
    __syncthreads();
  }
  for (int e = tid; e < kPanel * kPanel; e += nthreads) {
    const int r = e / kPanel, c = e % kPanel;
    if (r < nb && c <= r) a[(j0 + r) * n + j0 + c] = l11[r][c];
  }
  if (tid == 0) {
    *count += clamped;  // panels run one after another on the stream
    if (clamped > 0 && !clamp) *status |= 2;
  }
}

// Trailing update after the panel j0 .. j0+kPanel-1: a[i][k] -= sum_p a[i][p] a[k][p] for
// j1 <= k <= i < n; one workgroup per 32 x 32 tile (tiles above the diagonal leave).
// The panel's rows below its diagonal block: x L11^T = a[i][j0 .. j1-1] for i >= j1,
// one thread per row (forward substitution; a clamped column of L11, zero on its
// diagonal, gives a zero entry: the clamped column of the factor is zero). A separate
// launch over many workgroups: solving them in the panel's single workgroup held 32
// doubles per lane under a 1024-thread bound and spilled to scratch (up to 214 us per
// panel at n = 1000). The workgroup's rows go through LDS: loaded and stored as whole
// row segments (coalesced), solved in place with each thread's row in a column of xs.
constexpr int kSolveRows = 256;
__global__ void __launch_bounds__(kSolveRows) chol_solve_kernel(double* __restrict__ a, int64_t n, int64_t j0) {
  __shared__ double l11[kPanel][kPanel + 1];
  __shared__ double xs[kPanel][kSolveRows + 1];
  const int tid = threadIdx.x;
  const int64_t j1 = j0 + kPanel < n ? j0 + kPanel : n;
  const int nb = static_cast<int>(j1 - j0);
  const int64_t i0 = j1 + int64_t(blockIdx.x) * kSolveRows;  // first row of this workgroup
  const int rows = static_cast<int>(n - i0 < kSolveRows ? n - i0 : kSolveRows);
  for (int e = tid; e < kPanel * kPanel; e += kSolveRows) {
    const int r = e / kPanel, c = e % kPanel;
    l11[r][c] = (r < nb && c <= r) ? a[(j0 + r) * n + j0 + c] : 0.0;
  }
  for (int e = tid; e < kPanel * kSolveRows; e += kSolveRows) {  // (row, column): rows of 32 doubles
    const int r = e / kPanel, c = e % kPanel;
    xs[c][r] = (r < rows && c < nb) ? a[(i0 + r) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    // four partial sums, so the LDS reads of one step do not wait on the previous FMA
    double v[4] = {xs[j][tid], 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 4 <= j; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] -= xs[k + u][tid] * l11[j][k + u];
    }
    for (; k < j; ++k) v[0] -= xs[k][tid] * l11[j][k];
    const double sum = (v[0] + v[1]) + (v[2] + v[3]);
    xs[j][tid] = l11[j][j] == 0.0 ? 0.0 : sum / l11[j][j];
  }
  __syncthreads();
  for (int e = tid; e < kPanel * kSolveRows; e += kSolveRows) {
    const int r = e / kPanel, c = e % kPanel;
    if (r < rows && c < nb) a[(i0 + r) * n + j0 + c] = xs[c][r];
  }
}

__global__ void __launch_bounds__(256) chol_update_kernel(double* __restrict__ a, int64_t n, int64_t j0) {
  const int64_t j1 = j0 + kPanel;
  const int ti = blockIdx.y, tk = blockIdx.x;
  if (tk > ti) return;
  __shared__ double pi_[32][kPanel + 1], pk_[32][kPanel + 1];
  const int64_t i0 = j1 + int64_t(ti) * 32, k0 = j1 + int64_t(tk) * 32;
  for (int e = threadIdx.x; e < 32 * kPanel; e += blockDim.x) {
    const int r = e / kPanel, c = e % kPanel;
    pi_[r][c] = i0 + r < n ? a[(i0 + r) * n + j0 + c] : 0.0;
    pk_[r][c] = k0 + r < n ? a[(k0 + r) * n + j0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int r = e / 32, c = e % 32;
    const int64_t i = i0 + r, k = k0 + c;
    if (i >= n || k > i) continue;
    double v = 0.0;
    for (int p = 0; p < kPanel; ++p) v += pi_[r][p] * pk_[c][p];
    a[i * n + k] -= v;
  }
}

__global__ void chol_zero_upper_kernel(double* __restrict__ a, int64_t n) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  if (t % n > t / n) a[t] = 0.0;
}

template <typename TA>
__global__ void convert_level0_kernel(const double* __restrict__ l64, int64_t n,
                                      TA* __restrict__ lower, TA* __restrict__ upper) {
  const int64_t i = blockIdx.y;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  lower[i * n + j] = static_cast<TA>(l64[i * n + j]);
  upper[i * n + j] = static_cast<TA>(l64[j * n + i]);
}

// stationary: copy [NC][NW] as is; charted: transpose to [entry][set]
template <typename TA>
__global__ void convert_level_kernel(const double* __restrict__ src, int64_t nsets, int entries,
                                     int charted, TA* __restrict__ dst) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nsets * entries) return;
  const int64_t set = t / entries;
  const int e = static_cast<int>(t % entries);
  const TA v = static_cast<TA>(src[t]);
  if (charted) dst[static_cast<int64_t>(e) * nsets + set] = v;
  else dst[t] = v;
}

// Reflection-sector form of a stationary R. Per axis, the window (s_-1, s_0, s_+1)
// maps to even/odd channels (e, m, o) = (s_-1 + s_+1, s_0, s_+1 - s_-1) and the two
// children (o_0, o_1) to (S, D) = (o_0 + o_1, o_1 - o_0). A kernel that is invariant
// under reflecting any axis (every radial kernel on a regular grid) gives an R for
// which M = Q R P^-1 only couples sector sigma (S or D per axis) with channels t
// whose axes carry (e or m) where sigma is S and o where sigma is D: 3^d non-zeros
// instead of 2^d 3^d. Then R = B C P with C = M / 2^d on that pattern and B the
// per-axis butterfly o_0 = S - D, o_1 = S + D. One thread per channel t writes C[t],
// the largest off-pattern |M[., t]| and the on-pattern |M[sigma(t), t]|.
template <int D>
__global__ void sector_kernel(const double* __restrict__ r64, double* __restrict__ out) {
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  const int t = threadIdx.x;
  if (t >= NW) return;
  // P^-1 rows w in {-1,0,1} (index w+1), columns t in {e, m, o}
  const double pinv[3][3] = {{0.5, 0.0, -0.5}, {0.0, 1.0, 0.0}, {0.5, 0.0, 0.5}};
  int ta[D];
  {
    int rem = t;
    for (int a = D - 1; a >= 0; --a) { ta[a] = rem % 3; rem /= 3; }
  }
  int own = 0;
  for (int a = 0; a < D; ++a) own = (own << 1) | (ta[a] == 2 ? 1 : 0);
  double off = 0.0, on = 0.0, coef = 0.0;
  for (int sg = 0; sg < NC; ++sg) {
    double m = 0.0;
    for (int b = 0; b < NC; ++b) {
      double q = 1.0;
      for (int a = 0; a < D; ++a) {
        const int sa = (sg >> (D - 1 - a)) & 1, ba = (b >> (D - 1 - a)) & 1;
        q *= (sa == 1 && ba == 0) ? -1.0 : 1.0;   // Q = [[1, 1], [-1, 1]]
      }
      for (int w = 0; w < NW; ++w) {
        double pv = 1.0;
        int rem = w;
        for (int a = D - 1; a >= 0; --a) { pv *= pinv[rem % 3][ta[a]]; rem /= 3; }
        if (pv != 0.0) m += q * r64[b * NW + w] * pv;
      }
    }
    if (sg == own) { on = fabs(m); coef = m / NC; }
    else off = fmax(off, fabs(m));
  }
  out[t] = coef;
  out[NW + t] = off;
  out[2 * NW + t] = on;
}

// Shell-charted 3-D levels (one set per coarse plane): R is invariant under reflecting
// the second and third axes (angle and height of the cylinder chart) but not the
// first. Transforming only those two axes as in sector_kernel, M = Q_yx R P_yx^-1
// couples child sector (sy, sx) of z-child bz only with the window channels
// (wz, ty, tx) of the matching pattern, so R = B_yx C P_yx with 2 x 3 x 9 coefficients
// C[ty tx][bz][wz] = M / 4 (B_yx the butterflies of the two axes; the six values of a
// channel are adjacent). One thread per set writes C and sqrtD (packed by rows) to the
// FP32 table tab[set][kShellStride] and
// the largest off-pattern and on-pattern |M| of the set to chk[set][2].
__global__ void shell_sector_kernel(const double* __restrict__ r64, const double* __restrict__ s64,
                                    int64_t nsets, float* __restrict__ tab, double* __restrict__ chk) {
  const int64_t set = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (set >= nsets) return;
  const double pinv[3][3] = {{0.5, 0.0, -0.5}, {0.0, 1.0, 0.0}, {0.5, 0.0, 0.5}};
  const double* R = r64 + set * 8 * 27;
  float* out = tab + set * kShellStride;
  double off = 0.0, on = 0.0;
  for (int bz = 0; bz < 2; ++bz)
    for (int wz = 0; wz < 3; ++wz)
      for (int ty = 0; ty < 3; ++ty)
        for (int tx = 0; tx < 3; ++tx) {
          const int own = ((ty == 2) << 1) | (tx == 2);
          double coef = 0.0;
          for (int sg = 0; sg < 4; ++sg) {
            const int sy = sg >> 1, sx = sg & 1;
            double m = 0.0;
            for (int by = 0; by < 2; ++by)
              for (int bx = 0; bx < 2; ++bx) {
                const double q = ((sy == 1 && by == 0) ? -1.0 : 1.0) * ((sx == 1 && bx == 0) ? -1.0 : 1.0);
                for (int wy = 0; wy < 3; ++wy)
                  for (int wx = 0; wx < 3; ++wx) {
                    const double pv = pinv[wy][ty] * pinv[wx][tx];
                    if (pv != 0.0) m += q * R[(bz * 4 + by * 2 + bx) * 27 + wz * 9 + wy * 3 + wx] * pv;
                  }
              }
            if (sg == own) { on = fmax(on, fabs(m)); coef = m / 4.0; }
            else off = fmax(off, fabs(m));
          }
          out[(ty * 3 + tx) * 6 + bz * 3 + wz] = static_cast<float>(coef);
        }
  const double* S = s64 + set * 64;
  for (int c = 0; c < 8; ++c)
    for (int cp = 0; cp <= c; ++cp) out[54 + c * (c + 1) / 2 + cp] = static_cast<float>(S[c * 8 + cp]);
  for (int e = 90; e < kShellStride; ++e) out[e] = 0.0f;
  chk[2 * set] = off;
  chk[2 * set + 1] = on;
}

// Shell-charted 2-D levels: the FP32 row table of the fast 2-D kernels, per set R (36,
// [b][w]) then sqrtD lower by rows (10).
__global__ void shell2_table_kernel(const double* __restrict__ r64, const double* __restrict__ s64,
                                    int64_t nsets, float* __restrict__ tab) {
  const int64_t set = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (set >= nsets) return;
  float* out = tab + set * kShellStride;
  for (int e = 0; e < 36; ++e) out[e] = static_cast<float>(r64[set * 36 + e]);
  for (int c = 0; c < 4; ++c)
    for (int cp = 0; cp <= c; ++cp) out[36 + c * (c + 1) / 2 + cp] = static_cast<float>(s64[set * 16 + c * 4 + cp]);
  for (int e = 46; e < kShellStride; ++e) out[e] = 0.0f;
}

KernelSpec kernel_spec(const icr_plan* p) {
  return KernelSpec{p->cfg.kernel, p->cfg.scale * p->cfg.scale, p->cfg.length};
}
ChartSpec chart_spec(const icr_plan* p) {
  return ChartSpec{p->cfg.chart, p->cfg.chart_params[0], p->cfg.chart_params[1],
                   p->cfg.chart_params[2], p->cfg.chart_params[3]};
}
double tau_of(const icr_plan* p) {
  double t = 2.220446049250313e-16 * p->cfg.scale * p->cfg.scale;
  for (int a = 0; a < p->ndim; ++a) t *= 3.0;
  return t;
}

}  // namespace

hipError_t launch_build_k00(const icr_plan* p, double* a, hipStream_t st) {
  const int64_t n = p->n0;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n));
  const int* s = p->cfg.shape0;
  const double* d = p->cfg.distances0;
  switch (p->ndim) {
    case 1: build_k00_kernel<1><<<grid, 256, 0, st>>>(kernel_spec(p), chart_spec(p), s[0], 1, 1, d[0], 0, 0, n, a); break;
    case 2: build_k00_kernel<2><<<grid, 256, 0, st>>>(kernel_spec(p), chart_spec(p), s[0], s[1], 1, d[0], d[1], 0, n, a); break;
    default: build_k00_kernel<3><<<grid, 256, 0, st>>>(kernel_spec(p), chart_spec(p), s[0], s[1], s[2], d[0], d[1], d[2], n, a); break;
  }
  return hipGetLastError();
}

// dL_00 / d length into p->dl00_64 (plans built for hyperparameter gradients); scratch
// holds 2 n0^2 doubles.
hipError_t launch_level0_length_derivative(const icr_plan* p, double* scratch, hipStream_t st) {
  const int64_t n = p->n0;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n));
  const int* s = p->cfg.shape0;
  const double* d = p->cfg.distances0;
  double* a = scratch;
  double* y = scratch + n * n;
  switch (p->ndim) {
    case 1: build_k00_kernel<1, true><<<grid, 256, 0, st>>>(kernel_spec(p), chart_spec(p), s[0], 1, 1, d[0], 0, 0, n, a); break;
    case 2: build_k00_kernel<2, true><<<grid, 256, 0, st>>>(kernel_spec(p), chart_spec(p), s[0], s[1], 1, d[0], d[1], 0, n, a); break;
    default: build_k00_kernel<3, true><<<grid, 256, 0, st>>>(kernel_spec(p), chart_spec(p), s[0], s[1], s[2], d[0], d[1], d[2], n, a); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(double) * size_t(n);  // one column per wavefront (n <= 4096: 32 KB)
  dl00_solve_kernel<false><<<static_cast<unsigned>(n), 64, lds, st>>>(p->l00_64, a, a, n);
  dl00_solve_kernel<true><<<static_cast<unsigned>(n), 64, lds, st>>>(p->l00_64, a, y, n);
  dl00_product_kernel<<<grid, 256, 0, st>>>(p->l00_64, y, p->dl00_64, n);
  return hipGetLastError();
}

hipError_t launch_cholesky_level0(const icr_plan* p, double* a, int32_t* counts, int32_t* status,
                                  hipStream_t st) {
  const int clamp = (p->cfg.flags & ICR_FLAG_NO_CLAMP) ? 0 : 1;
  const int64_t n = p->n0;
  for (int64_t j0 = 0; j0 < n; j0 += kPanel) {
    chol_panel_kernel<<<1, 1024, 0, st>>>(a, n, j0, tau_of(p), clamp, counts, status);
    const int64_t m = n - j0 - kPanel;  // trailing size
    if (m > 0) {
      chol_solve_kernel<<<static_cast<unsigned>((m + kSolveRows - 1) / kSolveRows), kSolveRows, 0, st>>>(a, n, j0);
      const unsigned tiles = static_cast<unsigned>((m + 31) / 32);
      chol_update_kernel<<<dim3(tiles, tiles), 256, 0, st>>>(a, n, j0);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  chol_zero_upper_kernel<<<static_cast<unsigned>((n * n + 255) / 256), 256, 0, st>>>(a, n);
  return hipGetLastError();
}

hipError_t launch_level0_convert(const icr_plan* p, hipStream_t st) {
  const int64_t n = p->n0;
  const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n));
  if (p->precision == ICR_F64)
    convert_level0_kernel<double><<<grid, 256, 0, st>>>(p->l00_64, n, static_cast<double*>(p->l00_c),
                                                        static_cast<double*>(p->u00_c));
  else
    convert_level0_kernel<float><<<grid, 256, 0, st>>>(p->l00_64, n, static_cast<float*>(p->l00_c),
                                                       static_cast<float*>(p->u00_c));
  return hipGetLastError();
}

hipError_t launch_build_level(const icr_plan* p, int level, int32_t* counts, int32_t* status,
                              hipStream_t st) {
  const int d = p->ndim;
  LevelGeom g;
  for (int a = 0; a < 3; ++a) {
    g.origin[a] = a < d ? p->origins[level][a] : 0.0;
    g.spacing[a] = a < d ? p->spacings[level][a] : 0.0;
    g.interior[a] = a < d ? p->shapes[level][3 - d + a] - 2 : 1;
  }
  g.nsets = p->lev[level].nsets;
  g.shell = p->shell;
  const int clamp = (p->cfg.flags & ICR_FLAG_NO_CLAMP) ? 0 : 1;
  const unsigned threads = 64;  // one workgroup (one wavefront) per set
  const unsigned blocks = static_cast<unsigned>(g.nsets);
  const LevelMats& m = p->lev[level];
  switch (d) {
    case 1: build_level_kernel<1><<<blocks, threads, 0, st>>>(kernel_spec(p), chart_spec(p), g, tau_of(p), clamp, m.r64, m.s64, m.dr64, m.ds64, counts, status); break;
    case 2: build_level_kernel<2><<<blocks, threads, 0, st>>>(kernel_spec(p), chart_spec(p), g, tau_of(p), clamp, m.r64, m.s64, m.dr64, m.ds64, counts, status); break;
    default: build_level_kernel<3><<<blocks, threads, 0, st>>>(kernel_spec(p), chart_spec(p), g, tau_of(p), clamp, m.r64, m.s64, m.dr64, m.ds64, counts, status); break;
  }
  return hipGetLastError();
}

hipError_t launch_level_convert(const icr_plan* p, int level, hipStream_t st) {
  const LevelMats& m = p->lev[level];
  const int nc = 1 << p->ndim;
  const int nw = pow3(p->ndim);
  const unsigned threads = 256;
  const int parts = m.dr64 ? 4 : 2;  // R, sqrtD and, for hyperparameter gradients, their derivatives
  for (int which = 0; which < parts; ++which) {
    const int entries = which % 2 == 0 ? nc * nw : nc * nc;
    const double* src = which == 0 ? m.r64 : which == 1 ? m.s64 : which == 2 ? m.dr64 : m.ds64;
    void* dst = which == 0 ? m.r_c : which == 1 ? m.s_c : which == 2 ? m.dr_c : m.ds_c;
    const int64_t total = m.nsets * entries;
    const unsigned blocks = static_cast<unsigned>((total + threads - 1) / threads);
    if (p->precision == ICR_F64)
      convert_level_kernel<double><<<blocks, threads, 0, st>>>(src, m.nsets, entries, p->charted, static_cast<double*>(dst));
    else
      convert_level_kernel<float><<<blocks, threads, 0, st>>>(src, m.nsets, entries, p->charted, static_cast<float*>(dst));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sector(const icr_plan* p, int level, hipStream_t st) {
  const LevelMats& m = p->lev[level];
  switch (p->ndim) {
    case 1: sector_kernel<1><<<1, 64, 0, st>>>(m.r64, m.sector64); break;
    case 2: sector_kernel<2><<<1, 64, 0, st>>>(m.r64, m.sector64); break;
    default: sector_kernel<3><<<1, 64, 0, st>>>(m.r64, m.sector64); break;
  }
  if (m.dr64 && m.dsector64) {  // the length derivative of R has the same symmetry
    switch (p->ndim) {
      case 1: sector_kernel<1><<<1, 64, 0, st>>>(m.dr64, m.dsector64); break;
      case 2: sector_kernel<2><<<1, 64, 0, st>>>(m.dr64, m.dsector64); break;
      default: sector_kernel<3><<<1, 64, 0, st>>>(m.dr64, m.dsector64); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_shell_sector(const icr_plan* p, int level, hipStream_t st) {
  const LevelMats& m = p->lev[level];
  const unsigned threads = 64;
  const unsigned blocks = static_cast<unsigned>((m.nsets + threads - 1) / threads);
  if (p->ndim == 2) {  // dense rows; no symmetry needed
    shell2_table_kernel<<<blocks, threads, 0, st>>>(m.r64, m.s64, m.nsets, m.shell_tab);
    return hipGetLastError();
  }
  shell_sector_kernel<<<blocks, threads, 0, st>>>(m.r64, m.s64, m.nsets, m.shell_tab, m.shell_chk);
  if (m.dr64 && m.dshell_tab)
    shell_sector_kernel<<<blocks, threads, 0, st>>>(m.dr64, m.ds64, m.nsets, m.dshell_tab, m.dshell_chk);
  return hipGetLastError();
}

}  // namespace icr
