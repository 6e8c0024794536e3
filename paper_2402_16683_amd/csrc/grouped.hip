// Grouped sweep steps: one launch applies one step (level 0, or one refinement level,
// forward or adjoint) of many independent sweeps at once, each from its own plan: 1-D,
// 2-D and 3-D priors of any level sizes, depth and matrices share the launch. The served
// mode gives every pending request's k-th step to the k-th launch of a group.
//
// A table of tasks (one per sweep and step, sorted by first workgroup) tells each
// workgroup what it computes; a workgroup finds its task by binary search over the
// tasks' first workgroups, so every workgroup of a task sees the same task. The
// arithmetic per element is that of the general per-level kernels:
//   level-0 forward   out[i] = sum_{j<=i} L00[i][j] in[j]        (times w: metric epilogue)
//   level-0 adjoint   out[i] = sum_{j>=i} U00[i][j] in[j] + add
//   forward  (one thread per interior coarse pixel c)
//     s_{l+1}[2(c-1)+b] = sum_w R[b,w] s_l[c+w] + sum_{b'<=b} sqrtD[b,b'] xi_{l+1}[2(c-1)+b']
//   adjoint  (one thread per coarse pixel p, a gather: no atomics)
//     s_bar_l[p] = sum_{w, c = p - w interior} sum_b R_c[b,w] y[2(c-1)+b]
//     xi_bar_{l+1}[2(p-1)+b'] = sum_{b>=b'} sqrtD[b,b'] y[2(p-1)+b] + add
// A task's result depends only on the task, not on the others in the launch: a request
// gives the same bits alone and in any mix.
#include "grouped.h"

namespace icr {
namespace {

constexpr int kGroupThreads = 256;

template <int D>
__device__ __forceinline__ int64_t glin(const int* idx, const int* shape) {
  int64_t v = idx[0];
#pragma unroll
  for (int a = 1; a < D; ++a) v = v * shape[a] + idx[a];
  return v;
}

template <typename TA>
__device__ __forceinline__ TA gwave_sum(TA v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// one wavefront per output row; lanes stride the row with sixteen loads in flight
template <typename TS, bool kLower>
__device__ void level0_task(const GroupTask& t, int64_t u0) {
  using TA = typename Acc<TS>::type;
  const int lane = threadIdx.x & 63;
  const int64_t row = (u0 + threadIdx.x) >> 6;
  const int64_t n = t.n0;
  if (row >= n) return;  // whole wavefronts
  const TA* m = static_cast<const TA*>(t.m0) + row * n;
  const TS* in = static_cast<const TS*>(t.in);
  const int64_t j0 = kLower ? 0 : row;
  const int64_t j1 = kLower ? row + 1 : n;
  constexpr int kU = 16;  // as level0_kernel, so both compute the same sums
  TA part[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) part[u] = 0;
  for (int64_t base = j0; base < j1; base += 64 * kU) {
    TA mv[kU];
    TS xr[kU];  // widened after all loads are issued, as in level0_kernel
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
  const TA acc = gwave_sum(part[0]);
  if (lane == 0) {
    TA r = acc;
    if (kLower && t.w) r *= static_cast<const TA*>(t.w)[row];
    if (!kLower && t.add) r += load_acc(static_cast<const TS*>(t.add) + row);
    store_acc(static_cast<TS*>(t.out) + row, r);
  }
}

// stationary R and sqrtD staged in LDS (the whole workgroup has the same task)
template <typename TA, int NC, int NW>
__device__ __forceinline__ void stage_mats(const GroupTask& t, TA* lr, TA* ls, const TA*& R, const TA*& S) {
  R = static_cast<const TA*>(t.m0);
  S = static_cast<const TA*>(t.m1);
  if (t.charted) return;
  for (int e = threadIdx.x; e < NC * NW; e += blockDim.x) lr[e] = R[e];
  for (int e = threadIdx.x; e < NC * NC; e += blockDim.x) ls[e] = S[e];
  __syncthreads();
  R = lr;
  S = ls;
}

template <int D, typename TS>
__device__ void forward_task(const GroupTask& t, int64_t u0) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  __shared__ TA lr[NC * NW], ls[NC * NC];
  const TA* R;
  const TA* S;
  stage_mats<TA, NC, NW>(t, lr, ls, R, S);
  const int64_t u = u0 + threadIdx.x;
  if (u >= t.units) return;
  int c[D];
  {
    int64_t rem = u;
#pragma unroll
    for (int ax = D - 1; ax >= 0; --ax) {
      c[ax] = static_cast<int>(rem % t.mi[ax]) + 1;
      rem /= t.mi[ax];
    }
  }
  const TS* s_in = static_cast<const TS*>(t.in);
  const TS* xi = static_cast<const TS*>(t.xi);
  TS* s_out = static_cast<TS*>(t.out);
  const TA* w = static_cast<const TA*>(t.w);
  TA win[NW];
#pragma unroll
  for (int iw = 0; iw < NW; ++iw) {
    int q[D];
    int rem = iw;
#pragma unroll
    for (int ax = D - 1; ax >= 0; --ax) {
      q[ax] = c[ax] + (rem % 3) - 1;
      rem /= 3;
    }
    win[iw] = load_acc(s_in + glin<D>(q, t.nc));
  }
  TA fresh[NC];
  int64_t fidx[NC];
#pragma unroll
  for (int ib = 0; ib < NC; ++ib) {
    int q[D];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) q[ax] = 2 * (c[ax] - 1) + ((ib >> (D - 1 - ax)) & 1);
    fidx[ib] = glin<D>(q, t.nf);
    fresh[ib] = load_acc(xi + fidx[ib]);
  }
  const int64_t stride = t.charted ? t.msets : 1;
  const int64_t base = t.charted ? (t.shell ? c[0] - 1 : u) : 0;
#pragma unroll
  for (int ib = 0; ib < NC; ++ib) {
    TA acc = 0;
#pragma unroll
    for (int iw = 0; iw < NW; ++iw) acc += R[(ib * NW + iw) * stride + base] * win[iw];
#pragma unroll
    for (int jb = 0; jb <= ib; ++jb) acc += S[(ib * NC + jb) * stride + base] * fresh[jb];
    if (w) acc *= w[fidx[ib]];
    store_acc(s_out + fidx[ib], acc);
  }
}

template <int D, typename TS>
__device__ void adjoint_task(const GroupTask& t, int64_t u0) {
  using TA = typename Acc<TS>::type;
  constexpr int NW = pow3(D);
  constexpr int NC = 1 << D;
  __shared__ TA lr[NC * NW], ls[NC * NC];
  const TA* R;
  const TA* S;
  stage_mats<TA, NC, NW>(t, lr, ls, R, S);
  const int64_t u = u0 + threadIdx.x;
  if (u >= t.units) return;
  int p[D];
  {
    int64_t rem = u;
#pragma unroll
    for (int ax = D - 1; ax >= 0; --ax) {
      p[ax] = static_cast<int>(rem % t.nc[ax]);
      rem /= t.nc[ax];
    }
  }
  const TS* y = static_cast<const TS*>(t.in);
  const int64_t stride = t.charted ? t.msets : 1;
  // blocks outside the interior are read at a clamped position and weighted by zero
  TA acc = 0;
#pragma unroll
  for (int iw = 0; iw < NW; ++iw) {
    int c[D];
    bool inside = true;
    int rem = iw;
#pragma unroll
    for (int ax = D - 1; ax >= 0; --ax) {
      const int cv = p[ax] - ((rem % 3) - 1);
      rem /= 3;
      inside = inside && cv >= 1 && cv <= t.nc[ax] - 2;
      c[ax] = min(max(cv, 1), t.nc[ax] - 2);
    }
    int64_t set = 0;
    if (t.charted) {
      int ci[D];
#pragma unroll
      for (int ax = 0; ax < D; ++ax) ci[ax] = c[ax] - 1;
      set = t.shell ? ci[0] : glin<D>(ci, t.mi);
    }
    TA part = 0;
#pragma unroll
    for (int ib = 0; ib < NC; ++ib) {
      int q[D];
#pragma unroll
      for (int ax = 0; ax < D; ++ax) q[ax] = 2 * (c[ax] - 1) + ((ib >> (D - 1 - ax)) & 1);
      part += R[(ib * NW + iw) * stride + set] * load_acc(y + glin<D>(q, t.nf));
    }
    acc += inside ? part : TA(0);
  }
  store_acc(static_cast<TS*>(t.out2) + u, acc);
  bool interior = true;
#pragma unroll
  for (int ax = 0; ax < D; ++ax) interior = interior && p[ax] >= 1 && p[ax] <= t.nc[ax] - 2;
  if (!interior) return;
  int64_t set = 0;
  if (t.charted) {
    int ci[D];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) ci[ax] = p[ax] - 1;
    set = t.shell ? ci[0] : glin<D>(ci, t.mi);
  }
  TA yb[NC];
  int64_t fidx[NC];
#pragma unroll
  for (int ib = 0; ib < NC; ++ib) {
    int q[D];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) q[ax] = 2 * (p[ax] - 1) + ((ib >> (D - 1 - ax)) & 1);
    fidx[ib] = glin<D>(q, t.nf);
    yb[ib] = load_acc(y + fidx[ib]);
  }
  TS* xb = static_cast<TS*>(t.out);
  const TS* add = static_cast<const TS*>(t.add);
#pragma unroll
  for (int jb = 0; jb < NC; ++jb) {
    TA v = 0;
#pragma unroll
    for (int ib = jb; ib < NC; ++ib) v += S[(ib * NC + jb) * stride + set] * yb[ib];
    if (add) v += load_acc(add + fidx[jb]);
    store_acc(xb + fidx[jb], v);
  }
}

// One workgroup's share of a grouped step; `tasks` is the device table or the task pack
// passed in the kernel arguments.
template <typename TS, typename Tasks>
__device__ __forceinline__ void group_step(const Tasks& tasks, int ntasks) {
  // the task of this workgroup: the last one whose first workgroup is <= blockIdx.x
  const int64_t wg = blockIdx.x;
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].wg0 <= wg) lo = mid;
    else hi = mid - 1;
  }
  const GroupTask t = tasks[lo];
  const int64_t u0 = (wg - t.wg0) * kGroupThreads;
  switch (t.kind) {
    case kTaskLevel0Fwd: level0_task<TS, true>(t, u0); break;
    case kTaskLevel0Adj: level0_task<TS, false>(t, u0); break;
    case kTaskFwd:
      if (t.d == 1) forward_task<1, TS>(t, u0);
      else if (t.d == 2) forward_task<2, TS>(t, u0);
      else forward_task<3, TS>(t, u0);
      break;
    default:
      if (t.d == 1) adjoint_task<1, TS>(t, u0);
      else if (t.d == 2) adjoint_task<2, TS>(t, u0);
      else adjoint_task<3, TS>(t, u0);
      break;
  }
}

template <typename TS>
__global__ void __launch_bounds__(kGroupThreads) grouped_step(const GroupTask* __restrict__ tasks, int ntasks) {
  group_step<TS>(tasks, ntasks);
}

// The same step with at most kInlineTasks tasks carried in the kernel arguments: no table
// copy has to precede the launch.
template <typename TS>
__global__ void __launch_bounds__(kGroupThreads) grouped_step_inline(TaskPack pack, int ntasks) {
  group_step<TS>(pack.t, ntasks);
}

}  // namespace

int64_t task_workgroups(const GroupTask& t) {
  const int64_t threads = (t.kind == kTaskLevel0Fwd || t.kind == kTaskLevel0Adj) ? t.n0 * 64 : t.units;
  return (threads + kGroupThreads - 1) / kGroupThreads;
}

hipError_t launch_grouped_step(int precision, const GroupTask* dev_tasks, int ntasks, int64_t workgroups,
                               hipStream_t st) {
  if (ntasks <= 0 || workgroups <= 0) return hipSuccess;
  if (workgroups > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(workgroups));
  switch (precision) {
    case ICR_F64: grouped_step<double><<<grid, kGroupThreads, 0, st>>>(dev_tasks, ntasks); break;
    case ICR_F32: grouped_step<float><<<grid, kGroupThreads, 0, st>>>(dev_tasks, ntasks); break;
    default: grouped_step<bf16_t><<<grid, kGroupThreads, 0, st>>>(dev_tasks, ntasks); break;
  }
  return hipGetLastError();
}

hipError_t launch_grouped_step_inline(int precision, const TaskPack& pack, int ntasks, int64_t workgroups,
                                      hipStream_t st) {
  if (ntasks <= 0 || workgroups <= 0) return hipSuccess;
  if (ntasks > kInlineTasks || workgroups > INT32_MAX) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(workgroups));
  switch (precision) {
    case ICR_F64: grouped_step_inline<double><<<grid, kGroupThreads, 0, st>>>(pack, ntasks); break;
    case ICR_F32: grouped_step_inline<float><<<grid, kGroupThreads, 0, st>>>(pack, ntasks); break;
    default: grouped_step_inline<bf16_t><<<grid, kGroupThreads, 0, st>>>(pack, ntasks); break;
  }
  return hipGetLastError();
}

// The steps of one sample's sweep as tasks (see grouped.h).
int sweep_tasks(const icr_plan* p, int op, const void* in, void* out, const void* w, void* ws, int64_t large,
                GroupTask* tasks, int* large_step) {
  const int el = p->elem_bytes;
  const int L = p->depth;
  const int d = p->ndim;
  auto at = [&](const void* base, int64_t elems) {
    return static_cast<char*>(const_cast<void*>(base)) + elems * el;
  };
  auto level_task = [&](int kind, int level) {
    GroupTask t{};
    t.kind = kind;
    t.d = d;
    t.charted = p->charted;
    t.shell = p->shell;
    for (int a = 0; a < 3; ++a) {
      t.nc[a] = a < d ? p->shapes[level][3 - d + a] : 1;
      t.nf[a] = a < d ? p->shapes[level + 1][3 - d + a] : 1;
      t.mi[a] = a < d ? t.nc[a] - 2 : 1;
    }
    int64_t interior = 1, coarse = 1;
    for (int a = 0; a < d; ++a) {
      interior *= t.mi[a];
      coarse *= t.nc[a];
    }
    t.units = kind == kTaskFwd ? interior : coarse;
    t.msets = p->lev[level].nsets;
    t.m0 = p->lev[level].r_c;
    t.m1 = p->lev[level].s_c;
    return t;
  };
  auto is_large = [&](int level) { return p->offsets[level + 2] - p->offsets[level + 1] >= large; };
  int n = 0;
  *large_step = 0;
  const bool metric = op == 2;
  // forward part (forward and metric): level 0 into the workspace (or the output when
  // the prior has no refinement), then every level; the last one to the output (forward)
  // or times w to the metric's fine cotangent slot in the workspace
  if (op == 0 || metric) {
    void* fine_out = metric ? at(ws, p->offsets[L]) : out;
    GroupTask t0{};
    t0.kind = kTaskLevel0Fwd;
    t0.d = d;
    t0.n0 = p->n0;
    t0.units = p->n0 * 64;
    t0.m0 = p->l00_c;
    t0.in = in;
    t0.out = L == 0 ? fine_out : at(ws, p->offsets[0]);
    t0.w = L == 0 ? w : nullptr;
    tasks[n++] = t0;
    for (int l = 0; l < L; ++l) {
      GroupTask t = level_task(kTaskFwd, l);
      t.in = at(ws, p->offsets[l]);
      t.xi = at(in, p->offsets[l + 1]);
      t.out = l == L - 1 ? fine_out : at(ws, p->offsets[l + 1]);
      t.w = l == L - 1 ? w : nullptr;
      t.level = l;
      if (is_large(l)) *large_step |= 1;
      tasks[n++] = t;
    }
  }
  // adjoint part (adjoint and metric): from the fine cotangent down to level 0
  if (op == 1 || metric) {
    const void* y = metric ? at(ws, p->offsets[L]) : in;
    const void* add = metric ? in : nullptr;
    for (int l = L - 1; l >= 0; --l) {
      GroupTask t = level_task(kTaskAdj, l);
      t.in = l == L - 1 ? y : at(ws, p->offsets[l + 1]);
      t.out = at(out, p->offsets[l + 1]);
      t.out2 = at(ws, p->offsets[l]);
      t.add = add ? at(add, p->offsets[l + 1]) : nullptr;
      t.level = l;
      if (is_large(l)) *large_step |= 1;
      tasks[n++] = t;
    }
    GroupTask t0{};
    t0.kind = kTaskLevel0Adj;
    t0.d = d;
    t0.n0 = p->n0;
    t0.units = p->n0 * 64;
    t0.m0 = p->u00_c;
    t0.in = L == 0 ? y : at(ws, p->offsets[0]);
    t0.out = out;
    t0.add = add;
    tasks[n++] = t0;
  }
  return n;
}

}  // namespace icr
