// Grouped sweep steps (grouped.hip): one launch applies one step of many independent
// sweeps, each with its own plan. Used by the request server.
#pragma once

#include "icr_internal.h"

namespace icr {

enum GroupTaskKind : int32_t { kTaskLevel0Fwd = 0, kTaskLevel0Adj = 1, kTaskFwd = 2, kTaskAdj = 3 };

// One step of one sample's sweep. Shapes are in natural axis order (first d used). The
// matrices are the plan's arithmetic-type copies: level 0 L00 (forward) or U00 = L00^T
// (adjoint) in m0; a refinement level R in m0, sqrtD in m1 (charted: entry-major with
// msets sets). Buffers are device pointers to this sample's level slices.
struct GroupTask {
  int32_t kind;
  int32_t d;
  int32_t charted;
  int32_t shell;
  int32_t nc[3];
  int32_t nf[3];
  int32_t mi[3];
  int32_t level;
  int64_t units;    // level 0: rows * 64 (a wavefront per row); forward: interior coarse
                    // pixels; adjoint: coarse pixels
  int64_t wg0;      // first workgroup of the task in its launch
  int64_t msets;    // charted: sets, the stride between a set's entries
  int64_t n0;       // level 0: matrix order
  const void* m0;
  const void* m1;
  const void* in;   // level-0 fwd: xi_0; level-0 adj: s_bar_0; fwd: s_l; adj: y_{l+1}
  const void* xi;   // fwd: xi_{l+1}
  void* out;        // level 0: s_0 / xi_bar_0; fwd: s_{l+1}; adj: xi_bar_{l+1}
  void* out2;       // adj: s_bar_l
  const void* w;    // forward epilogue of the final level: out *= w (arithmetic type)
  const void* add;  // adjoint epilogue: out += add (storage type)
};

// Up to kInlineTasks tasks of one grouped launch passed by value in the kernel arguments
// (about 1.3 KB), so a small group needs no table copy before its launches.
constexpr int kInlineTasks = 8;
struct TaskPack {
  GroupTask t[kInlineTasks];
};

// Workgroups a task takes in a grouped launch.
int64_t task_workgroups(const GroupTask& t);

// One grouped launch: dev_tasks (device copy, sorted by wg0 with wg0 of the first task 0)
// of one storage precision; `workgroups` = the sum of task_workgroups.
hipError_t launch_grouped_step(int precision, const GroupTask* dev_tasks, int ntasks, int64_t workgroups,
                               hipStream_t st);

// The same launch with the tasks (ntasks <= kInlineTasks, sorted by wg0, the first 0) in
// the kernel arguments.
hipError_t launch_grouped_step_inline(int precision, const TaskPack& pack, int ntasks, int64_t workgroups,
                                      hipStream_t st);

// The steps of one sample's sweep in order: op 0 forward (in = xi, out = s), 1 adjoint
// (in = s_bar, out = xi_bar), 2 metric (in = v, out = L^T (w * L v) + v, w the weights
// of this sample). ws: the sample's workspace (n_xi - n_out elements; n_xi for the
// metric), laid out as icr_forward / icr_metric_apply lay theirs out. Writes at most
// 2 (depth + 1) tasks (wg0 unset) and returns how many; *large_step is set when a
// refinement level has at least `large` fine pixels.
int sweep_tasks(const icr_plan* p, int op, const void* in, void* out, const void* w, void* ws, int64_t large,
                GroupTask* tasks, int* large_step);

}  // namespace icr
