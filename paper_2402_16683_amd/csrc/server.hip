// Served ICR: a request server with continuous batching.
//
// Callers submit forward / adjoint / metric requests against plans registered with the
// server, or against prior configurations whose plans a builder thread builds on first
// use and caches; each request brings its own device input and output buffers. A worker
// thread
//   1. retires work whose completion events have fired (records completion times, returns
//      memory to the arena, marks captured graphs free),
//   2. in grouped mode, gathers the pending requests on 2-D and 3-D priors whose
//      refinement levels are all below the large-step size, of any prior and op, oldest
//      first, into a group while fewer than group_streams groups run: every request's
//      workspace comes from the arena, the steps of all sweeps go to the device in one
//      table (a small group, at most eight tasks per launch, passes them in the kernel
//      arguments instead), and the k-th grouped launch applies the k-th step of every
//      sweep; each request's completion event follows its own last step,
//   3. forms homogeneous batches from the other pending requests with the same
//      (plan, op), oldest first, up to the largest power of two <= min(pending,
//      max_batch), admits a batch only if its buffers fit in the fixed HBM arena (first
//      fit), and launches it on a free stream: gather the inputs into a contiguous batch,
//      run the batched sweep (replaying a hipGraph captured once per (plan, op, batch
//      size) when graphs are enabled and the batch needs at most 1/32 of the arena;
//      larger batches launch eagerly), scatter the outputs, record an event. A single
//      request without a graph, or with input rows of 1 MiB or more, runs the sweep on
//      its own buffers (only its workspace comes from the arena).
// Requests that arrive while others run join the queue and are admitted as streams and
// memory free up, so work of different priors overlaps on the device. With max_batch = 1,
// one stream, no graphs and no grouping the same server is the one-launch-per-request
// baseline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <utility>
#include <unordered_map>
#include <vector>

#include "grouped.h"
#include "icr_internal.h"
#include "icr_server.h"

namespace {

constexpr int kMaxBatch = 64;
constexpr int kBuilders = 4;  // builder threads (and streams) of the plan cache
constexpr size_t kAlign = 256;

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct PtrTable {
  const void* p[kMaxBatch];
};

// rows[r] (n elements each) <-> contiguous [k][n]; 16-byte vectors when aligned
__global__ void gather_rows(PtrTable src, void* __restrict__ dst, int64_t bytes_per_row, int vec) {
  const int r = blockIdx.y;
  const char* s = static_cast<const char*>(src.p[r]);
  char* d = static_cast<char*>(dst) + r * bytes_per_row;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (vec) {
    const int64_t n = bytes_per_row / 16;
    for (int64_t i = t0; i < n; i += stride)
      reinterpret_cast<uint4*>(d)[i] = reinterpret_cast<const uint4*>(s)[i];
  } else {
    for (int64_t i = t0; i < bytes_per_row; i += stride) d[i] = s[i];
  }
}

__global__ void scatter_rows(const void* __restrict__ src, PtrTable dst, int64_t bytes_per_row, int vec) {
  const int r = blockIdx.y;
  const char* s = static_cast<const char*>(src) + r * bytes_per_row;
  char* d = static_cast<char*>(const_cast<void*>(dst.p[r]));
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (vec) {
    const int64_t n = bytes_per_row / 16;
    for (int64_t i = t0; i < n; i += stride)
      reinterpret_cast<uint4*>(d)[i] = reinterpret_cast<const uint4*>(s)[i];
  } else {
    for (int64_t i = t0; i < bytes_per_row; i += stride) d[i] = s[i];
  }
}

// First-fit allocator over one device arena.
class Arena {
 public:
  bool init(size_t bytes) {
    if (hipMalloc(&base_, bytes) != hipSuccess) return false;
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  ~Arena() {
    if (base_) (void)hipFree(base_);
  }
  void* alloc(size_t bytes) {
    bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_[off] = bytes;
        in_use_ += bytes;
        return static_cast<char*>(base_) + off;
      }
    }
    return nullptr;
  }
  void release(void* p) {
    const size_t off = static_cast<char*>(p) - static_cast<char*>(base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, len = u->second;
    used_.erase(u);
    in_use_ -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      free_.erase(next);
    }
    auto prev = free_.lower_bound(start);
    if (prev != free_.begin()) {
      --prev;
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t capacity() const { return size_; }
  size_t in_use() const { return in_use_; }

 private:
  void* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;
};

struct PlanEntry {
  const icr_plan* plan;
  int64_t n_xi, n_out;
  int elem, acc;
  bool large = false;   // a refinement level has at least large_step fine pixels
  // requests run on their own kernels, never in groups: large plans, and 1-D plans (their
  // own sweep runs the small levels in one fused launch where a group takes one launch
  // per level, and a long 1-D sweep held its group stream through all its steps)
  bool own = false;
  bool owned = false;   // built by the server for a prior configuration (destroyed with it)
  int64_t active = 0;   // requests pending or in flight
  double last_used = 0.0;
  std::string key;      // owned: the configuration it was built for
};

constexpr int kMaxSteps = 2 * (ICR_MAX_DEPTH + 1);  // steps of a metric sweep

// A group: requests of any prior and op whose sweeps advance one step per grouped
// launch, on one stream; each request's own event marks its end.
struct Group {
  std::vector<int64_t> ids;
  int stream = -1;
};

// The plan cache entry of a prior configuration.
struct CacheEntry {
  int state = 0;                 // 0 building, 1 ready, 2 failed
  int32_t plan_id = -1;
  icr_status status = ICR_OK;
  std::string message;
  std::vector<int64_t> waiting;  // requests submitted while the plan was built
};

struct Request {
  int32_t plan_id;
  int32_t op;
  const void* in;
  void* out;
  const void* w;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
  double t_submit = 0.0, t_launch = 0.0, t_done = 0.0;
  int32_t batch_size = 0;
  bool done = false;
  icr_status status = ICR_OK;  // the build status of a request whose plan failed to build
  std::string message;
  hipEvent_t finished = nullptr;  // grouped: recorded after the request's last step
  void* ws = nullptr;             // grouped: the request's workspace in the arena
};

// Device buffers of one batch: [k][n_in] inputs, [k][n_out_op] outputs, [k][n_out] w,
// the sweep workspace.
struct Buffers {
  void* in = nullptr;
  void* out = nullptr;
  void* w = nullptr;
  void* ws = nullptr;
  size_t bytes = 0;
};

struct Graph {
  hipGraphExec_t exec = nullptr;
  Buffers buf;
  bool busy = false;
  double last_used = 0.0;
};

struct Batch {
  std::vector<int64_t> ids;
  int32_t plan_id = 0, op = 0;
  int stream = -1;
  hipEvent_t done = nullptr;
  Buffers buf;          // owned when no graph is used
  Graph* graph = nullptr;
};

}  // namespace

struct icr_server {
  icr_server_config cfg{};
  Arena arena;
  std::vector<PlanEntry> plans;
  std::unordered_map<int64_t, Request> requests;
  std::deque<int64_t> pending;
  std::vector<hipStream_t> streams;
  std::vector<Batch*> inflight;  // per stream
  std::vector<Group*> grouped;   // per stream
  std::vector<hipEvent_t> event_pool;
  std::map<std::tuple<int, int, int>, std::vector<Graph*>> graphs;
  // grouped launches: per stream a pinned host table of steps and its device copy
  std::vector<icr::GroupTask*> host_tables;
  std::vector<icr::GroupTask*> dev_tables;
  size_t table_tasks = 0;        // tasks each table holds
  // plan cache of prior configurations and its builder thread
  std::map<std::string, CacheEntry> cache;
  std::deque<std::string> build_jobs;
  std::condition_variable build_cv;
  std::vector<std::thread> builders;      // builds of different configurations overlap
  std::vector<hipStream_t> build_streams; // one per builder
  int64_t next_id = 1;
  int64_t completed = 0, batches = 0, batched_requests = 0, graph_captures = 0, admissions_deferred = 0;
  int64_t groups = 0, grouped_requests = 0, plans_built = 0, plan_cache_hits = 0;
  std::string error;
  std::mutex mu;
  std::condition_variable cv;
  std::atomic<bool> stop{false};
  std::thread worker;
  int device = 0;
};

namespace {

size_t up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// input rows of at least this size are never gathered for a batch of one
constexpr size_t kDirectRowBytes = size_t(1) << 20;

int64_t in_elems(const PlanEntry& pe, int op) { return op == ICR_OP_ADJOINT ? pe.n_out : pe.n_xi; }
int64_t out_elems(const PlanEntry& pe, int op) { return op == ICR_OP_FORWARD ? pe.n_out : pe.n_xi; }
int64_t ws_elems(const PlanEntry& pe, int op) { return op == ICR_OP_METRIC ? pe.n_xi : pe.n_xi - pe.n_out; }

size_t batch_bytes(const PlanEntry& pe, int op, int k) {
  size_t b = up(size_t(k) * in_elems(pe, op) * pe.elem) + up(size_t(k) * out_elems(pe, op) * pe.elem) +
             up(size_t(k) * std::max<int64_t>(ws_elems(pe, op), 1) * pe.elem);
  if (op == ICR_OP_METRIC) b += up(size_t(k) * pe.n_out * pe.acc);
  return b;
}

// Allocate `bytes` of the arena; if it is full, evict idle captured graphs (least
// recently used first) until the request fits. Fails only while the memory is held by
// batches in flight, which retire and free it.
void* alloc_evicting(icr_server* s, size_t bytes) {
  if (void* p = s->arena.alloc(bytes)) return p;
  std::vector<std::pair<double, std::tuple<int, int, int>>> idle;
  for (auto& kv : s->graphs)
    for (Graph* h : kv.second)
      if (!h->busy) idle.push_back({h->last_used, kv.first});
  std::sort(idle.begin(), idle.end());
  for (auto& cand : idle) {
    auto& l2 = s->graphs[cand.second];
    for (size_t i = 0; i < l2.size(); ++i) {
      if (!l2[i]->busy && l2[i]->last_used == cand.first) {
        (void)hipGraphExecDestroy(l2[i]->exec);
        s->arena.release(l2[i]->buf.in);
        delete l2[i];
        l2.erase(l2.begin() + i);
        break;
      }
    }
    if (void* p = s->arena.alloc(bytes)) return p;
  }
  return nullptr;
}

// contiguous batch buffers: inputs, outputs, workspace (and weights) of k requests
bool carve_evicting(icr_server* s, const PlanEntry& pe, int op, int k, Buffers* b) {
  const size_t total = batch_bytes(pe, op, k);
  char* p = static_cast<char*>(alloc_evicting(s, total));
  if (!p) return false;
  b->bytes = total;
  b->in = p; p += up(size_t(k) * in_elems(pe, op) * pe.elem);
  b->out = p; p += up(size_t(k) * out_elems(pe, op) * pe.elem);
  b->ws = p; p += up(size_t(k) * std::max<int64_t>(ws_elems(pe, op), 1) * pe.elem);
  b->w = op == ICR_OP_METRIC ? p : nullptr;
  return true;
}

// the batched sweep on contiguous buffers
icr_status sweep(const PlanEntry& pe, int op, int k, const Buffers& b, hipStream_t st) {
  switch (op) {
    case ICR_OP_FORWARD: return icr_forward(pe.plan, k, b.in, b.out, b.ws, st);
    case ICR_OP_ADJOINT: return icr_adjoint(pe.plan, k, b.in, b.out, b.ws, st);
    default: return icr_metric_apply(pe.plan, k, b.w, pe.n_out, b.in, b.out, b.ws, st);
  }
}

hipError_t copy_rows(const std::vector<const void*>& ptrs, void* contiguous, int64_t bytes_per_row, bool gather,
                     hipStream_t st) {
  PtrTable t{};
  bool vec = bytes_per_row % 16 == 0 && (reinterpret_cast<uintptr_t>(contiguous) % 16) == 0;
  for (size_t r = 0; r < ptrs.size(); ++r) {
    t.p[r] = ptrs[r];
    vec = vec && (reinterpret_cast<uintptr_t>(ptrs[r]) % 16) == 0;
  }
  const int64_t units = vec ? bytes_per_row / 16 : bytes_per_row;
  const unsigned gx = static_cast<unsigned>(std::min<int64_t>(std::max<int64_t>((units + 255) / 256, 1), 1024));
  const dim3 grid(gx, static_cast<unsigned>(ptrs.size()));
  if (gather) gather_rows<<<grid, 256, 0, st>>>(t, contiguous, bytes_per_row, vec ? 1 : 0);
  else scatter_rows<<<grid, 256, 0, st>>>(contiguous, t, bytes_per_row, vec ? 1 : 0);
  return hipGetLastError();
}

// Carve a batch's buffers; if the arena is full, evict idle captured graphs (least
// recently used first) until the buffers fit. Fails only while the memory is held by
// batches in flight, which retire and free it.
Graph* find_graph(icr_server* s, const PlanEntry& pe, int plan_id, int op, int k, hipStream_t st, bool* oom) {
  auto& list = s->graphs[std::make_tuple(plan_id, op, k)];
  for (Graph* g : list)
    if (!g->busy) return g;
  // capture a new instance with its own buffers
  Graph* g = new Graph;
  if (!carve_evicting(s, pe, op, k, &g->buf)) {
    delete g;
    *oom = true;
    return nullptr;
  }
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    s->arena.release(g->buf.in);
    delete g;
    return nullptr;
  }
  const icr_status rs = sweep(pe, op, k, g->buf, st);
  const hipError_t ec = hipStreamEndCapture(st, &graph);
  if (rs != ICR_OK || ec != hipSuccess || hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    s->arena.release(g->buf.in);
    delete g;
    return nullptr;
  }
  (void)hipGraphDestroy(graph);
  ++s->graph_captures;
  list.push_back(g);
  return g;
}

// An event from the pool (created when the pool is empty); nullptr if creation fails.
hipEvent_t take_event(icr_server* s) {
  if (s->event_pool.empty()) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
    return ev;
  }
  hipEvent_t ev = s->event_pool.back();
  s->event_pool.pop_back();
  return ev;
}

// Record the batch's completion event and book it as in flight on stream `si`.
bool finish_launch(icr_server* s, int si, Batch* b, const std::vector<int64_t>& ids, hipError_t e) {
  hipStream_t st = s->streams[si];
  const int k = static_cast<int>(ids.size());
  b->done = take_event(s);
  if (e == hipSuccess && b->done) e = hipEventRecord(b->done, st);
  if (e != hipSuccess) s->error = std::string("batch launch: ") + hipGetErrorString(e);
  if (b->graph) {
    b->graph->busy = true;
    b->graph->last_used = now_s();
  }
  const double t = now_s();
  for (int64_t id : ids) {
    s->requests[id].t_launch = t;
    s->requests[id].batch_size = k;
  }
  s->inflight[si] = b;
  ++s->batches;
  s->batched_requests += k;
  return true;
}

bool stream_free(const icr_server* s, size_t si) { return !s->inflight[si] && !s->grouped[si]; }

// Launch a group on stream `si`: every request's workspace from the arena (requests that
// do not fit wait for the next group), the steps of all sweeps in one table copy, then
// per step and precision one grouped launch, and each request's event after its last
// step. `ids` is reduced to the requests admitted; false if none was.
bool launch_group(icr_server* s, int si, std::vector<int64_t>& ids) {
  hipStream_t st = s->streams[si];
  std::vector<int64_t> admitted;
  std::vector<std::vector<icr::GroupTask>> steps;  // per request
  for (int64_t id : ids) {
    Request& r = s->requests[id];
    const PlanEntry& pe = s->plans[r.plan_id];
    const size_t bytes = up(size_t(std::max<int64_t>(ws_elems(pe, r.op), 1)) * pe.elem);
    void* ws = alloc_evicting(s, bytes);
    if (!ws) {
      ++s->admissions_deferred;
      break;  // keep arrival order: later requests wait with this one
    }
    r.ws = ws;
    std::vector<icr::GroupTask> t(kMaxSteps);
    int large = 0;
    t.resize(icr::sweep_tasks(pe.plan, r.op, r.in, r.out, r.w, ws, INT64_MAX, t.data(), &large));
    steps.push_back(std::move(t));
    admitted.push_back(id);
  }
  ids = admitted;
  if (ids.empty()) return false;
  hipError_t e = hipSuccess;
  for (int64_t id : ids) {
    const Request& r = s->requests[id];
    if (e == hipSuccess && r.ready) e = hipStreamWaitEvent(st, r.ready, 0);
  }
  // the table: step k of every request, per precision, tasks sorted by first workgroup
  struct Launch {
    int precision;
    size_t first;
    int ntasks;
    int64_t workgroups;
  };
  std::vector<Launch> launches;
  std::vector<std::pair<size_t, int64_t>> last_launch;  // per request: launch index of its last step
  last_launch.assign(ids.size(), {0, 0});
  icr::GroupTask* host = s->host_tables[si];
  size_t used = 0;
  size_t max_steps = 0;
  for (const auto& t : steps) max_steps = std::max(max_steps, t.size());
  for (size_t k = 0; k < max_steps; ++k) {
    for (int prec = ICR_F64; prec <= ICR_BF16_F32ACC; ++prec) {
      Launch L{prec, used, 0, 0};
      for (size_t i = 0; i < ids.size(); ++i) {
        const Request& r = s->requests[ids[i]];
        if (k >= steps[i].size() || s->plans[r.plan_id].plan->precision != prec) continue;
        icr::GroupTask t = steps[i][k];
        t.wg0 = L.workgroups;
        L.workgroups += icr::task_workgroups(t);
        host[used++] = t;
        ++L.ntasks;
        if (k + 1 == steps[i].size()) last_launch[i] = {launches.size(), 0};
      }
      if (L.ntasks > 0) launches.push_back(L);
    }
  }
  // small groups (every launch at most kInlineTasks tasks, a lone request's sweep among
  // them) carry their tasks in the kernel arguments: no table copy precedes the launches
  bool inline_tasks = true;
  for (const Launch& L : launches) inline_tasks = inline_tasks && L.ntasks <= icr::kInlineTasks;
  if (e == hipSuccess && !inline_tasks)
    e = hipMemcpyAsync(s->dev_tables[si], host, used * sizeof(icr::GroupTask), hipMemcpyHostToDevice, st);
  Group* g = new Group;
  g->ids = ids;
  g->stream = si;
  for (size_t li = 0; li < launches.size() && e == hipSuccess; ++li) {
    const Launch& L = launches[li];
    if (inline_tasks) {
      icr::TaskPack pack;
      std::memset(&pack, 0, sizeof(pack));
      std::copy(host + L.first, host + L.first + L.ntasks, pack.t);
      e = icr::launch_grouped_step_inline(L.precision, pack, L.ntasks, L.workgroups, st);
    } else {
      e = icr::launch_grouped_step(L.precision, s->dev_tables[si] + L.first, L.ntasks, L.workgroups, st);
    }
    for (size_t i = 0; i < ids.size() && e == hipSuccess; ++i) {
      if (last_launch[i].first != li) continue;
      Request& r = s->requests[ids[i]];
      r.finished = take_event(s);
      e = r.finished ? hipEventRecord(r.finished, st) : hipErrorOutOfMemory;
    }
  }
  if (e != hipSuccess) s->error = std::string("group launch: ") + hipGetErrorString(e);
  const double t = now_s();
  for (int64_t id : ids) {
    Request& r = s->requests[id];
    r.t_launch = t;
    r.batch_size = static_cast<int32_t>(ids.size());
  }
  s->grouped[si] = g;
  ++s->groups;
  s->grouped_requests += static_cast<int64_t>(ids.size());
  return true;
}

// A request is done: times, counters, its plan's activity; events back to the pool.
void complete(icr_server* s, Request& r, double t) {
  r.t_done = t;
  r.done = true;
  if (r.ready) {
    s->event_pool.push_back(r.ready);
    r.ready = nullptr;
  }
  if (r.finished) {
    s->event_pool.push_back(r.finished);
    r.finished = nullptr;
  }
  if (r.plan_id >= 0) {
    PlanEntry& pe = s->plans[r.plan_id];
    pe.active -= 1;
    pe.last_used = t;
  }
  ++s->completed;
}


// Launch one batch on stream `si`; returns false if it could not be admitted (memory).
bool launch_batch(icr_server* s, int si, std::vector<int64_t>& ids) {
  const Request& r0 = s->requests[ids[0]];
  const PlanEntry& pe = s->plans[r0.plan_id];
  const int op = r0.op;
  const int k = static_cast<int>(ids.size());
  hipStream_t st = s->streams[si];
  // the batch reads its requests' inputs only after the work their callers queued before
  // submitting (waits issued before any capture, so a captured graph holds none of them)
  for (int64_t id : ids) {
    const Request& r = s->requests[id];
    if (r.ready && hipStreamWaitEvent(st, r.ready, 0) != hipSuccess) {
      s->error = "hipStreamWaitEvent on a request's ready event failed";
      return false;
    }
  }
  Batch* b = new Batch;
  b->ids = ids;
  b->plan_id = r0.plan_id;
  b->op = op;
  b->stream = si;
  Buffers buf;
  // graphs pay off for small, launch-bound batches; a batch larger than 1/32 of the
  // arena runs eagerly so captured graphs never crowd the arena (evicting and
  // recapturing them would cost more host time than the launches they save)
  // a lone request with large rows runs on its own buffers even with graphs on: the
  // gather and scatter around a replay would move its rows twice more, which costs the
  // device more time than the launches a replay saves the host
  const bool direct = k == 1 && size_t(in_elems(pe, op)) * pe.elem >= kDirectRowBytes;
  const bool use_graph = s->cfg.use_graphs && !direct && batch_bytes(pe, op, k) * 32 <= s->arena.capacity();
  if (use_graph) {
    bool oom = false;
    b->graph = find_graph(s, pe, r0.plan_id, op, k, st, &oom);
    if (!b->graph) {
      delete b;
      if (!oom) s->error = "graph capture failed";
      return false;
    }
    buf = b->graph->buf;
  } else if (k == 1) {
    // one request without a graph: sweep its own buffers, only the workspace comes from
    // the arena (no gather or scatter launch)
    const size_t bytes = up(size_t(std::max<int64_t>(ws_elems(pe, op), 1)) * pe.elem);
    void* ws = alloc_evicting(s, bytes);
    if (!ws) {
      delete b;
      return false;
    }
    b->buf.in = ws;  // the arena allocation, released when the batch retires
    b->buf.bytes = bytes;
    Buffers d;
    d.in = const_cast<void*>(r0.in);
    d.out = r0.out;
    d.ws = ws;
    d.w = const_cast<void*>(r0.w);
    const hipError_t e = sweep(pe, op, 1, d, st) == ICR_OK ? hipSuccess : hipErrorLaunchFailure;
    return finish_launch(s, si, b, ids, e);
  } else {
    if (!carve_evicting(s, pe, op, k, &b->buf)) {
      delete b;
      return false;
    }
    buf = b->buf;
  }
  std::vector<const void*> in_ptrs, out_ptrs, w_ptrs;
  for (int64_t id : ids) {
    const Request& r = s->requests[id];
    in_ptrs.push_back(r.in);
    out_ptrs.push_back(r.out);
    w_ptrs.push_back(r.w);
  }
  hipError_t e = copy_rows(in_ptrs, buf.in, in_elems(pe, op) * pe.elem, true, st);
  if (e == hipSuccess && op == ICR_OP_METRIC) e = copy_rows(w_ptrs, buf.w, pe.n_out * pe.acc, true, st);
  if (e == hipSuccess) {
    if (b->graph) e = hipGraphLaunch(b->graph->exec, st);
    else if (sweep(pe, op, k, buf, st) != ICR_OK) e = hipErrorLaunchFailure;
  }
  if (e == hipSuccess) e = copy_rows(out_ptrs, buf.out, out_elems(pe, op) * pe.elem, false, st);
  return finish_launch(s, si, b, ids, e);
}

void retire(icr_server* s) {
  for (size_t si = 0; si < s->inflight.size(); ++si) {
    Batch* b = s->inflight[si];
    if (!b) continue;
    if (b->done && hipEventQuery(b->done) == hipErrorNotReady) continue;
    const double t = now_s();
    for (int64_t id : b->ids) complete(s, s->requests[id], t);
    if (b->graph) b->graph->busy = false;
    else if (b->buf.in) s->arena.release(b->buf.in);
    if (b->done) s->event_pool.push_back(b->done);
    delete b;
    s->inflight[si] = nullptr;
  }
  for (size_t si = 0; si < s->grouped.size(); ++si) {
    Group* g = s->grouped[si];
    if (!g) continue;
    bool all = true;
    for (int64_t id : g->ids) {
      Request& r = s->requests[id];
      if (r.done) continue;
      if (r.finished && hipEventQuery(r.finished) == hipErrorNotReady) {
        all = false;
        continue;
      }
      if (r.ws) s->arena.release(r.ws);
      r.ws = nullptr;
      complete(s, r, now_s());
    }
    if (all) {
      delete g;
      s->grouped[si] = nullptr;
    }
  }
}

bool groupable(const icr_server* s, const Request& r) {
  return s->cfg.grouped && !s->plans[r.plan_id].own;
}

void remove_pending(icr_server* s, const std::vector<int64_t>& ids) {
  for (int64_t id : ids) {
    auto it = std::find(s->pending.begin(), s->pending.end(), id);
    if (it != s->pending.end()) s->pending.erase(it);
  }
}

// Form and launch groups and batches on free streams; oldest pending request first.
void schedule(icr_server* s) {
  if (s->cfg.grouped) {
    int running = 0;
    for (Group* g : s->grouped) running += g != nullptr;
    for (size_t si = 0; si < s->streams.size() && running < s->cfg.group_streams; ++si) {
      if (!stream_free(s, si)) continue;
      std::vector<int64_t> ids;
      for (int64_t id : s->pending) {
        if (groupable(s, s->requests[id])) ids.push_back(id);
        if (static_cast<int>(ids.size()) >= s->cfg.max_batch) break;
      }
      if (ids.empty() || !launch_group(s, static_cast<int>(si), ids)) break;
      remove_pending(s, ids);
      ++running;
    }
  }
  for (size_t si = 0; si < s->inflight.size() && !s->pending.empty(); ++si) {
    if (!stream_free(s, si)) continue;
    int64_t head = -1;
    for (int64_t id : s->pending)
      if (!groupable(s, s->requests[id])) {
        head = id;
        break;
      }
    if (head < 0) break;
    const Request& rh = s->requests[head];
    std::vector<int64_t> ids;
    for (int64_t id : s->pending) {
      const Request& r = s->requests[id];
      if (r.plan_id == rh.plan_id && r.op == rh.op) ids.push_back(id);
      if (static_cast<int>(ids.size()) >= s->cfg.max_batch) break;
    }
    size_t k = 1;
    while (k * 2 <= ids.size()) k *= 2;
    ids.resize(k);
    bool admitted = false;
    while (!ids.empty()) {
      if (launch_batch(s, static_cast<int>(si), ids)) {
        admitted = true;
        break;
      }
      ++s->admissions_deferred;
      if (ids.size() == 1) break;
      ids.resize(ids.size() / 2);  // a smaller batch may fit
    }
    if (!admitted) break;  // wait for memory to free up; keep arrival order
    remove_pending(s, ids);
  }
}

bool any_in_flight(const icr_server* s) {
  for (size_t si = 0; si < s->streams.size(); ++si)
    if (!stream_free(s, si)) return true;
  return false;
}

// Host-side sizes of a prior configuration (the plan's n_xi and n_out).
void config_sizes(const icr_config& c, int64_t* n_xi, int64_t* n_out) {
  int64_t total = 0, last = 0;
  int64_t n[3] = {1, 1, 1};
  for (int a = 0; a < c.ndim; ++a) n[a] = c.shape0[a];
  for (int l = 0; l <= c.depth; ++l) {
    last = n[0] * n[1] * n[2];
    total += last;
    for (int a = 0; a < c.ndim; ++a) n[a] = 2 * (n[a] - 2);
  }
  *n_xi = total;
  *n_out = last;
}

bool plan_is_large(const icr_plan* p, int64_t large) {
  for (int l = 0; l < p->depth; ++l)
    if (p->offsets[l + 2] - p->offsets[l + 1] >= large) return true;
  return false;
}

int32_t add_plan(icr_server* s, const icr_plan* plan, bool owned, const std::string& key) {
  PlanEntry pe{plan, plan->n_xi, plan->n_out, plan->elem_bytes, plan->precision == ICR_F64 ? 8 : 4};
  pe.large = plan_is_large(plan, s->cfg.large_step);
  pe.own = pe.large || plan->ndim == 1;
  pe.owned = owned;
  pe.key = key;
  pe.last_used = now_s();
  s->plans.push_back(pe);
  return static_cast<int32_t>(s->plans.size() - 1);
}

// Destroy the least recently used idle plans the server built while the cache holds
// more than max_plans ready entries (entries stay as tombstones: their plan_id is reset).
void evict_plans(icr_server* s) {
  for (;;) {
    int ready = 0;
    for (auto& kv : s->cache) ready += kv.second.state == 1;
    if (ready <= s->cfg.max_plans) return;
    std::string victim;
    double oldest = 0.0;
    for (auto& kv : s->cache) {
      if (kv.second.state != 1) continue;
      const PlanEntry& pe = s->plans[kv.second.plan_id];
      if (pe.active > 0) continue;
      if (victim.empty() || pe.last_used < oldest) {
        victim = kv.first;
        oldest = pe.last_used;
      }
    }
    if (victim.empty()) return;
    PlanEntry& pe = s->plans[s->cache[victim].plan_id];
    // idle graphs captured for the plan go with it
    for (auto& kv : s->graphs) {
      if (std::get<0>(kv.first) != s->cache[victim].plan_id) continue;
      for (Graph* g : kv.second) {
        (void)hipGraphExecDestroy(g->exec);
        s->arena.release(g->buf.in);
        delete g;
      }
      kv.second.clear();
    }
    (void)icr_plan_destroy(const_cast<icr_plan*>(pe.plan));
    pe.plan = nullptr;
    s->cache.erase(victim);
  }
}

// Builder thread: builds the plans of new prior configurations on its own stream while
// the worker keeps serving; the requests waiting for a plan become pending when it is
// ready, or complete with the build's status when it fails.
void builder_loop(icr_server* s, int index) {
  (void)hipSetDevice(s->device);
  hipStream_t build_stream = s->build_streams[index];
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    if (s->build_jobs.empty()) {
      s->build_cv.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    const std::string key = s->build_jobs.front();
    s->build_jobs.pop_front();
    icr_config cfg;
    std::memcpy(&cfg, key.data(), sizeof(cfg));
    lk.unlock();
    icr_plan* plan = nullptr;
    const icr_status st = icr_build_matrices(&cfg, build_stream, &plan);
    const std::string msg = st == ICR_OK ? std::string() : std::string(icr_last_error());
    lk.lock();
    CacheEntry& ce = s->cache[key];
    const double t = now_s();
    if (st == ICR_OK) {
      ce.state = 1;
      ce.plan_id = add_plan(s, plan, true, key);
      ++s->plans_built;
      PlanEntry& pe = s->plans[ce.plan_id];
      for (int64_t id : ce.waiting) {
        Request& r = s->requests[id];
        r.plan_id = ce.plan_id;
        pe.active += 1;
        // back into arrival order among the pending requests
        auto it = std::lower_bound(s->pending.begin(), s->pending.end(), id);
        s->pending.insert(it, id);
      }
    } else {
      ce.state = 2;
      ce.status = st;
      ce.message = msg;
      for (int64_t id : ce.waiting) {
        Request& r = s->requests[id];
        r.status = st;
        r.message = msg;
        r.plan_id = -1;
        complete(s, r, t);
      }
    }
    ce.waiting.clear();
    evict_plans(s);
    s->cv.notify_one();
  }
}

void worker_loop(icr_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    retire(s);
    schedule(s);
    const bool busy = any_in_flight(s);
    if (!busy && s->pending.empty()) {
      s->cv.wait_for(lk, std::chrono::milliseconds(2));
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(5));
      lk.lock();
    }
  }
}

}  // namespace

extern "C" {

icr_status icr_server_create(const icr_server_config* cfg, icr_server** out) {
  icr::clear_error();
  if (!cfg || !out) {
    icr::set_error("cfg or out is NULL");
    return ICR_ERR_INVALID_ARG;
  }
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > kMaxBatch || cfg->n_streams < 1 || cfg->n_streams > 16 ||
      cfg->hbm_budget_bytes < int64_t(kAlign) || cfg->large_step < 0 || cfg->group_streams < 0 ||
      cfg->group_streams > cfg->n_streams || cfg->max_plans < 0 || (cfg->grouped != 0 && cfg->grouped != 1)) {
    icr::set_error("max_batch must be 1..64, n_streams 1..16, hbm_budget_bytes >= 256, grouped 0 or 1, "
                   "large_step >= 0, group_streams 0..n_streams, max_plans >= 0");
    return ICR_ERR_INVALID_ARG;
  }
  icr_server* s = new icr_server;
  s->cfg = *cfg;
  if (s->cfg.large_step == 0) s->cfg.large_step = int64_t(1) << 20;
  if (s->cfg.group_streams == 0) s->cfg.group_streams = 1;
  if (s->cfg.max_plans == 0) s->cfg.max_plans = 256;
  (void)hipGetDevice(&s->device);
  if (!s->arena.init(static_cast<size_t>(cfg->hbm_budget_bytes))) {
    delete s;
    icr::set_error("could not allocate the server's HBM arena");
    return ICR_ERR_OUT_OF_MEMORY;
  }
  for (int i = 0; i < cfg->n_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      icr::set_error("hipStreamCreate failed");
      return ICR_ERR_HIP;
    }
    s->streams.push_back(st);
  }
  s->inflight.assign(cfg->n_streams, nullptr);
  s->grouped.assign(cfg->n_streams, nullptr);
  s->table_tasks = size_t(kMaxSteps) * kMaxBatch;
  bool ok = true;
  for (int i = 0; i < kBuilders && ok; ++i) {
    hipStream_t bs = nullptr;
    ok = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) == hipSuccess;
    if (ok) s->build_streams.push_back(bs);
  }
  for (int i = 0; i < cfg->n_streams && ok; ++i) {
    void* h = nullptr;
    void* d = nullptr;
    ok = hipHostMalloc(&h, s->table_tasks * sizeof(icr::GroupTask), hipHostMallocDefault) == hipSuccess;
    s->host_tables.push_back(static_cast<icr::GroupTask*>(h));
    if (ok) ok = hipMalloc(&d, s->table_tasks * sizeof(icr::GroupTask)) == hipSuccess;
    s->dev_tables.push_back(static_cast<icr::GroupTask*>(d));
  }
  if (!ok) {
    for (void* h : s->host_tables)
      if (h) (void)hipHostFree(h);
    for (void* d : s->dev_tables)
      if (d) (void)hipFree(d);
    for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    for (hipStream_t x : s->build_streams) (void)hipStreamDestroy(x);
    delete s;
    icr::set_error("could not allocate the server's step tables or build stream");
    return ICR_ERR_OUT_OF_MEMORY;
  }
  s->worker = std::thread(worker_loop, s);
  for (int i = 0; i < kBuilders; ++i) s->builders.emplace_back(builder_loop, s, i);
  *out = s;
  return ICR_OK;
}

icr_status icr_server_register_plan(icr_server* s, const icr_plan* plan, int32_t* plan_id) {
  icr::clear_error();
  if (!s || !plan || !plan_id) {
    icr::set_error("server, plan or plan_id is NULL");
    return ICR_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  *plan_id = add_plan(s, plan, false, std::string());
  return ICR_OK;
}

icr_status icr_server_submit(icr_server* s, int32_t plan_id, int32_t op, const void* in, void* out,
                             const void* w, void* hip_stream, int64_t* request_id) {
  icr::clear_error();
  if (!s || !in || !out || !request_id) {
    icr::set_error("server, in, out or request_id is NULL");
    return ICR_ERR_INVALID_ARG;
  }
  if (op < ICR_OP_FORWARD || op > ICR_OP_METRIC || (op == ICR_OP_METRIC && !w)) {
    icr::set_error("unknown op, or a metric request without w");
    return ICR_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (plan_id < 0 || plan_id >= static_cast<int32_t>(s->plans.size()) || !s->plans[plan_id].plan) {
    icr::set_error("unknown plan_id");
    return ICR_ERR_INVALID_ARG;
  }
  PlanEntry& pe = s->plans[plan_id];
  if (batch_bytes(pe, op, 1) > s->arena.capacity()) {
    icr::set_error("request needs more memory than the server's HBM budget");
    return ICR_ERR_OUT_OF_MEMORY;
  }
  Request r;
  r.plan_id = plan_id;
  r.op = op;
  r.in = in;
  r.out = out;
  r.w = w;
  if (s->event_pool.empty()) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      icr::set_error("hipEventCreate failed");
      return ICR_ERR_HIP;
    }
    s->event_pool.push_back(ev);
  }
  r.ready = s->event_pool.back();
  if (hipEventRecord(r.ready, static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
    icr::set_error("hipEventRecord on the caller's stream failed");
    return ICR_ERR_HIP;
  }
  s->event_pool.pop_back();
  r.t_submit = now_s();
  const int64_t id = s->next_id++;
  s->requests[id] = r;
  s->pending.push_back(id);
  pe.active += 1;
  *request_id = id;
  s->cv.notify_one();
  return ICR_OK;
}

icr_status icr_server_submit_prior(icr_server* s, const icr_config* cfg, int32_t op, const void* in, void* out,
                                   const void* w, void* hip_stream, int64_t* request_id) {
  icr::clear_error();
  if (!s || !cfg || !in || !out || !request_id) {
    icr::set_error("server, cfg, in, out or request_id is NULL");
    return ICR_ERR_INVALID_ARG;
  }
  if (op < ICR_OP_FORWARD || op > ICR_OP_METRIC || (op == ICR_OP_METRIC && !w)) {
    icr::set_error("unknown op, or a metric request without w");
    return ICR_ERR_INVALID_ARG;
  }
  if (cfg->ndim < 1 || cfg->ndim > 3 || cfg->depth < 0 || cfg->depth > ICR_MAX_DEPTH ||
      cfg->precision < ICR_F64 || cfg->precision > ICR_BF16_F32ACC) {
    icr::set_error("invalid prior configuration");
    return ICR_ERR_INVALID_ARG;
  }
  for (int a = 0; a < cfg->ndim; ++a)
    if (cfg->shape0[a] < 3 || cfg->shape0[a] > 65536) {
      icr::set_error("invalid prior configuration (level-0 shape)");
      return ICR_ERR_INVALID_ARG;
    }
  const std::string key(reinterpret_cast<const char*>(cfg), sizeof(icr_config));
  std::lock_guard<std::mutex> lk(s->mu);
  // the buffers the request needs, from sizes alone: refused now if they never fit
  PlanEntry sizes{nullptr, 0, 0, cfg->precision == ICR_F64 ? 8 : cfg->precision == ICR_F32 ? 4 : 2,
                  cfg->precision == ICR_F64 ? 8 : 4};
  config_sizes(*cfg, &sizes.n_xi, &sizes.n_out);
  if (batch_bytes(sizes, op, 1) > s->arena.capacity()) {
    icr::set_error("request needs more memory than the server's HBM budget");
    return ICR_ERR_OUT_OF_MEMORY;
  }
  Request r;
  r.plan_id = -1;
  r.op = op;
  r.in = in;
  r.out = out;
  r.w = w;
  r.ready = take_event(s);
  if (!r.ready || hipEventRecord(r.ready, static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
    if (r.ready) s->event_pool.push_back(r.ready);
    icr::set_error("hipEventRecord on the caller's stream failed");
    return ICR_ERR_HIP;
  }
  r.t_submit = now_s();
  const int64_t id = s->next_id++;
  auto it = s->cache.find(key);
  if (it == s->cache.end()) {
    CacheEntry ce;
    ce.waiting.push_back(id);
    s->cache.emplace(key, std::move(ce));
    s->build_jobs.push_back(key);
    s->build_cv.notify_one();
  } else if (it->second.state == 0) {
    it->second.waiting.push_back(id);
    ++s->plan_cache_hits;
  } else if (it->second.state == 1) {
    r.plan_id = it->second.plan_id;
    s->plans[r.plan_id].active += 1;
    ++s->plan_cache_hits;
  } else {  // the configuration failed to build before: fail the same way
    s->event_pool.push_back(r.ready);
    icr::set_error(it->second.message);
    return it->second.status;
  }
  s->requests[id] = r;
  if (r.plan_id >= 0) s->pending.push_back(id);
  *request_id = id;
  s->cv.notify_one();
  return ICR_OK;
}

icr_status icr_server_query(icr_server* s, int64_t request_id, int32_t* done, double* t_submit,
                            double* t_launch, double* t_done, int32_t* batch_size) {
  icr::clear_error();
  if (!s || !done) {
    icr::set_error("server or done is NULL");
    return ICR_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(request_id);
  if (it == s->requests.end()) {
    icr::set_error("unknown request_id");
    return ICR_ERR_INVALID_ARG;
  }
  const Request& r = it->second;
  *done = r.done ? 1 : 0;
  if (t_submit) *t_submit = r.t_submit;
  if (t_launch) *t_launch = r.t_launch;
  if (t_done) *t_done = r.t_done;
  if (batch_size) *batch_size = r.batch_size;
  if (r.status != ICR_OK) {
    icr::set_error("the prior's plan could not be built: " + r.message);
    return r.status;
  }
  return ICR_OK;
}

icr_status icr_server_drain(icr_server* s, double timeout_s) {
  icr::clear_error();
  if (!s) {
    icr::set_error("server is NULL");
    return ICR_ERR_INVALID_ARG;
  }
  const double t0 = now_s();
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      bool busy = !s->pending.empty() || any_in_flight(s) || !s->build_jobs.empty();
      for (auto& kv : s->cache) busy = busy || kv.second.state == 0;
      if (!s->error.empty()) {
        icr::set_error(s->error);
        return ICR_ERR_HIP;
      }
      if (!busy) return ICR_OK;
    }
    if (timeout_s > 0 && now_s() - t0 > timeout_s) {
      icr::set_error("drain timed out");
      return ICR_ERR_HIP;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

icr_status icr_server_stats(icr_server* s, icr_server_statistics* st) {
  icr::clear_error();
  if (!s || !st) {
    icr::set_error("server or stats is NULL");
    return ICR_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  st->completed = s->completed;
  st->pending = static_cast<int64_t>(s->pending.size());
  st->batches = s->batches;
  st->batched_requests = s->batched_requests;
  st->graph_captures = s->graph_captures;
  st->admissions_deferred = s->admissions_deferred;
  st->arena_bytes = static_cast<int64_t>(s->arena.capacity());
  st->arena_in_use = static_cast<int64_t>(s->arena.in_use());
  st->groups = s->groups;
  st->grouped_requests = s->grouped_requests;
  st->plans_built = s->plans_built;
  st->plan_cache_hits = s->plan_cache_hits;
  return ICR_OK;
}

icr_status icr_server_destroy(icr_server* s) {
  icr::clear_error();
  if (!s) return ICR_OK;
  s->stop.store(true);
  s->cv.notify_one();
  s->build_cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (std::thread& b : s->builders)
    if (b.joinable()) b.join();
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (hipStream_t st : s->build_streams) (void)hipStreamSynchronize(st);
  for (Batch* b : s->inflight) delete b;
  for (Group* g : s->grouped) delete g;
  for (auto& kv : s->requests) {
    if (kv.second.finished) (void)hipEventDestroy(kv.second.finished);
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  }
  for (PlanEntry& pe : s->plans)
    if (pe.owned && pe.plan) (void)icr_plan_destroy(const_cast<icr_plan*>(pe.plan));
  for (void* h : s->host_tables)
    if (h) (void)hipHostFree(h);
  for (void* d : s->dev_tables)
    if (d) (void)hipFree(d);
  for (hipStream_t st : s->build_streams) (void)hipStreamDestroy(st);
  for (auto& kv : s->graphs)
    for (Graph* g : kv.second) {
      if (g->exec) (void)hipGraphExecDestroy(g->exec);
      delete g;
    }
  for (hipEvent_t e : s->event_pool)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return ICR_OK;
}

}  // extern "C"
