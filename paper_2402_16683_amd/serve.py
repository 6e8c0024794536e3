"""Served ICR: binding of the request server (include/icr_server.h) and a driver that
plays a Poisson stream of mixed forward / adjoint / metric requests through it.

The server (C++ in libicr.so) does the batching, admission and launching; this module
only marshals arguments, draws the synthetic request stream and summarises latencies.
"""

from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import icr as B

OPS = {"forward": 0, "adjoint": 1, "metric": 2}


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("use_graphs", ctypes.c_int32), ("grouped", ctypes.c_int32),
                ("large_step", ctypes.c_int64), ("group_streams", ctypes.c_int32), ("max_plans", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("completed", "pending", "batches", "batched_requests",
                                              "graph_captures", "admissions_deferred", "arena_bytes",
                                              "arena_in_use", "groups", "grouped_requests", "plans_built",
                                              "plan_cache_hits")]


def _lib():
    lib = B.load_library()
    if not getattr(lib, "_server_bound", False):
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sigs = {
            "icr_server_create": [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)],
            "icr_server_register_plan": [vp, vp, ctypes.POINTER(i32)],
            "icr_server_submit": [vp, i32, i32, vp, vp, vp, vp, ctypes.POINTER(i64)],
            "icr_server_submit_prior": [vp, ctypes.POINTER(B.IcrConfig), i32, vp, vp, vp, vp, ctypes.POINTER(i64)],
            "icr_server_query": [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                 ctypes.POINTER(dbl), ctypes.POINTER(i32)],
            "icr_server_drain": [vp, dbl],
            "icr_server_stats": [vp, ctypes.POINTER(ServerStats)],
            "icr_server_destroy": [vp],
        }
        for name, args in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib._server_bound = True
    return lib


class Server:
    """An icr_server: continuous batching of ICR requests on the current device."""

    def __init__(self, hbm_budget_bytes: int, max_batch: int = 16, n_streams: int = 4, use_graphs: bool = True,
                 grouped: bool = False, large_step: int = 0, group_streams: int = 0, max_plans: int = 0):
        cfg = ServerConfig(hbm_budget_bytes, max_batch, n_streams, 1 if use_graphs else 0, 1 if grouped else 0,
                           large_step, group_streams, max_plans)
        self.handle = ctypes.c_void_p()
        B._check(_lib().icr_server_create(ctypes.byref(cfg), ctypes.byref(self.handle)))
        self.plans = []
        self._held = {}   # request id -> tensors the request reads or writes, until it is done

    def register(self, plan: B.Plan) -> int:
        pid = ctypes.c_int32()
        B._check(_lib().icr_server_register_plan(self.handle, plan.handle, ctypes.byref(pid)))
        self.plans.append(plan)
        return pid.value

    def submit(self, plan_id: int, op: str, inp, out, w=None, stream=None) -> int:
        """Queue one request; `inp` and `w` may still be in production on `stream` (default:
        torch's current stream): the request waits for the work queued there before this
        call. The tensors are kept alive here until the request is reported done."""
        rid = ctypes.c_int64()
        B._check(_lib().icr_server_submit(self.handle, plan_id, OPS[op], inp.data_ptr(), out.data_ptr(),
                                          None if w is None else w.data_ptr(), B._stream_handle(stream),
                                          ctypes.byref(rid)))
        self._held[rid.value] = (inp, out, w)
        return rid.value

    def submit_prior(self, cfg: B.IcrConfig, op: str, inp, out, w=None, stream=None) -> int:
        """Queue one request against a prior configuration; the server builds its plan on
        first use (inside that request's latency) and caches it."""
        rid = ctypes.c_int64()
        B._check(_lib().icr_server_submit_prior(self.handle, ctypes.byref(cfg), OPS[op], inp.data_ptr(),
                                                out.data_ptr(), None if w is None else w.data_ptr(),
                                                B._stream_handle(stream), ctypes.byref(rid)))
        self._held[rid.value] = (inp, out, w)
        return rid.value

    def query(self, rid: int):
        done, ts, tl, td, bs = (ctypes.c_int32(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double(),
                                ctypes.c_int32())
        B._check(_lib().icr_server_query(self.handle, rid, ctypes.byref(done), ctypes.byref(ts), ctypes.byref(tl),
                                         ctypes.byref(td), ctypes.byref(bs)))
        if done.value:
            self._held.pop(rid, None)
        return bool(done.value), ts.value, tl.value, td.value, bs.value

    def drain(self, timeout_s: float = 0.0):
        B._check(_lib().icr_server_drain(self.handle, timeout_s))
        self._held.clear()   # nothing is pending or in flight after a successful drain

    def stats(self) -> dict:
        st = ServerStats()
        B._check(_lib().icr_server_stats(self.handle, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            B._check(_lib().icr_server_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- workload

@dataclass
class Prior:
    ndim: int
    n0: int
    depth: int
    kernel: str
    length: float

    def config(self, precision: str = "f32") -> B.IcrConfig:
        return B.make_config(self.ndim, (self.n0,) * self.ndim, self.depth, (self.delta0,) * self.ndim,
                             kernel=self.kernel, length=self.length, precision=precision)

    @property
    def sizes(self):
        """(n_xi, n_out) of the prior: level sizes n_{l+1} = 2 (n_l - 2)."""
        n, total = self.n0, 0
        for _ in range(self.depth + 1):
            total += n ** self.ndim
            last = n ** self.ndim
            n = 2 * (n - 2)
        return total, last

    @property
    def delta0(self) -> float:
        # final-grid extent 1: delta_L = 1 / n_L, delta_0 = 2^L / n_L
        n = self.n0
        for _ in range(self.depth):
            n = 2 * (n - 2)
        return 2.0 ** self.depth / n


def draw_priors(n_priors: int, seed: int) -> list:
    """A pool of priors mixing 1-D (level-0 8-64, 4-10 levels), 2-D (8-32, 4-7 levels) and
    3-D (6-12, 3-5 levels) with Matern-3/2 or -5/2 kernels and log-uniform length scales in
    [0.05, 0.3]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_priors):
        d = 1 + i % 3
        lo, hi, dlo, dhi = {1: (8, 64, 4, 10), 2: (8, 32, 4, 7), 3: (6, 12, 3, 5)}[d]
        out.append(Prior(d, int(rng.integers(lo, hi + 1)), int(rng.integers(dlo, dhi + 1)),
                         "matern32" if rng.random() < 0.5 else "matern52",
                         float(math.exp(rng.uniform(math.log(0.05), math.log(0.3))))))
    return out


@dataclass
class Stream:
    arrivals: np.ndarray   # seconds from the start
    prior: np.ndarray      # index into the pool
    op: np.ndarray         # 0 forward, 1 adjoint, 2 metric
    seeds: np.ndarray


def draw_stream(n_requests: int, n_priors: int, rate: float, seed: int) -> Stream:
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests) if rate > 0 else np.zeros(n_requests)
    return Stream(np.cumsum(gaps), rng.integers(0, n_priors, n_requests), rng.integers(0, 3, n_requests),
                  rng.integers(0, 2 ** 31, n_requests))


@dataclass
class Slots:
    """Per-prior ring of request buffers (inputs drawn once, outputs per slot)."""
    xi: list = field(default_factory=list)
    ybar: list = field(default_factory=list)
    w: list = field(default_factory=list)
    out_s: list = field(default_factory=list)
    out_x: list = field(default_factory=list)
    last: list = field(default_factory=list)


def build_pool(priors, precision="f32", slots=8, seed=11, plans=True):
    """Request buffers per prior (inputs drawn once, outputs per slot) and, with plans,
    each prior's plan built here; without, the plans list is empty and requests go to
    the server by configuration (the server builds and caches the plans)."""
    import torch
    dtype = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[precision]
    acc = torch.float64 if precision == "f64" else torch.float32
    built, pool = [], []
    for k, pr in enumerate(priors):
        if plans:
            built.append(B.icr_build_matrices(pr.config(precision)))
        n_xi, n_out = pr.sizes
        g = torch.Generator(device="cuda")
        g.manual_seed(seed + k)
        sl = Slots()
        for _ in range(slots):
            sl.xi.append(torch.randn(n_xi, device="cuda", generator=g).to(dtype))
            sl.ybar.append(torch.randn(n_out, device="cuda", generator=g).to(dtype))
            sl.w.append((torch.rand(n_out, device="cuda", generator=g) < 0.7).to(acc) * 100.0)
            sl.out_s.append(torch.empty(n_out, dtype=dtype, device="cuda"))
            sl.out_x.append(torch.empty(n_xi, dtype=dtype, device="cuda"))
            sl.last.append(None)
        pool.append(sl)
    torch.cuda.synchronize()
    return built, pool


def register_all(server: Server, plans) -> list:
    return [server.register(p) for p in plans]


def run_stream(server: Server, plan_ids, pool, stream: Stream, pace: bool = True, slot_timeout_s: float = 60.0):
    """Submit the stream at its arrival times; returns per-request latency (s), batch size
    and the wall time of the run. `plan_ids` are the pool's ids in this server, or the
    priors' configurations (IcrConfig) to submit by configuration. A request that can
    never fit the server's memory budget is refused at submission: its latency is NaN
    and its batch size 0."""
    ids_for = list(plan_ids)
    names = ("forward", "adjoint", "metric")
    n = len(stream.op)
    rids = np.zeros(n, dtype=np.int64)
    lag = np.zeros(n)
    for sl in pool:
        sl.last = [None] * len(sl.xi)
    counters = [0] * len(pool)
    t0 = time.perf_counter()
    for i in range(n):
        k = int(stream.prior[i])
        sl = pool[k]
        j = counters[k] % len(sl.xi)
        counters[k] += 1
        if sl.last[j] is not None:       # the slot's previous request must be finished
            deadline = time.perf_counter() + slot_timeout_s
            while not server.query(sl.last[j])[0]:
                if time.perf_counter() > deadline:
                    raise RuntimeError(f"request {sl.last[j]} did not finish within {slot_timeout_s} s")
                time.sleep(20e-6)
        if pace:
            target = t0 + stream.arrivals[i]
            while time.perf_counter() < target:
                pass
        op = names[int(stream.op[i])]
        submit = server.submit_prior if isinstance(ids_for[k], B.IcrConfig) else server.submit
        try:
            if op == "forward":
                rid = submit(ids_for[k], op, sl.xi[j], sl.out_s[j])
            elif op == "adjoint":
                rid = submit(ids_for[k], op, sl.ybar[j], sl.out_x[j])
            else:
                rid = submit(ids_for[k], op, sl.xi[j], sl.out_x[j], sl.w[j])
        except B.ICRError as e:
            if e.status != 4:           # only "does not fit the server's budget" is a refusal
                raise
            rid = -1
        lag[i] = max(0.0, time.perf_counter() - (t0 + stream.arrivals[i])) if pace else 0.0
        sl.last[j] = rid if rid >= 0 else sl.last[j]
        rids[i] = rid
    server.drain(slot_timeout_s)
    wall = time.perf_counter() - t0
    lat = np.zeros(n)
    bs = np.zeros(n, dtype=np.int64)
    for i, rid in enumerate(rids):
        if rid < 0:                     # refused at submission
            lat[i], bs[i] = np.nan, 0
            continue
        done, ts, _, td, b = server.query(int(rid))
        lat[i] = (td - ts) + lag[i]
        bs[i] = b
    return lat, bs, wall


def fine_pixels(priors, stream: Stream, served=None) -> int:
    """Fine pixels of the stream's requests (only those with served[i] True, if given)."""
    keep = np.ones(len(stream.prior), dtype=bool) if served is None else np.asarray(served)
    return int(sum(priors[int(k)].sizes[1] for k, ok in zip(stream.prior, keep) if ok))
