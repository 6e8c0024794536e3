"""Benchmark of the ICR hot path on one MI355X: forward + adjoint throughput.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision f32|bf16]

One step is icr_forward followed by icr_adjoint over one batch of the workload
(every level, level 0 included) with inputs resident in HBM, every kernel launched from
the host (--graph replays a captured HIP graph instead). Buffers rotate over
two sets (> 2 GB for the 3-D workload) so timed passes stream from HBM rather
than the 256 MB Infinity Cache. Prints one JSON line:

  value        fine pixels per second, batch * n_L^d / (time of one step)
  roofline     the dominant kernel (the last level's forward or adjoint) timed alone
               in the same launch configuration, HIP events around a run of launches on
               the stream they go to: algorithmic bytes per launch (the fine level's
               input read and output write, 2 batch n_L^d elements; the coarse level's
               read or write is implementation traffic, reported beside it) / average
               duration, against the 8 TB/s HBM peak
  cpu_baseline the FP64 oracle on the host, one sample of the same workload,
               forward + adjoint, one thread
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="icr3d_m52_10to388")
    ap.add_argument("--precision", default=None, help="f32 or bf16 (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes for the all-cores oracle baseline (0: skip it)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--levels", action="store_true", help="also time every level's kernels")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests in the served-mode stream (0: skip the served measurement)")
    ap.add_argument("--serve-priors", type=int, default=24)
    ap.add_argument("--serve-large-step", type=int, default=0,
                    help="grouped served form: fine pixels of a level from which a request runs its own kernels "
                         "(0: the library default)")
    ap.add_argument("--bf16-steps", type=int, default=20,
                    help="timed steps of the same workload in BF16 storage (0: skip; f32 workloads only)")
    ap.add_argument("--cf-reps", type=int, default=11,
                    help="repetitions per size of the correlated-field M_p benchmark (0: skip it)")
    ap.add_argument("--hypergrad-steps", type=int, default=20,
                    help="timed hyperparameter-gradient evaluations (0: skip that measurement)")
    ap.add_argument("--cg-iters", type=int, default=None,
                    help="CG iterations on the metric (default: 200 for a charted workload, else none)")
    ap.add_argument("--graph", action="store_true",
                    help="replay the step from a captured HIP graph (measured slower than launching "
                         "every kernel from the host on this stack, so off by default)")
    ap.add_argument("--legs", default="icr2d_se_16to1540_b16,icr2d_chart_24to1284,icr1d_m32_12to260",
                    help="other workloads measured compactly in the same line (empty: none)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device copy (calibrates rocprofv3 byte counters)")
    return ap.parse_args()


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """Digest of the sources of the sweep kernels, to tie counter files to a build."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_16683_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_tag: str, digest: str):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE, if recorded for the current kernel sources."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel_tag)
    if not rec or rec.get("source_digest") != digest:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(wl: dict, quiet: bool):
    """The FP64 oracle, one sample of the workload, forward + adjoint, one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import icr_oracle as O
    model = O.build(O.ICRConfig(ndim=wl["ndim"], shape0=wl["shape0"], depth=wl["depth"],
                                delta0=wl["delta0"], kernel=wl["kernel"], scale=wl["scale"],
                                length=wl["length"], chart=wl["chart"],
                                chart_params=wl.get("chart_params", (0.1, 2.302585092994046, 1.5707963267948966))))
    xi = W.standard_normal(model.n_xi, seed=0)
    y = W.standard_normal(model.out_size, seed=1)
    log(f"cpu baseline: oracle forward+adjoint on {model.shapes[-1]} ...", quiet)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        model.forward(xi)
        model.adjoint(y)
        dt = time.perf_counter() - t0
    return {"value": model.out_size / dt, "unit": "fine px/s", "cores": 1, "kind": "oracle",
            "sample": f"one sample of the full workload ({'x'.join(map(str, model.shapes[-1]))} final "
                      f"pixels), forward + adjoint, numpy FP64, 1 thread, {dt:.1f} s"}


def host_info() -> dict:
    """CPU model, logical CPUs and memory of the host (Linux /proc)."""
    info = {"logical_cpus": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_gb"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def _oracle_sample(args):
    """One oracle forward + adjoint in a worker process, one thread; returns seconds."""
    key, seed = args
    from threadpoolctl import threadpool_limits

    from oracle import icr_oracle as O
    wl = W.WORKLOADS[key]
    model = O.build(O.ICRConfig(ndim=wl["ndim"], shape0=wl["shape0"], depth=wl["depth"],
                                delta0=wl["delta0"], kernel=wl["kernel"], scale=wl["scale"],
                                length=wl["length"], chart=wl["chart"],
                                chart_params=wl.get("chart_params", (0.1, 2.302585092994046, 1.5707963267948966))))
    xi = W.standard_normal(model.n_xi, seed=seed)
    y = W.standard_normal(model.out_size, seed=seed + 1)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        model.forward(xi)
        model.adjoint(y)
        return time.perf_counter() - t0, model.out_size


def cpu_baseline_parallel(key: str, workers: int, quiet: bool) -> dict:
    """The oracle on `workers` host cores at once: one independent sample per process."""
    import multiprocessing as mp
    log(f"cpu baseline: {workers} oracle samples in parallel ...", quiet)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_sample, [(key, 100 + 2 * i) for i in range(workers)])
    wall = time.perf_counter() - t0
    px = sum(n for _, n in res)
    return {"value": px / wall, "unit": "fine px/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} independent samples of the full workload, one per process and core, "
                      f"numpy FP64, {wall:.1f} s wall (process start included)"}


def served(n_requests: int, n_priors: int, quiet: bool, large_step: int = 0) -> dict:
    """Mixed 1-D/2-D/3-D forward/adjoint/metric requests over a pool of priors with random
    length scales, submitted by prior configuration: every server starts with an empty
    plan cache and builds each prior's plan when its first request arrives (inside that
    request's latency). First the one-launch-per-request capacity (warm cache, back to
    back), then Poisson streams at 0.5, 0.8 and 1.2x that rate through the grouped served
    form (requests of any prior and op share launches, 8 GB arena), the homogeneous
    batched form (same prior and op only, hipGraphs) and the plain form; at 0.8x also the
    grouped form under a 256 MB arena; the forms back to back for their saturated rates."""
    import torch

    from paper_2402_16683_amd import serve as S
    budget = 8 << 30
    priors = S.draw_priors(n_priors, seed=5)
    configs = [pr.config() for pr in priors]
    _, pool = S.build_pool(priors, slots=8, plans=False)
    kinds = {"served": dict(max_batch=16, n_streams=8, use_graphs=False, grouped=True, group_streams=2,
                            large_step=large_step),
             "served_homogeneous": dict(max_batch=16, n_streams=8, use_graphs=True),
             "plain": dict(max_batch=1, n_streams=1, use_graphs=False)}

    def fresh(name, hbm=budget):
        return S.Server(hbm, **kinds[name])

    base = S.draw_stream(n_requests, n_priors, rate=0.0, seed=6)
    plain = fresh("plain")
    t0 = time.perf_counter()
    S.run_stream(plain, configs, pool, S.draw_stream(min(200, n_requests), n_priors, 0.0, seed=7), pace=False)
    _, _, wall = S.run_stream(plain, configs, pool, S.draw_stream(4 * n_priors, n_priors, 0.0, seed=9), pace=False)
    build_s = time.perf_counter() - t0
    _, _, wall = S.run_stream(plain, configs, pool, base, pace=False)
    capacity = n_requests / wall
    st = plain.stats()
    plain.close()
    out = {"requests": n_requests, "priors": n_priors, "plain_capacity_req_per_s": capacity,
           "hbm_budget_bytes": budget, "warmup_s_with_builds": build_s, "plans_built_per_server": st["plans_built"],
           "priors_by_dim": {str(d): sum(pr.ndim == d for pr in priors) for d in (1, 2, 3)}}

    def one(name, stream, rate, hbm=budget):
        srv = fresh(name, hbm)
        lat, bs, wall = S.run_stream(srv, configs, pool, stream)
        st = srv.stats()
        srv.close()
        ok = ~np.isnan(lat)
        r = {"p50_ms": float(np.percentile(lat[ok], 50) * 1e3), "p99_ms": float(np.percentile(lat[ok], 99) * 1e3),
             "fine_px_per_s": S.fine_pixels(priors, stream, ok) / wall, "requests_per_s": int(ok.sum()) / wall,
             "mean_batch": float(bs[ok].mean()), "launch_sequences": st["batches"] + st["groups"],
             "grouped_requests": st["grouped_requests"], "plans_built": st["plans_built"],
             "admissions_deferred": st["admissions_deferred"], "refused": int((~ok).sum())}
        dims = np.array([priors[k].ndim for k in stream.prior])
        r["p50_ms_by_dim"] = {str(d): float(np.percentile(lat[ok & (dims == d)], 50) * 1e3)
                              for d in (1, 2, 3) if np.any(ok & (dims == d))}
        log(f"served: {name} at {rate:.0f} req/s: p50 {r['p50_ms']:.3f} ms p99 {r['p99_ms']:.3f} ms "
            f"{r['fine_px_per_s']:.3g} px/s, mean batch {r['mean_batch']:.2f}, grouped {r['grouped_requests']}", quiet)
        return r

    out["rates"] = []
    for factor in (0.5, 0.8, 1.2):
        rate = factor * capacity
        stream = S.draw_stream(n_requests, n_priors, rate=rate, seed=6)
        row = {"factor": factor, "arrival_rate_req_per_s": rate}
        for name in ("served", "served_homogeneous", "plain"):
            row[name] = one(name, stream, rate)
        if factor == 0.8:
            row["served_256MB"] = one("served", stream, rate, hbm=256 << 20)
            out.update({"arrival_rate_req_per_s": rate, "served": row["served"], "plain": row["plain"],
                        "served_homogeneous": row["served_homogeneous"], "served_256MB": row["served_256MB"]})
        out["rates"].append(row)
    # saturation: the stream back to back (cold caches: builds included)
    for name in ("served", "served_homogeneous"):
        srv = fresh(name)
        _, bs, wall = S.run_stream(srv, configs, pool, base, pace=False)
        out[f"{name}_saturated_req_per_s"] = n_requests / wall
        out[f"{name}_saturated_mean_batch"] = float(bs.mean())
        srv.close()
    del pool
    torch.cuda.empty_cache()
    return out


def cg_solve(B, plan, wl: dict, iters: int, quiet: bool, solves: int = 5) -> dict:
    """MGVI-style metric solve on the workload: d = mask * L xi* + 0.1 noise with a
    Bernoulli(0.7) mask, w = mask / 0.1^2, b = L^T (w * d); `iters` CG steps of
    (L^T W L + 1) x = b on the device (each step one metric product), timed over
    several solves."""
    import torch
    info = plan.info
    n_xi, n_out = info["n_xi"], info["n_out"]
    xi_true = torch.from_numpy(W.standard_normal_f32(n_xi, seed=2)).cuda().to(plan.dtype)
    noise = torch.from_numpy(W.standard_normal_f32(n_out, seed=3)).cuda().to(plan.acc_dtype)
    mask = torch.from_numpy(W.bernoulli_mask(n_out, 0.7, seed=4)).cuda().to(plan.acc_dtype)
    w = mask / 0.01
    s = B.icr_forward(plan, xi_true[None])[0].to(plan.acc_dtype)
    d = mask * s + 0.1 * noise
    b = B.icr_adjoint(plan, (w * d).to(plan.dtype)[None])[0]
    ws = torch.empty(B.icr_cg_workspace_bytes(plan, 1), dtype=torch.uint8, device="cuda")
    x = torch.empty_like(b)
    x, norms = B.icr_cg_metric(plan, w, b, iters, x=x, residual_norms=True, workspace=ws)
    torch.cuda.synchronize()
    n_solves = solves
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_solves)]
    for e0, e1 in evs:
        e0.record()
        B.icr_cg_metric(plan, w, b, iters, x=x, workspace=ws)
        e1.record()
    torch.cuda.synchronize()
    ms = statistics.median(e0.elapsed_time(e1) for e0, e1 in evs)
    nr = norms[0].double().cpu().numpy()
    out = {"iterations": iters, "ms_per_solve": ms, "us_per_metric_product": ms * 1e3 / iters,
           "metric_products_per_s": iters / (ms * 1e-3),
           "fine_px_per_s": 2 * iters * n_out / (ms * 1e-3),
           "residual_reduction": float(nr[-1] / nr[0]),
           "data": "truth xi* seed 2, noise sigma 0.1 seed 3, 70% observed (Bernoulli seed 4)"}
    log(f"cg: {iters} iterations in {ms:.2f} ms ({out['us_per_metric_product']:.1f} us per metric product), "
        f"|r|/|r0| = {out['residual_reduction']:.2e}", quiet)
    return out


def time_runs(fn, n: int) -> float:
    """Mean ms per call of fn(k), k = 0 .. n-1, from one pair of HIP events around the
    whole run on the current stream (the calls launch there)."""
    import torch
    for k in range(3):
        fn(k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(n):
        fn(k)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def workload_leg(B, key: str, steps: int, quiet: bool, prec=None, cg_iters: int = 0) -> dict:
    """A compact measurement of another workload: the step (icr_forward + icr_adjoint over
    its batch, two rotating buffer sets), the last level's forward and adjoint launches
    with their algorithmic bandwidth, and for charted workloads CG and one MGVI iteration."""
    import torch
    wl = dict(W.WORKLOADS[key])
    prec = prec or wl["precision"]
    cfg = B.make_config(wl["ndim"], wl["shape0"], wl["depth"], wl["delta0"], kernel=wl["kernel"],
                        scale=wl["scale"], length=wl["length"], chart=wl["chart"],
                        chart_params=wl.get("chart_params", (0.1, 2.302585092994046, 1.5707963267948966)),
                        precision=prec)
    t0 = time.perf_counter()
    plan = B.icr_build_matrices(cfg)
    build_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info
    batch, L, el = wl["batch"], info["depth"], info["elem_bytes"]
    n_xi, n_out, offs = info["n_xi"], info["n_out"], info["level_offsets"]
    xi_h = torch.from_numpy(W.standard_normal_f32(n_xi, seed=0, batch=batch))
    y_h = torch.from_numpy(W.standard_normal_f32(n_out, seed=1, batch=batch))
    sets = [dict(xi=xi_h.to("cuda").to(plan.dtype), y=y_h.to("cuda").to(plan.dtype),
                 s=torch.empty((batch, n_out), dtype=plan.dtype, device="cuda"),
                 xib=torch.empty((batch, n_xi), dtype=plan.dtype, device="cuda"),
                 wsf=B.workspace_for(plan, batch), wsa=B.workspace_for(plan, batch)) for _ in range(2)]

    def step(k):
        b = sets[k % 2]
        B.icr_forward(plan, b["xi"], b["s"], b["wsf"])
        B.icr_adjoint(plan, b["y"], b["xib"], b["wsa"])

    def fwd_last(k):
        b = sets[k % 2]
        B.icr_forward_level(plan, L - 1, b["wsf"][:, offs[L - 1]:offs[L]], b["xi"][:, offs[L]:], b["s"])

    def adj_last(k):
        b = sets[k % 2]
        B.icr_adjoint_level(plan, L - 1, b["y"], b["xib"][:, offs[L]:], b["wsa"][:, offs[L - 1]:offs[L]])

    ms = time_runs(step, steps)
    out = {"workload": key, "precision": prec, "batch": batch, "final_shape": list(info["level_shapes"][-1]),
           "build_ms": build_ms, "ms_per_step": ms, "us_per_step": ms * 1e3,
           "fine_px_per_s": batch * n_out / (ms * 1e-3),
           "step_hbm_frac": 2 * batch * (n_xi + n_out) * el / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}
    if L > 0 and batch * n_out >= 1 << 20:
        alg = 2 * batch * n_out * el
        out["fwd_last_ms"] = time_runs(fwd_last, steps)
        out["adj_last_ms"] = time_runs(adj_last, steps)
        out["fwd_last_frac"] = alg / (out["fwd_last_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
        out["adj_last_frac"] = alg / (out["adj_last_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
    log(f"{key} {prec}: {ms * 1e3:.1f} us per step (batch {batch})", quiet)
    if cg_iters > 0:
        out["cg"] = cg_solve(B, plan, wl, cg_iters, quiet)
        out["mgvi"] = mgvi_bench(B, plan, wl, 3, quiet)
        if prec == "f32":
            # the same CG on an FP64 plan, for the residual reduction FP32 reaches against it
            cfg64 = B.make_config(wl["ndim"], wl["shape0"], wl["depth"], wl["delta0"], kernel=wl["kernel"],
                                  scale=wl["scale"], length=wl["length"], chart=wl["chart"],
                                  chart_params=wl.get("chart_params", (0.1, 2.302585092994046, 1.5707963267948966)),
                                  precision="f64")
            plan64 = B.icr_build_matrices(cfg64)
            out["cg_f64"] = cg_solve(B, plan64, wl, cg_iters, quiet, solves=1)
            B.icr_plan_destroy(plan64)
    del sets
    B.icr_plan_destroy(plan)
    return out


def bf16_leg(B, wl: dict, steps: int, quiet: bool) -> dict:
    """The same step in BF16 storage (FP32 arithmetic): time per step and the last level's
    forward and adjoint launches (HIP events), with their algorithmic bandwidth."""
    import torch
    cfg = B.make_config(wl["ndim"], wl["shape0"], wl["depth"], wl["delta0"], kernel=wl["kernel"],
                        scale=wl["scale"], length=wl["length"], chart=wl["chart"],
                        chart_params=wl.get("chart_params", (0.1, 2.302585092994046, 1.5707963267948966)),
                        precision="bf16")
    plan = B.icr_build_matrices(cfg)
    info = plan.info
    batch, L = wl["batch"], info["depth"]
    n_xi, n_out, offs = info["n_xi"], info["n_out"], info["level_offsets"]
    xi_h = torch.from_numpy(W.standard_normal_f32(n_xi, seed=0, batch=batch))
    y_h = torch.from_numpy(W.standard_normal_f32(n_out, seed=1, batch=batch))
    sets = [dict(xi=xi_h.to("cuda").to(plan.dtype), y=y_h.to("cuda").to(plan.dtype),
                 s=torch.empty((batch, n_out), dtype=plan.dtype, device="cuda"),
                 xib=torch.empty((batch, n_xi), dtype=plan.dtype, device="cuda"),
                 wsf=B.workspace_for(plan, batch), wsa=B.workspace_for(plan, batch)) for _ in range(2)]

    def step(k):
        b = sets[k % 2]
        B.icr_forward(plan, b["xi"], b["s"], b["wsf"])
        B.icr_adjoint(plan, b["y"], b["xib"], b["wsa"])

    def fwd_last(k):
        b = sets[k % 2]
        B.icr_forward_level(plan, L - 1, b["wsf"][:, offs[L - 1]:offs[L]], b["xi"][:, offs[L]:], b["s"])

    def adj_last(k):
        b = sets[k % 2]
        B.icr_adjoint_level(plan, L - 1, b["y"], b["xib"][:, offs[L]:], b["wsa"][:, offs[L - 1]:offs[L]])

    out = {}
    for name, fn, n in (("ms_per_step", step, steps), ("fwd_last_ms", fwd_last, steps), ("adj_last_ms", adj_last, steps)):
        for k in range(3):
            fn(k)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for k in range(n):
            evs[k][0].record()
            fn(k)
            evs[k][1].record()
        torch.cuda.synchronize()
        out[name] = statistics.mean(a.elapsed_time(b) for a, b in evs)
    step_bytes = 2 * batch * (n_xi + n_out) * 2
    # as for the FP32 roofline: a launch's fine level read and written; the coarse level
    # it reads (forward) or writes (adjoint) is reported apart
    launch_bytes = batch * 2 * n_out * 2
    out["alg_bytes_per_launch"] = launch_bytes
    out["coarse_level_bytes_per_launch"] = batch * (offs[L] - offs[L - 1]) * 2
    out["fine_px_per_s"] = batch * n_out / (out["ms_per_step"] * 1e-3)
    out["step_hbm_frac"] = step_bytes / (out["ms_per_step"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
    out["adj_last_frac"] = launch_bytes / (out["adj_last_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
    out["fwd_last_frac"] = launch_bytes / (out["fwd_last_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
    log(f"bf16: {out['ms_per_step']:.3f} ms per step (event-timed), last level forward "
        f"{out['fwd_last_ms'] * 1e3:.1f} us, adjoint {out['adj_last_ms'] * 1e3:.1f} us", quiet)
    return out


def mgvi_bench(B, plan, wl: dict, pairs: int, quiet: bool) -> dict:
    """One MGVI iteration on the workload as the paper configures it: `pairs`
    antithetic sample pairs, each delta by 100 CG steps on the metric, then one
    Newton-CG step of the expansion point with 35 CG steps (mask Bernoulli(0.7),
    noise sigma 0.1, data from a truth drawn with seed 2)."""
    import torch
    info = plan.info
    n_xi, n_out = info["n_xi"], info["n_out"]
    mask = torch.from_numpy(W.bernoulli_mask(n_out, 0.7, seed=4)).cuda().to(plan.acc_dtype)
    w = mask / 0.01
    xi_true = torch.from_numpy(W.standard_normal_f32(n_xi, seed=2)).cuda().to(plan.dtype)
    noise = torch.from_numpy(W.standard_normal_f32(n_out, seed=3)).cuda().to(plan.dtype)
    s = B.icr_forward(plan, xi_true[None])[0]
    d = (mask.to(plan.dtype) * s + 0.1 * noise).contiguous()
    # the standard-normal draws are inputs: drawn and uploaded before the timed region
    eta = torch.from_numpy(W.standard_normal_f32(n_xi, seed=7, batch=pairs)).cuda().to(plan.dtype)
    eta_d = torch.from_numpy(W.standard_normal_f32(n_out, seed=8, batch=pairs)).cuda().to(plan.dtype)
    b = B.icr_weighted_adjoint(plan, w, d[None], half=False)
    mean = torch.zeros((1, n_xi), dtype=plan.dtype, device="cuda")
    wss = (B.workspace_for(plan, pairs, metric=True),
           torch.empty(B.icr_cg_workspace_bytes(plan, pairs), dtype=torch.uint8, device="cuda"),
           torch.empty(B.icr_mgvi_workspace_bytes(plan, 1), dtype=torch.uint8, device="cuda"))
    B.mgvi_step(plan, w, b, mean, eta, eta_d, 100, 35, workspaces=wss)
    torch.cuda.synchronize()
    mean0 = mean.clone()

    def iteration_ms(absdelta=None, done=None):
        # median of three timed pairs of iterations (one timing has been seen far off)
        times = []
        for _ in range(3):
            mean.copy_(mean0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(2):
                B.mgvi_step(plan, w, b, mean, eta, eta_d, 100, 35, workspaces=wss, absdelta=absdelta,
                            iterations_done=done)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 2)
        return statistics.median(times)

    ms = iteration_ms()
    products = pairs * 100 + 35 + 1   # metric products on single samples (the samples' CG runs batched)
    # the paper's example stops the samples' CG by the energy change: absdelta = 1e-4 size / 10,
    # at most 100 steps; also with a threshold 10x lower (on this metric the first steps
    # lower the energy by about as much as the example's threshold)
    rules = []
    for scale in (1.0, 0.1):
        absdelta = scale * 1e-4 * n_xi / 10.0
        done = torch.zeros(pairs, dtype=torch.int32, device="cuda")
        ms_sl = iteration_ms(absdelta, done)
        rules.append({"absdelta": absdelta, "max_iterations": 100, "ms_per_iteration": ms_sl,
                      "sample_cg_steps_taken": [int(v) for v in done.cpu()]})
    out = {"antithetic_pairs": pairs, "sample_cg_iterations": 100, "newton_cg_iterations": 35,
           "ms_per_iteration": ms, "sample_metric_products_per_iteration": products,
           "us_per_sample_metric_product": ms * 1e3 / products,
           "energy_rule": rules,
           "data": "draws eta seed 7, eta' seed 8 (uploaded before timing); truth seed 2, noise seed 3, mask seed 4"}
    log(f"mgvi: {ms:.1f} ms per iteration ({pairs} pairs x 100 CG steps + Newton 35 CG steps); energy rule "
        + ", ".join(f"absdelta {r['absdelta']:.3g}: {r['ms_per_iteration']:.1f} ms, steps {r['sample_cg_steps_taken']}"
                    for r in rules), quiet)
    return out


def correlated_field_bench(sizes, reps: int, quiet: bool) -> list:
    """The paper's benchmark operator on the correlated-field model: building M_p at a
    random position (the Poisson rate) and applying it to random input, per 2-D size
    (median of `reps` timed repetitions with HIP events). One call timed alone includes
    the host's submission latency; the device time per apply comes from a HIP graph of
    back-to-back applies, checked bitwise against a direct call."""
    import torch
    from paper_2402_16683_amd.cf import CorrelatedField
    rows = []
    for n in sizes:
        cf = CorrelatedField(n)
        p = torch.from_numpy(0.5 * W.standard_normal_f32(n * n, seed=71)).cuda().reshape(n, n)
        v = torch.from_numpy(W.standard_normal_f32(n * n, seed=72)).cuda().reshape(n, n)
        lam = torch.empty_like(p)
        out = torch.empty_like(p)
        cf.rate(p, lam)
        cf.metric_apply(lam, v, out)
        torch.cuda.synchronize()
        times = {"build": [], "apply": []}
        for _ in range(reps):
            for key, fn in (("build", lambda: cf.rate(p, lam)), ("apply", lambda: cf.metric_apply(lam, v, out))):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                times[key].append(e0.elapsed_time(e1))
        b_ms, a_ms = statistics.median(times["build"]), statistics.median(times["apply"])
        # device time per apply without the host's submission latency: a HIP graph of
        # `chain` back-to-back applies, replayed and timed with events
        chain = 20
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                for _ in range(chain):
                    cf.metric_apply(lam, v, out, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        graph.replay()
        torch.cuda.synchronize()
        dev = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            graph.replay()
            e1.record()
            torch.cuda.synchronize()
            dev.append(e0.elapsed_time(e1) / chain)
        d_ms = statistics.median(dev)
        check = torch.empty_like(out)
        cf.metric_apply(lam, v, check)
        torch.cuda.synchronize()
        if not torch.equal(check, out):
            raise RuntimeError(f"correlated field {n}^2: graph replay differs from the direct call")
        rows.append({"n": n, "pixels": n * n, "ms_build": b_ms, "ms_apply": a_ms, "ms_build_and_apply": b_ms + a_ms,
                     "us_apply_device": d_ms * 1e3})
        log(f"correlated field {n}^2: build M_p {b_ms * 1e3:.1f} us, apply {a_ms * 1e3:.1f} us (one call, "
            f"event-timed), {d_ms * 1e3:.1f} us per apply on the device ({chain} applies in a graph)", quiet)
    return rows


def hyper_grad_bench(B, wl: dict, prec: str, steps: int, quiet: bool) -> dict:
    """Hyperparameter gradients on the workload: a plan built with the length
    derivatives, then per step icr_forward + icr_adjoint + icr_hyper_grad (the full
    cost of dE/d(scale, length) for E = <ybar, L xi>), and the contraction alone."""
    import torch
    cfg = B.make_config(wl["ndim"], wl["shape0"], wl["depth"], wl["delta0"], kernel=wl["kernel"],
                        scale=wl["scale"], length=wl["length"], chart=wl["chart"],
                        chart_params=wl.get("chart_params", (0.1, 2.302585092994046, 1.5707963267948966)),
                        precision=prec, hypergrad=True)
    t0 = time.perf_counter()
    plan = B.icr_build_matrices(cfg)
    build_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info
    batch = wl["batch"]
    xi = torch.from_numpy(W.standard_normal_f32(info["n_xi"], seed=0, batch=batch)).cuda().to(plan.dtype)
    y = torch.from_numpy(W.standard_normal_f32(info["n_out"], seed=1, batch=batch)).cuda().to(plan.dtype)
    ws_f = B.workspace_for(plan, batch)
    ws_a = B.workspace_for(plan, batch)
    s = torch.empty((batch, info["n_out"]), dtype=plan.dtype, device="cuda")
    xb = torch.empty((batch, info["n_xi"]), dtype=plan.dtype, device="cuda")
    grad = torch.empty((batch, 2), dtype=torch.float64, device="cuda")
    hws = torch.empty((batch, info["hypergrad_workspace_elems"]), dtype=torch.float64, device="cuda")

    def full():
        B.icr_forward(plan, xi, s, ws_f)
        B.icr_adjoint(plan, y, xb, ws_a)
        B.icr_hyper_grad(plan, xi, s, ws_f, y, ws_a, grad, hws)

    def contraction():
        B.icr_hyper_grad(plan, xi, s, ws_f, y, ws_a, grad, hws)

    out = {"build_ms_with_derivatives": build_ms}
    for name, fn in (("ms_per_gradient", full), ("ms_contraction", contraction)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
    out["gradient"] = [float(v) for v in grad[0].cpu()]
    log(f"hyper_grad: {out['ms_per_gradient']:.3f} ms per gradient (forward + adjoint + contraction), "
        f"contraction {out['ms_contraction']:.3f} ms, build with derivatives {build_ms:.0f} ms", quiet)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    # the all-cores oracle baseline runs first, before this process touches the GPU: its
    # worker processes start from a process without any device state
    par = None
    if not args.no_cpu_baseline and args.cpu_workers > 0 and not args.copy_probe:
        par = cpu_baseline_parallel(args.workload, args.cpu_workers, args.quiet)
    import torch

    from paper_2402_16683_amd import icr as B

    torch.cuda.set_device(0)
    wl = dict(W.WORKLOADS[args.workload])
    prec = args.precision or wl["precision"]
    batch = wl["batch"]
    cfg = B.make_config(wl["ndim"], wl["shape0"], wl["depth"], wl["delta0"], kernel=wl["kernel"],
                        scale=wl["scale"], length=wl["length"], chart=wl["chart"],
                        chart_params=wl.get("chart_params", (0.1, 2.302585092994046, 1.5707963267948966)),
                        precision=prec)
    t0 = time.perf_counter()
    plan = B.icr_build_matrices(cfg)
    build_s = time.perf_counter() - t0
    info = plan.info
    L = info["depth"]
    el = info["elem_bytes"]
    n_xi, n_out = info["n_xi"], info["n_out"]
    offs = info["level_offsets"]
    n_prev = offs[L] - offs[L - 1]
    log(f"workload {args.workload} {prec}: levels {info['level_shapes']}, batch {batch}, "
        f"build {build_s * 1e3:.1f} ms", args.quiet)

    # two rotating sets of every buffer, inputs drawn once on the host
    sets = []
    xi_host = torch.from_numpy(W.standard_normal_f32(n_xi, seed=0, batch=batch))
    y_host = torch.from_numpy(W.standard_normal_f32(n_out, seed=1, batch=batch))
    for _ in range(2):
        sets.append(dict(
            xi=xi_host.to("cuda").to(plan.dtype), y=y_host.to("cuda").to(plan.dtype),
            s=torch.empty((batch, n_out), dtype=plan.dtype, device="cuda"),
            xib=torch.empty((batch, n_xi), dtype=plan.dtype, device="cuda"),
            wsf=torch.empty((batch, info["workspace_elems"]), dtype=plan.dtype, device="cuda"),
            wsa=torch.empty((batch, info["workspace_elems"]), dtype=plan.dtype, device="cuda")))
    torch.cuda.synchronize()

    def step(k):
        b = sets[k % 2]
        B.icr_forward(plan, b["xi"], b["s"], b["wsf"])
        B.icr_adjoint(plan, b["y"], b["xib"], b["wsa"])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    run = step
    if args.graph:
        # the step's launch sequence captured once per buffer set and replayed: no host
        # work per launch (the sweep calls allocate nothing and use the current stream)
        graphs = []
        for k in range(2):
            gph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gph):
                step(k)
            graphs.append(gph)
        torch.cuda.synchronize()
        run = lambda k: graphs[k % 2].replay()
        for k in range(2):
            run(k)
        torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        run(k)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms_per_step = wall * 1e3 / args.steps
    q = np.quantile(per, [0.16, 0.5, 0.84])

    # dominant kernels: the last level's forward and adjoint, timed launch by launch
    def time_launches(fn, n):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for k in range(n):
            evs[k][0].record()
            fn(k)
            evs[k][1].record()
        torch.cuda.synchronize()
        return statistics.mean(a.elapsed_time(b) for a, b in evs)

    def fwd_last(k):
        b = sets[k % 2]
        B.icr_forward_level(plan, L - 1, b["wsf"][:, offs[L - 1]:offs[L]], b["xi"][:, offs[L]:], b["s"])

    def adj_last(k):
        b = sets[k % 2]
        B.icr_adjoint_level(plan, L - 1, b["y"], b["xib"][:, offs[L]:], b["wsa"][:, offs[L - 1]:offs[L]])

    n_launch = max(args.steps, 10)
    fwd_ms = time_runs(fwd_last, n_launch)
    adj_ms = time_runs(adj_last, n_launch)
    # algorithmic bytes of one last-level launch: its fine input (xi_L, or the cotangent
    # y_L) read once and its fine output (s_L, or xi_bar_L) written once; the coarse
    # level's read (forward) or write (adjoint) is implementation traffic
    launch_bytes = batch * 2 * n_out * el
    coarse_bytes = batch * n_prev * el
    dom, dom_ms = ("refine_adj_last", adj_ms) if adj_ms >= fwd_ms else ("refine_fwd_last", fwd_ms)
    achieved = launch_bytes / (dom_ms * 1e-3) / 1e9
    digest = kernel_source_digest()
    tag = f"{dom}:{args.workload}:{prec}"

    levels = None
    if args.levels:
        levels = []
        for l in range(-1, L):
            lo, hi = offs[l + 1], offs[l + 2]
            if l < 0:
                f = lambda k: B.icr_forward_level(plan, -1, None, sets[k % 2]["xi"][:, :hi],
                                                  sets[k % 2]["wsf"][:, :hi])
                g = lambda k: B.icr_adjoint_level(plan, -1, sets[k % 2]["wsa"][:, :hi],
                                                  sets[k % 2]["xib"][:, :hi], None)
            else:
                def f(k, l=l, lo=lo, hi=hi):
                    b = sets[k % 2]
                    out = b["s"] if l == L - 1 else b["wsf"][:, lo:hi]
                    B.icr_forward_level(plan, l, b["wsf"][:, offs[l]:lo], b["xi"][:, lo:hi], out)

                def g(k, l=l, lo=lo, hi=hi):
                    b = sets[k % 2]
                    yin = b["y"] if l == L - 1 else b["wsa"][:, lo:hi]
                    B.icr_adjoint_level(plan, l, yin, b["xib"][:, lo:hi], b["wsa"][:, offs[l]:lo])
            levels.append({"level": l, "fwd_ms": time_launches(f, 20), "adj_ms": time_launches(g, 20),
                           "fine_elems": batch * (hi - lo)})
    copy_gbs = None
    if not args.copy_probe:
        # on-box streaming reference: a 1 GiB device-to-device copy (read + write)
        csrc = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        cdst = torch.empty_like(csrc)
        for _ in range(2):
            cdst.copy_(csrc)
        copy_ms = time_launches(lambda k: cdst.copy_(csrc), 10)
        copy_gbs = 2 * csrc.numel() * 4 / (copy_ms * 1e-3) / 1e9
        del csrc, cdst
    else:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    step_bytes = 2 * batch * (n_xi + n_out) * el
    value = batch * n_out / (ms_per_step * 1e-3)
    out = {
        "metric": "ICR fine-pixels/s fwd+adj",
        "value": value,
        "unit": "fine px/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16-storage/f32"}.get(prec, prec),
        "data": "synthetic: seeded N(0,1) excitations and cotangents",
        "config": {"workload": args.workload, "ndim": wl["ndim"], "shape0": list(wl["shape0"]),
                   "depth": L, "final_shape": list(info["level_shapes"][-1]), "kernel": wl["kernel"],
                   "length": wl["length"], "batch": batch, "precision": prec,
                   "launch": "hipgraph" if args.graph else "eager"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(tag, digest),
                     "kernel": dom, "launch_ms": dom_ms, "alg_bytes_per_launch": launch_bytes,
                     "coarse_level_bytes_per_launch": coarse_bytes,
                     "fwd_last_ms": fwd_ms, "adj_last_ms": adj_ms,
                     "fwd_last_frac": launch_bytes / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "copy_reference_gbs": copy_gbs},
        "step": {"alg_bytes": step_bytes,
                 "hbm_frac": step_bytes / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9),
                 "ms_p16_p50_p84": [float(v) for v in q], "build_ms": build_s * 1e3},
        "source_digest": digest,
    }
    if levels is not None:
        out["levels"] = levels
    cg_iters = args.cg_iters if args.cg_iters is not None else (200 if wl["chart"] != "regular" else 0)
    if cg_iters > 0 and not args.copy_probe and prec != "bf16":
        out["cg"] = cg_solve(B, plan, wl, cg_iters, args.quiet)
        out["mgvi"] = mgvi_bench(B, plan, wl, 3, args.quiet)
    if args.bf16_steps > 0 and prec == "f32" and not args.copy_probe:
        out["bf16_storage"] = bf16_leg(B, wl, args.bf16_steps, args.quiet)
    if args.cf_reps > 0 and not args.copy_probe:
        out["correlated_field_metric"] = correlated_field_bench([64, 128, 256, 512, 1024, 2048, 4096], args.cf_reps,
                                                                args.quiet)
    if args.hypergrad_steps > 0 and not args.copy_probe:
        try:
            out["hyper_grad"] = hyper_grad_bench(B, wl, prec, args.hypergrad_steps, args.quiet)
        except B.ICRError as e:  # e.g. a workload whose factors clamp pivots has no length derivative
            out["hyper_grad"] = {"skipped": str(e)}
    if args.legs and not args.copy_probe:
        out["workloads"] = {}
        for key in [k for k in args.legs.split(",") if k and k != args.workload]:
            charted = W.WORKLOADS[key]["chart"] != "regular"
            out["workloads"][key] = workload_leg(B, key, 20, args.quiet, cg_iters=200 if charted else 0)
    if args.serve_requests > 0 and not args.copy_probe:
        out["served"] = served(args.serve_requests, args.serve_priors, args.quiet, args.serve_large_step)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.quiet)
        out["cpu_baseline"]["host"] = host_info()
        if par is not None:
            out["cpu_baseline_all_cores"] = par
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
