"""Served mode: continuous batching must not change any result.

Each request's output from the server (batched with others, replayed hipGraphs, several
streams in flight, admission under a memory budget) is compared with the same request
computed alone by a direct batch-1 call. Every sample is computed by the same kernels in
the same order whatever the batch, so the comparison is bitwise. Graph replays are
checked over two rounds with eager work and synchronisation in between.
"""

import math

import numpy as np
import pytest

import workloads as W
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

POOL = [
    C.case(1, (20,), 5, (0.05,), "matern32", 0.2, name="s1"),
    C.case(2, (12, 12), 4, (0.03, 0.03), "matern52", 0.15, name="s2"),
    C.case(3, (8, 8, 8), 3, (0.06, 0.06, 0.06), "matern52", 0.2, name="s3"),
    C.case(3, (7, 9, 8), 2, (0.05, 0.06, 0.07), "matern32", 0.3, name="s4"),
    C.case(2, (9, 10), 3, (0.04, 0.05), "matern32", 0.1, precision="bf16", name="s5"),
    # charted priors (one matrix set per radial shell) served like the stationary ones
    C.case(2, (10, 12), 3, (0.1, 1 / 12), "matern32", 0.1, chart="logradial2d", name="s6"),
    C.case(3, (6, 6, 6), 2, (1 / 6,) * 3, "matern32", 0.2, chart="logradial_cyl3d",
           chart_params=(0.1, math.log(10.0), math.pi / 2, 1.0), name="s7"),
]


def _plans():
    return [C.gpu_plan(c) for c in POOL]


def _requests(plans, n, seed):
    import torch
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        k = int(rng.integers(0, len(plans)))
        op = ("forward", "adjoint", "metric")[int(rng.integers(0, 3))]
        p = plans[k]
        g = torch.Generator(device="cuda")
        g.manual_seed(seed * 100003 + i)
        n_in = p.info["n_out"] if op == "adjoint" else p.info["n_xi"]
        n_out = p.info["n_out"] if op == "forward" else p.info["n_xi"]
        inp = torch.randn(n_in, device="cuda", generator=g).to(p.dtype)
        w = (torch.rand(p.info["n_out"], device="cuda", generator=g) < 0.7).to(p.acc_dtype) * 100.0
        reqs.append(dict(k=k, op=op, inp=inp, w=w, out=torch.full((n_out,), float("nan"), dtype=p.dtype,
                                                                  device="cuda")))
    return reqs


def _alone(plan, r):
    from paper_2402_16683_amd import icr as B
    if r["op"] == "forward":
        return B.icr_forward(plan, r["inp"][None])[0]
    if r["op"] == "adjoint":
        return B.icr_adjoint(plan, r["inp"][None])[0]
    return B.icr_metric_apply(plan, r["w"], r["inp"][None])[0]


def _serve(server, plans, reqs):
    ids = [server.register(p) for p in plans]
    rids = []
    for r in reqs:
        rids.append(server.submit(ids[r["k"]], r["op"], r["inp"], r["out"], r["w"] if r["op"] == "metric" else None))
    server.drain(120.0)
    return [server.query(rid) for rid in rids]


@pytest.mark.parametrize("graphs", [True, False])
def test_results_in_the_mix_equal_results_alone(graphs):
    import torch
    from paper_2402_16683_amd.serve import Server
    plans = _plans()
    server = Server(hbm_budget_bytes=1 << 30, max_batch=8, n_streams=4, use_graphs=graphs)
    for rnd in range(2):
        reqs = _requests(plans, 150, seed=rnd + 1)
        info = _serve(server, plans, reqs)
        assert all(q[0] for q in info)
        torch.cuda.synchronize()
        for r in reqs:
            alone = _alone(plans[r["k"]], r)
            torch.cuda.synchronize()
            assert torch.equal(r["out"], alone), (r["k"], r["op"])
    st = server.stats()
    assert st["completed"] == 300 and st["pending"] == 0
    assert st["batches"] < 300                     # requests were batched
    if graphs:
        assert 0 < st["graph_captures"] <= st["batches"]
    server.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_served_results_match_the_oracle(graphs):
    """Every served request (batched, several streams, graphs or not) against the FP64
    oracle of its prior on the values the device holds, at the precision's tolerance."""
    import torch
    from paper_2402_16683_amd.serve import Server
    plans = _plans()
    models = [C.oracle_model(c) for c in POOL]
    server = Server(hbm_budget_bytes=1 << 30, max_batch=8, n_streams=4, use_graphs=graphs)
    reqs = _requests(plans, 120, seed=11)
    info = _serve(server, plans, reqs)
    assert all(q[0] for q in info)
    torch.cuda.synchronize()
    seen = set()
    for r in reqs:
        c, m = POOL[r["k"]], models[r["k"]]
        inp = C.to_numpy(r["inp"])
        if r["op"] == "forward":
            ref = m.forward(inp)
        elif r["op"] == "adjoint":
            ref = m.adjoint(inp)
        else:
            ref = m.metric(C.to_numpy(r["w"]), inp)
        got = C.to_numpy(r["out"])
        assert np.all(np.isfinite(got)), (r["k"], r["op"])
        rms, mx = C.rel_errors(got, ref)
        tol_rms, tol_max = C.TOL[c["precision"]]
        assert rms <= tol_rms and mx <= tol_max, (c["name"], r["op"], rms, mx)
        seen.add((r["k"], r["op"]))
    assert len(seen) == 3 * len(POOL)          # every prior with every op
    server.close()


def test_admission_under_a_tight_budget():
    import torch
    from paper_2402_16683_amd.serve import Server
    from paper_2402_16683_amd import icr as B
    plans = _plans()
    biggest = max(p.info["n_xi"] * 4 * 4 for p in plans)   # about two metric requests of the largest prior
    server = Server(hbm_budget_bytes=2 * biggest, max_batch=8, n_streams=4, use_graphs=False)
    reqs = _requests(plans, 80, seed=7)
    info = _serve(server, plans, reqs)
    assert all(q[0] for q in info)
    st = server.stats()
    assert st["admissions_deferred"] > 0 and st["arena_in_use"] == 0
    for r in reqs:
        assert torch.equal(r["out"], _alone(plans[r["k"]], r))
    # a request that can never fit is refused at submission
    tiny = Server(hbm_budget_bytes=4096, max_batch=4, n_streams=1, use_graphs=False)
    pid = tiny.register(plans[2])
    with pytest.raises(B.ICRError) as e:
        tiny.submit(pid, "forward", reqs[0]["inp"], reqs[0]["out"])
    assert e.value.status == 4
    tiny.close()
    server.close()


def test_plain_mode_runs_one_request_per_launch():
    import torch
    from paper_2402_16683_amd.serve import Server
    plans = _plans()
    server = Server(hbm_budget_bytes=1 << 28, max_batch=1, n_streams=1, use_graphs=False)
    reqs = _requests(plans, 40, seed=9)
    info = _serve(server, plans, reqs)
    assert all(q[0] and q[4] == 1 for q in info)
    assert server.stats()["batches"] == 40
    for r in reqs:
        assert torch.equal(r["out"], _alone(plans[r["k"]], r))
    server.close()


def test_poisson_stream_driver_reports_latencies():
    from paper_2402_16683_amd import serve as S
    priors = S.draw_priors(6, seed=5)
    for pr in priors:                      # keep the test small: shallow copies of the mix
        pr.depth = min(pr.depth, 3 if pr.ndim == 3 else 4)
    plans, pool = S.build_pool(priors, slots=4)
    stream = S.draw_stream(200, len(priors), rate=20000.0, seed=3)
    server = S.Server(hbm_budget_bytes=1 << 30, max_batch=8, n_streams=4, use_graphs=True)
    lat, bs, wall = S.run_stream(server, S.register_all(server, plans), pool, stream)
    assert np.all(lat > 0) and np.all(bs >= 1) and wall > 0
    assert server.stats()["completed"] == 200
    server.close()


def _batch_bytes(info, op, k=1, acc=4):
    up = lambda v: (v + 255) // 256 * 256
    el = info["elem_bytes"]
    n_in = info["n_out"] if op == "adjoint" else info["n_xi"]
    n_out = info["n_out"] if op == "forward" else info["n_xi"]
    ws = info["n_xi"] if op == "metric" else max(info["n_xi"] - info["n_out"], 1)
    b = up(k * n_in * el) + up(k * n_out * el) + up(k * ws * el)
    return b + (up(k * info["n_out"] * acc) if op == "metric" else 0)


def test_idle_graphs_are_evicted_for_a_large_request():
    """A batch too large for a graph runs eagerly from the arena; when idle captured
    graphs hold the memory it needs, they are evicted (the request is not starved)."""
    import torch
    from paper_2402_16683_amd.serve import Server
    plans = _plans()
    small, big = plans[0], plans[2]
    need = _batch_bytes(big.info, "metric")
    assert _batch_bytes(small.info, "forward") * 32 <= need + 256   # the small one is graphed
    server = Server(hbm_budget_bytes=need + 256, max_batch=1, n_streams=1, use_graphs=True)
    sid, bid = server.register(small), server.register(big)
    xs = torch.randn(small.info["n_xi"], device="cuda")
    out_s = torch.empty(small.info["n_out"], device="cuda")
    server.submit(sid, "forward", xs, out_s)
    server.drain(30.0)
    assert server.stats()["graph_captures"] == 1        # its graph stays in the arena
    v = torch.randn(big.info["n_xi"], device="cuda")
    w = (torch.rand(big.info["n_out"], device="cuda") < 0.7).float() * 100.0
    out_b = torch.full((big.info["n_xi"],), float("nan"), device="cuda")
    rid = server.submit(bid, "metric", v, out_b, w)
    server.drain(30.0)                                   # raises on a time-out
    assert server.query(rid)[0]
    from paper_2402_16683_amd import icr as B
    assert torch.equal(out_b, B.icr_metric_apply(big, w, v[None])[0])
    assert torch.equal(out_s, B.icr_forward(small, xs[None])[0])
    server.close()


def test_a_lone_request_with_large_rows_skips_the_graph():
    """With graphs on, a batch of one whose input rows reach 1 MiB sweeps its own buffers
    (no capture, no gather or scatter) and gives the direct call's bits; a small lone
    request is still captured."""
    import torch
    from paper_2402_16683_amd.serve import Server
    from paper_2402_16683_amd import icr as B
    big = C.gpu_plan(C.case(3, (8, 8, 8), 4, (0.06, 0.06, 0.06), "matern52", 0.2, name="big_rows"))
    small = _plans()[0]
    assert big.info["n_xi"] * big.info["elem_bytes"] >= 1 << 20
    assert big.info["n_out"] * big.info["elem_bytes"] >= 1 << 20
    assert small.info["n_xi"] * small.info["elem_bytes"] < 1 << 20
    server = Server(hbm_budget_bytes=1 << 30, max_batch=1, n_streams=1, use_graphs=True)
    bid, sid = server.register(big), server.register(small)
    for op in ("forward", "adjoint", "metric"):
        n_in = big.info["n_out"] if op == "adjoint" else big.info["n_xi"]
        n_out = big.info["n_out"] if op == "forward" else big.info["n_xi"]
        x = torch.randn(n_in, device="cuda")
        w = (torch.rand(big.info["n_out"], device="cuda") < 0.7).float() * 10.0
        out = torch.full((n_out,), float("nan"), device="cuda")
        torch.cuda.synchronize()
        rid = server.submit(bid, op, x, out, w if op == "metric" else None)
        server.drain(30.0)
        assert server.query(rid)[0]
        if op == "forward":
            ref = B.icr_forward(big, x[None])[0]
        elif op == "adjoint":
            ref = B.icr_adjoint(big, x[None])[0]
        else:
            ref = B.icr_metric_apply(big, w, x[None])[0]
        assert torch.equal(out, ref), op
    assert server.stats()["graph_captures"] == 0
    xs = torch.randn(small.info["n_xi"], device="cuda")
    out_s = torch.empty(small.info["n_out"], device="cuda")
    torch.cuda.synchronize()
    server.submit(sid, "forward", xs, out_s)
    server.drain(30.0)
    assert server.stats()["graph_captures"] == 1
    assert torch.equal(out_s, B.icr_forward(small, xs[None])[0])
    server.close()


# --- grouped mode: requests of any prior and op share launches ----------------------

def _serve_one_at_a_time(server, ids, r):
    rid = server.submit(ids[r["k"]], r["op"], r["inp"], r["out"], r["w"] if r["op"] == "metric" else None)
    server.drain(60.0)
    return server.query(rid)


def _oracle_check(reqs, models):
    for r in reqs:
        c, m = POOL[r["k"]], models[r["k"]]
        inp = C.to_numpy(r["inp"])
        if r["op"] == "forward":
            ref = m.forward(inp)
        elif r["op"] == "adjoint":
            ref = m.adjoint(inp)
        else:
            ref = m.metric(C.to_numpy(r["w"]), inp)
        got = C.to_numpy(r["out"])
        assert np.all(np.isfinite(got)), (c["name"], r["op"])
        rms, mx = C.rel_errors(got, ref)
        tol_rms, tol_max = C.TOL[c["precision"]]
        assert rms <= tol_rms and mx <= tol_max, (c["name"], r["op"], rms, mx)


@pytest.mark.parametrize("group_streams", [1, 2])
def test_grouped_requests_match_the_oracle_and_their_results_alone(group_streams):
    """Every prior of the pool (1-D, 2-D, 3-D, charted, FP32 and BF16) with every op: the
    2-D and 3-D requests in groups sharing launches, the 1-D ones in homogeneous batches
    (their own sweep fuses the small levels into one launch). Each result matches the FP64
    oracle and equals, bit for bit, the same request served alone by a grouped server."""
    import torch
    from paper_2402_16683_amd.serve import Server
    plans = _plans()
    models = [C.oracle_model(c) for c in POOL]
    server = Server(hbm_budget_bytes=1 << 30, max_batch=16, n_streams=4, use_graphs=False, grouped=True,
                    large_step=1 << 40, group_streams=group_streams)
    reqs = _requests(plans, 150, seed=21)
    info = _serve(server, plans, reqs)
    assert all(q[0] for q in info)
    torch.cuda.synchronize()
    st = server.stats()
    n1 = sum(POOL[r["k"]]["ndim"] == 1 for r in reqs)
    assert 0 < n1 < 150
    assert st["grouped_requests"] == 150 - n1 and st["batched_requests"] == n1
    assert st["groups"] < 150 - n1               # requests shared launches
    assert max(q[4] for q in info) > 1
    _oracle_check(reqs, models)
    alone = Server(hbm_budget_bytes=1 << 30, max_batch=16, n_streams=1, use_graphs=False, grouped=True,
                   large_step=1 << 40)
    ids = [alone.register(p) for p in plans]
    for r in reqs[:60]:
        mixed = r["out"].clone()
        r["out"].fill_(float("nan"))
        q = _serve_one_at_a_time(alone, ids, r)
        torch.cuda.synchronize()
        assert q[0] and q[4] == 1
        assert torch.equal(r["out"], mixed), (r["k"], r["op"])
    alone.close()
    server.close()


def test_grouped_and_homogeneous_paths_together():
    """With a small large-step size some priors run as homogeneous batches beside the
    groups; all results match the oracle, and a tight budget defers admissions."""
    import torch
    from paper_2402_16683_amd.serve import Server
    plans = _plans()
    models = [C.oracle_model(c) for c in POOL]
    for budget in (1 << 30, 3 * max(p.info["n_xi"] * 4 * 4 for p in plans)):
        server = Server(hbm_budget_bytes=budget, max_batch=8, n_streams=4, use_graphs=False, grouped=True,
                        large_step=2000, group_streams=2)
        reqs = _requests(plans, 100, seed=22)
        info = _serve(server, plans, reqs)
        assert all(q[0] for q in info)
        torch.cuda.synchronize()
        st = server.stats()
        assert st["grouped_requests"] > 0 and st["batched_requests"] > 0 and st["arena_in_use"] == 0
        _oracle_check(reqs, models)
        server.close()


def test_submission_by_configuration_builds_caches_and_evicts_plans():
    """Requests by prior configuration: the server builds each new configuration's plan
    once (a builder thread, inside the request's latency), serves later requests from the
    cache, evicts idle plans beyond max_plans, and reports a failed build through the
    request's query."""
    import torch
    from paper_2402_16683_amd import icr as B
    from paper_2402_16683_amd.serve import Server
    cases = POOL[:4]
    cfgs = [B.make_config(c["ndim"], c["shape0"], c["depth"], c["delta0"], kernel=c["kernel"], length=c["length"],
                          chart=c["chart"], chart_params=c["chart_params"], precision=c["precision"]) for c in cases]
    models = [C.oracle_model(c) for c in cases]
    server = Server(hbm_budget_bytes=1 << 30, max_batch=8, n_streams=4, use_graphs=False, grouped=True,
                    large_step=1 << 40, max_plans=2)
    rng = np.random.default_rng(23)
    done = []
    for i in range(40):
        k = int(rng.integers(0, 4))
        n_xi = models[k].n_xi
        v = torch.from_numpy(W.standard_normal(n_xi, seed=100 + i)).float().cuda()
        out = torch.full((models[k].out_size,), float("nan"), device="cuda")
        rid = server.submit_prior(cfgs[k], "forward", v, out)
        done.append((rid, k, v, out))
        if i % 10 == 9:
            server.drain(60.0)
    server.drain(60.0)
    torch.cuda.synchronize()
    for rid, k, v, out in done:
        assert server.query(rid)[0]
        rms, _ = C.rel_errors(C.to_numpy(out), models[k].forward(C.to_numpy(v)))
        assert rms <= 1e-5
    st = server.stats()
    assert st["plans_built"] >= 4 and st["plan_cache_hits"] > 0 and st["completed"] == 40
    # an indefinite configuration with clamping disabled fails to build
    bad = B.make_config(2, (16, 16), 7, (128 / 1540,) * 2, kernel="sqexp", length=0.05, clamp=False)
    n_xi = sum((2 ** l * (16 - 4) + 4) ** 2 if l else 256 for l in range(8))
    v = torch.zeros(n_xi, device="cuda")
    out = torch.zeros(1540 * 1540, device="cuda")
    rid = server.submit_prior(bad, "forward", v, out)
    server.drain(120.0)
    with pytest.raises(B.ICRError) as e:
        server.query(rid)
    assert e.value.status == 2
    server.close()
