"""Differentiation through the HIP sweep and the on-device CG metric solve.

* autograd: the backward of s = L xi is icr_adjoint. torch.autograd.gradcheck on the FP64
  path (the map is linear, so finite differences are exact up to rounding); on the FP32
  path the gradient of a nonlinear Gaussian-likelihood loss is compared with central finite
  differences along random directions; the backward equals the oracle's L^T.
* CG: icr_cg_metric on the charted 2-D prior against a dense solve of the oracle's metric
  (FP64), its residual norms against the oracle's residuals, and FP32 against FP64.
"""

import math

import numpy as np
import pytest

import workloads as W
from oracle import icr_oracle as O
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

SMALL_F64 = C.case(2, (6, 5), 2, (0.1, 0.12), "matern32", 0.3, precision="f64", name="grad_2d_f64")
SMALL_F32 = C.case(3, (5, 6, 5), 2, (0.1, 0.1, 0.1), "matern52", 0.4, precision="f32", name="grad_3d_f32")
CHART = C.from_workload("icr2d_chart_24to1284", depth=1, name="cg_chart_24to44")


def test_gradcheck_fp64():
    import torch
    from paper_2402_16683_amd.autograd import icr_sample
    plan = C.gpu_plan(SMALL_F64)
    xi = torch.from_numpy(W.standard_normal(plan.info["n_xi"], seed=1, batch=2)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: icr_sample(plan, x), (xi,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_backward_is_the_oracle_transpose():
    import torch
    from paper_2402_16683_amd.autograd import icr_sample
    plan = C.gpu_plan(SMALL_F64)
    model = C.oracle_model(SMALL_F64)
    xi = torch.zeros((1, plan.info["n_xi"]), dtype=torch.float64, device="cuda", requires_grad=True)
    g = W.standard_normal(plan.info["n_out"], seed=3, batch=1)
    (icr_sample(plan, xi) * torch.from_numpy(g).cuda()).sum().backward()
    ref = model.adjoint(g)
    rms, _ = C.rel_errors(xi.grad.cpu().numpy(), ref)
    assert rms <= 1e-10


def test_fp32_gradient_of_a_gaussian_likelihood_matches_finite_differences():
    import torch
    from paper_2402_16683_amd.autograd import icr_sample
    plan = C.gpu_plan(SMALL_F32)
    n_xi, n_out = plan.info["n_xi"], plan.info["n_out"]
    mask = torch.from_numpy(W.bernoulli_mask(n_out, 0.7, seed=4)).float().cuda()
    truth = torch.from_numpy(W.standard_normal(n_xi, seed=2, batch=1)).float().cuda()
    noise = 0.1 * torch.from_numpy(W.standard_normal(n_out, seed=3, batch=1)).float().cuda()
    data = mask * icr_sample(plan, truth).detach() + noise

    def loss(xi):  # 0.5 sum mask (d - s)^2 / sigma^2 + 0.5 |xi|^2, accumulated in FP64
        s = icr_sample(plan, xi)
        r = (mask * (data - s)).double()
        return 0.5 * (r * r).sum() / 0.01 + 0.5 * (xi.double() ** 2).sum()

    xi0 = torch.from_numpy(W.standard_normal(n_xi, seed=5, batch=1)).float().cuda().requires_grad_(True)
    loss(xi0).backward()
    grad = xi0.grad.double()
    rng = np.random.default_rng(6)
    for _ in range(3):
        d = torch.from_numpy(rng.standard_normal((1, n_xi))).float().cuda()
        d /= d.norm()
        h = 1e-2
        with torch.no_grad():
            fd = (loss(xi0 + h * d) - loss(xi0 - h * d)) / (2 * h)
        an = (grad * d.double()).sum()
        assert abs(float(fd - an)) <= 1e-3 * max(1.0, abs(float(an)))


def _charted_problem(precision, sigma_n=0.1):
    plan = C.gpu_plan(CHART, precision)
    model = C.oracle_model(CHART)
    n_xi, n_out = plan.info["n_xi"], plan.info["n_out"]
    mask = W.bernoulli_mask(n_out, 0.7, seed=4)
    w = mask / sigma_n ** 2
    truth = W.standard_normal(n_xi, seed=2)
    data = mask * model.forward(truth) + sigma_n * W.standard_normal(n_out, seed=3)
    b = model.adjoint(w * data)[None] + W.standard_normal(n_xi, seed=7, batch=1)
    return plan, model, w, b


def _textbook_cg(apply, b, iterations):
    """Conjugate gradients from x_0 = 0 (Hestenes & Stiefel), FP64, on the oracle's metric."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    for _ in range(iterations):
        q = apply(p)
        alpha = rr / (p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, np.sqrt(rr)


def test_cg_iterates_match_textbook_cg_on_the_oracle_metric():
    """On the workload's likelihood (sigma_n = 0.1) M has cond ~1.5e4 and CG iterates soon
    stop being determined by the algorithm: perturbing every product by 1e-15 relative moves
    the 25th iterate by ~1e-2 and its CG energy 0.5 x.Mx - b.x by ~3e-5 in FP64 numpy, while
    after 200 iterations the energy is stable to ~1e-9. So iterates are compared while they
    are well-determined (k <= 5) and the energy after 200 iterations. Identical matrices (the
    oracle's) are loaded into the plan."""
    import torch
    from paper_2402_16683_amd import icr as B
    plan, model, w, b = _charted_problem("f64")
    C.upload_oracle_matrices(plan, model)
    energy = lambda x: 0.5 * x @ model.metric(w, x) - b[0] @ x
    for k in (1, 3, 5, 200):
        x, norms = B.icr_cg_metric(plan, torch.from_numpy(w).cuda(), C.to_device(b, plan), k,
                                   residual_norms=True)
        torch.cuda.synchronize()
        ref, ref_norm = _textbook_cg(lambda v: model.metric(w, v), b[0], k)
        got = C.to_numpy(x)[0]
        if k <= 5:
            rms, _ = C.rel_errors(got, ref)
            assert rms <= 1e-10, (k, rms)
            assert abs(norms.cpu().numpy()[0, -1] - ref_norm) <= 1e-8 * ref_norm
        e_got, e_ref = energy(got), energy(ref)
        assert abs(e_got - e_ref) <= (1e-12 if k <= 5 else 1e-7) * abs(e_ref), (k, e_got, e_ref)
        nr = norms.cpu().numpy()[0]
        assert nr[-1] < nr[0]


def test_cg_converges_to_the_dense_solve():
    import torch
    from paper_2402_16683_amd import icr as B
    plan, model, w, b = _charted_problem("f64", sigma_n=1.0)
    x, norms = B.icr_cg_metric(plan, torch.from_numpy(w).cuda(), C.to_device(b, plan), 400,
                               residual_norms=True)
    torch.cuda.synchronize()
    n = plan.info["n_xi"]
    mat = np.stack([model.metric(w, e) for e in np.eye(n)], axis=1)
    ref = np.linalg.solve(mat, b[0])
    nr = norms.cpu().numpy()[0]
    assert nr[-1] <= 1e-9 * nr[0]
    rms, _ = C.rel_errors(C.to_numpy(x)[0], ref)
    assert rms <= 1e-8
    assert np.linalg.norm(b[0] - model.metric(w, C.to_numpy(x)[0])) <= 1e-8 * nr[0]


def test_cg_fp32_tracks_fp64_and_is_reproducible():
    import torch
    from paper_2402_16683_amd import icr as B
    plan64, _, w, b = _charted_problem("f64", sigma_n=1.0)
    plan32 = C.gpu_plan(CHART, "f32")
    x64 = B.icr_cg_metric(plan64, torch.from_numpy(w).cuda(), C.to_device(b, plan64), 60)
    wd = torch.from_numpy(w).float().cuda()
    x32a = B.icr_cg_metric(plan32, wd, C.to_device(b, plan32), 60)
    x32b = B.icr_cg_metric(plan32, wd, C.to_device(b, plan32), 60)
    torch.cuda.synchronize()
    assert torch.equal(x32a, x32b)
    rms, _ = C.rel_errors(C.to_numpy(x32a), C.to_numpy(x64))
    assert rms <= 1e-4


def test_cg_batched_right_hand_sides_are_independent():
    import torch
    from paper_2402_16683_amd import icr as B
    plan, model, w, b = _charted_problem("f64")
    b2 = np.concatenate([b, 2.0 * b + 1.0])
    xb = B.icr_cg_metric(plan, torch.from_numpy(w).cuda(), C.to_device(b2, plan), 40)
    x0 = B.icr_cg_metric(plan, torch.from_numpy(w).cuda(), C.to_device(b2[1:], plan), 40)
    torch.cuda.synchronize()
    assert torch.equal(xb[1:], x0)



def test_fp32_cg_with_the_split_dot_on_two_right_hand_sides():
    """FP32 CG on a 2-D chart, where p.q comes from the fused metric level (<L p, w L p>)
    and the previous p update (p.p) instead of a pass over p and q. Two right-hand sides of
    different size under the energy rule stop after different step counts; each sample's
    result equals, bit for bit, the fixed-count run of its step count in the same batch
    (a stopped sample's x, r, p no longer change), and agrees with the FP64 plan's
    fixed-count run of that many steps."""
    import torch
    from paper_2402_16683_amd import icr as B
    plan32, _, w, b = _charted_problem("f32", sigma_n=math.sqrt(10.0))
    plan64 = C.gpu_plan(CHART, "f64")
    n_xi = plan32.info["n_xi"]
    b2 = np.concatenate([b, 5.0 * b + W.standard_normal(n_xi, seed=8, batch=1)])
    wd = torch.from_numpy(w).float().cuda()
    bd = C.to_device(b2, plan32)
    absdelta = 1e-4 * n_xi / 10.0
    done = torch.zeros(2, dtype=torch.int32, device="cuda")
    x_sl = B.icr_cg_metric(plan32, wd, bd, 80, absdelta=absdelta, iterations_done=done)
    torch.cuda.synchronize()
    steps = done.cpu().numpy()
    print(f"[steps] FP32 energy rule on two right-hand sides: {steps.tolist()}")
    assert steps[0] != steps[1] and np.all((steps >= 2) & (steps < 80)), steps
    for k in range(2):
        x_fix = B.icr_cg_metric(plan32, wd, bd, int(steps[k]))
        x64 = B.icr_cg_metric(plan64, torch.from_numpy(w).cuda(), C.to_device(b2[k:k + 1], plan64), int(steps[k]))
        torch.cuda.synchronize()
        assert torch.equal(x_sl[k], x_fix[k]), k
        rms, _ = C.rel_errors(C.to_numpy(x_sl[k]), C.to_numpy(x64[0]))
        assert rms <= 1e-4, (k, rms)

# --- the charted workload at its stated size and shape -------------------------------

CHART_FULL = C.from_workload("icr2d_chart_24to1284", name="cg_chart_24to1284")
# a charted copy with a 32 x 32 output: 11^2 -> 18^2 -> 32^2, the same chart and kernel
CHART_32 = C.case(2, (11, 11), 2, (1 / 11, 1 / 11), "matern32", 0.05, chart="logradial2d", name="chart_32x32")
CHART_DEEP = C.from_workload("icr2d_chart_24to1284", depth=4, name="cg_chart_24to324")


def test_fp32_gradient_on_a_32x32_charted_copy_matches_finite_differences():
    """Central finite differences of the charted workload's likelihood energy
    0.5 sum mask (d - s)^2 / sigma^2 + 0.5 |xi|^2 (sigma 0.1, 30 % masked) on a copy whose
    output is 32 x 32, along random directions, against the autograd gradient (FP32)."""
    import torch
    from paper_2402_16683_amd.autograd import icr_sample
    plan = C.gpu_plan(CHART_32)
    n_xi, n_out = plan.info["n_xi"], plan.info["n_out"]
    assert plan.info["level_shapes"][-1] == (32, 32)
    mask = torch.from_numpy(W.bernoulli_mask(n_out, 0.7, seed=4)).float().cuda()
    truth = torch.from_numpy(W.standard_normal(n_xi, seed=2, batch=1)).float().cuda()
    noise = 0.1 * torch.from_numpy(W.standard_normal(n_out, seed=3, batch=1)).float().cuda()
    data = mask * icr_sample(plan, truth).detach() + noise

    def loss(xi):
        s = icr_sample(plan, xi)
        r = (mask * (data - s)).double()
        return 0.5 * (r * r).sum() / 0.01 + 0.5 * (xi.double() ** 2).sum()

    xi0 = torch.from_numpy(W.standard_normal(n_xi, seed=5, batch=1)).float().cuda().requires_grad_(True)
    loss(xi0).backward()
    grad = xi0.grad.double()
    rng = np.random.default_rng(8)
    for _ in range(4):
        d = torch.from_numpy(rng.standard_normal((1, n_xi))).float().cuda()
        d /= d.norm()
        h = 1e-2
        with torch.no_grad():
            fd = (loss(xi0 + h * d) - loss(xi0 - h * d)) / (2 * h)
        an = (grad * d.double()).sum()
        assert abs(float(fd - an)) <= 1e-3 * max(1.0, abs(float(an))), (float(fd), float(an))


def _workload_problem(case, precision, sigma_n=0.1):
    """The charted workload's data and right-hand side b = L^T W d (truth seed 2, noise
    seed 3, 70 % observed by a Bernoulli mask of seed 4), from the oracle."""
    plan = C.gpu_plan(case, precision)
    model = C.oracle_model(case)
    n_xi, n_out = plan.info["n_xi"], plan.info["n_out"]
    mask = W.bernoulli_mask(n_out, 0.7, seed=4)
    w = mask / sigma_n ** 2
    data = mask * model.forward(W.standard_normal(n_xi, seed=2)) + sigma_n * W.standard_normal(n_out, seed=3)
    b = model.adjoint(w * data)[None]
    return plan, model, w, b


def test_cg_iterates_on_a_deeper_chart_match_textbook_cg():
    """As the depth-1 comparison above, on the chart refined four times (24^2 -> 324^2):
    the first iterates to 1e-10, and the CG energy after 200 iterations to 3e-4. CG is far
    from converged there and its later iterates depend on rounding: perturbing every
    metric product of the FP64 oracle by 1e-15 (1e-14) relative moves the 200th energy by
    4e-6 (4.4e-5) and the iterate by 2e-3 (2e-2), measured; the device's FP64 sums run in
    another order."""
    import torch
    from paper_2402_16683_amd import icr as B
    plan, model, w, b = _workload_problem(CHART_DEEP, "f64")
    C.upload_oracle_matrices(plan, model)
    energy = lambda x: 0.5 * x @ model.metric(w, x) - b[0] @ x
    for k in (1, 4, 200):
        x = B.icr_cg_metric(plan, torch.from_numpy(w).cuda(), C.to_device(b, plan), k)
        torch.cuda.synchronize()
        ref, _ = _textbook_cg(lambda v: model.metric(w, v), b[0], k)
        got = C.to_numpy(x)[0]
        if k <= 4:
            rms, _ = C.rel_errors(got, ref)
            assert rms <= 1e-10, (k, rms)
        e_got, e_ref = energy(got), energy(ref)
        assert abs(e_got - e_ref) <= (1e-12 if k <= 4 else 3e-4) * abs(e_ref), (k, e_got, e_ref)


def test_fp32_cg_on_the_full_charted_workload_tracks_fp64():
    """200 CG iterations (metric products) on the charted workload at its stated size
    (24^2 -> 1284^2, sigma_n 0.1): the FP32 plan's residual reduction is within 10x of the
    FP64 plan's, and so is the true residual |b - M x| / |b| of its solution evaluated by
    the FP64 oracle. (The metric has cond ~1e4; both precisions reduce the residual
    by ~3e-3 in 200 steps.)"""
    import torch
    from paper_2402_16683_amd import icr as B
    plan64, model, w, b = _workload_problem(CHART_FULL, "f64")
    plan32 = C.gpu_plan(CHART_FULL, "f32")
    x64, n64 = B.icr_cg_metric(plan64, torch.from_numpy(w).cuda(), C.to_device(b, plan64), 200, residual_norms=True)
    x32, n32 = B.icr_cg_metric(plan32, torch.from_numpy(w).float().cuda(), C.to_device(b, plan32), 200,
                               residual_norms=True)
    torch.cuda.synchronize()
    red64 = float(n64[0, -1] / n64[0, 0])
    red32 = float(n32[0, -1] / n32[0, 0])
    true32 = np.linalg.norm(b[0] - model.metric(w, C.to_numpy(x32)[0])) / np.linalg.norm(b[0])
    print(f"[errors] charted CG 200 steps: |r|/|r0| FP64 {red64:.2e}, FP32 {red32:.2e}, FP32 true {true32:.2e}")
    assert red64 < 1e-1
    assert red32 <= 10 * red64 and true32 <= 10 * red64


def test_cg_energy_rule_matches_the_oracle():
    """icr_cg_metric_sl against the oracle's energy-change CG on identical matrices (FP64,
    weights 0.1 per observed pixel, where the iterates are well-determined: perturbing the
    oracle's products by 1e-14 moves them by ~1e-14, measured; at weight 1 the 18th iterate
    already moves by 1e-4): two right-hand sides of different size stop after different
    step counts, each equal to the oracle's; the solutions agree; a stopped sample's
    residual norm is repeated to the end."""
    import torch
    from paper_2402_16683_amd import icr as B
    plan, model, w, _ = _workload_problem(CHART, "f64", sigma_n=math.sqrt(10.0))
    C.upload_oracle_matrices(plan, model)
    n_xi = plan.info["n_xi"]
    b0 = W.standard_normal(n_xi, seed=7)
    b = np.stack([b0, 5.0 * b0 + W.standard_normal(n_xi, seed=8)])
    apply = lambda v: model.metric(w, v)
    maxiter = 80
    absdelta = 1e-4 * n_xi / 10.0            # the paper's example: 1e-4 * size / 10
    refs = [O.conjugate_gradient_sl(apply, bk, absdelta, maxiter) for bk in b]
    for _, steps, dec in refs:                # no decrease sits on the threshold
        assert steps < maxiter and np.min(np.abs(dec / absdelta - 1.0)) > 1e-6
    assert refs[0][1] != refs[1][1]
    done = torch.zeros(2, dtype=torch.int32, device="cuda")
    x, norms = B.icr_cg_metric(plan, torch.from_numpy(w).cuda(), C.to_device(b, plan), maxiter,
                               residual_norms=True, absdelta=absdelta, iterations_done=done)
    torch.cuda.synchronize()
    got_steps = done.cpu().numpy()
    nr = norms.cpu().numpy()
    for k, (xr, steps, _) in enumerate(refs):
        assert got_steps[k] == steps, (k, got_steps[k], steps)
        rms, _ = C.rel_errors(C.to_numpy(x)[k], xr)
        assert rms <= 1e-9, (k, rms)
        assert np.all(nr[k, steps:] == nr[k, steps])


def test_cg_energy_rule_halts_the_remaining_kernels():
    """On the full charted workload (FP32) a threshold reached early stops CG on the
    device: the result equals a fixed-count run of that many steps bit for bit, and the
    call takes far less time than the fixed-count run to the limit: kernels queued after
    the halt return at once, and the host stops enqueuing once it reads the pinned word
    the device raises with the flag. Eight copies of the right-hand side are solved
    together, so that a working step (~113 us at three, over twice that at eight) clearly
    outweighs the launches of the few halted steps the host enqueues before it sees the
    word (36-80 us of host time each)."""
    import torch
    from paper_2402_16683_amd import icr as B
    plan, model, w, b = _workload_problem(CHART_FULL, "f32")
    wd = torch.from_numpy(w).float().cuda()
    nrhs = 8
    bd = C.to_device(np.repeat(b, nrhs, axis=0), plan)
    mb = model.metric(w, C.stored_values(b[0], "f32"))
    bs = C.stored_values(b[0], "f32")
    first = 0.5 * (bs @ bs) ** 2 / (bs @ mb)   # the first step's energy decrease
    absdelta = 1e-3 * first
    ws = torch.empty(B.icr_cg_workspace_bytes(plan, nrhs), dtype=torch.uint8, device="cuda")
    done = torch.zeros(nrhs, dtype=torch.int32, device="cuda")
    maxiter = 100
    x_sl = B.icr_cg_metric(plan, wd, bd, maxiter, workspace=ws, absdelta=absdelta, iterations_done=done)
    torch.cuda.synchronize()
    counts = done.cpu().numpy()
    steps = int(counts[0])
    assert np.all(counts == steps) and 2 <= steps <= 60, counts
    x_fix = B.icr_cg_metric(plan, wd, bd, steps, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(x_sl, x_fix)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    t_sl = timed(lambda: B.icr_cg_metric(plan, wd, bd, maxiter, workspace=ws, absdelta=absdelta))
    t_fix = timed(lambda: B.icr_cg_metric(plan, wd, bd, maxiter, workspace=ws))
    print(f"[timing] energy rule stopped after {steps} of {maxiter} steps: {t_sl:.2f} ms vs {t_fix:.2f} ms")
    assert t_sl < 0.8 * t_fix


def test_cg_energy_rule_calls_back_to_back():
    """Early-stopping solves enqueued back to back without synchronising, on one stream and
    on two: a solve whose threshold stops it after one step, then one that stops by the
    rule after more steps (two right-hand sides of different size: different counts).
    Each result equals, bit for bit, the fixed-count run of the steps it took. So the
    pinned host word that an earlier solve's device work raises never stops a later solve
    early (each call holds its own word, handed out again only after its call's work has
    finished), and the host, which stops enqueuing once it reads the word, never stops a
    solve before it has finished."""
    import torch
    from paper_2402_16683_amd import icr as B
    plan, _, w, b = _charted_problem("f32", sigma_n=math.sqrt(10.0))
    n_xi = plan.info["n_xi"]
    wd = torch.from_numpy(w).float().cuda()
    bd = C.to_device(np.concatenate([b, 5.0 * b + W.standard_normal(n_xi, seed=8, batch=1)]), plan)
    maxiter = 80
    rule = 1e-4 * n_xi / 10.0                    # stops after 9 and 11 steps
    thresholds = [1e30, rule, 1e30, rule]        # 1e30: every sample stops after its first step
    ws_bytes = B.icr_cg_workspace_bytes(plan, 2)
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()                   # default priority
    runs = []
    for k, ad in enumerate(thresholds):
        st = main if k < 2 else side
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        x = torch.empty_like(bd)
        done = torch.zeros(2, dtype=torch.int32, device="cuda")
        if st is side:
            side.wait_stream(main)
        B.icr_cg_metric(plan, wd, bd, maxiter, x=x, workspace=ws, stream=st, absdelta=ad, iterations_done=done)
        runs.append((ad, x, done, ws))
    torch.cuda.synchronize()
    counts = [r[2].cpu().numpy() for r in runs]
    print(f"[steps] {[c.tolist() for c in counts]}")
    assert np.all(counts[0] == 1) and np.all(counts[2] == 1)
    for c in (counts[1], counts[3]):
        assert c[0] != c[1] and np.all((c >= 2) & (c < maxiter)), c
    for (ad, x, done, ws), c in zip(runs, counts):
        for j in range(2):
            x_fix = B.icr_cg_metric(plan, wd, bd, int(c[j]))
            torch.cuda.synchronize()
            assert torch.equal(x[j], x_fix[j]), (ad, j, int(c[j]))
