"""Differentiation through the HIP sweep and the on-device CG metric solve.

* autograd: the backward of s = L xi is icr_adjoint. torch.autograd.gradcheck on the FP64
  path (the map is linear, so finite differences are exact up to rounding); on the FP32
  path the gradient of a nonlinear Gaussian-likelihood loss is compared with central finite
  differences along random directions; the backward equals the oracle's L^T.
* CG: icr_cg_metric on the charted 2-D prior against a dense solve of the oracle's metric
  (FP64), its residual norms against the oracle's residuals, and FP32 against FP64.
"""

import numpy as np
import pytest

import workloads as W
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
