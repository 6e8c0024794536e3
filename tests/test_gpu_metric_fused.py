"""The metric's fused finest level (2-D): icr_metric_apply runs the forward of the finest
level times w and its adjoint plus v in one kernel, without storing the weighted fine
field. Its result is compared with the two separate sweeps the metric is made of,
out = icr_adjoint(w * icr_forward(v)) + v, on the same device plans: with FP32 storage
both do the same floating-point operations in the same order (agreement to rounding of
the final sum at most); with bfloat16 storage the separate sweeps round w * s to bfloat16
before the adjoint and the fused kernel does not, so they agree to the storage
tolerance. The oracle comparisons of the metric are in test_gpu_parity.py and
test_gpu_sweep.py; here the cases also cover the row marches the fused kernel takes at
batch 1, 3 and 16 (one, several and six rows per wavefront on the finest level) and a
level whose odd row count leaves a ragged last chunk."""

import numpy as np
import pytest

import workloads as W
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

CASES = [
    C.from_workload("icr2d_chart_24to1284", name="2d_chart_full_b1_f32"),
    C.from_workload("icr2d_chart_24to1284", batch=3, name="2d_chart_full_b3_f32"),
    C.from_workload("icr2d_chart_24to1284", precision="bf16", batch=2, name="2d_chart_full_b2_bf16"),
    C.from_workload("icr2d_se_16to1540_b16", name="2d_se_full_b16_f32"),
    C.case(2, (11, 8), 4, (0.03, 0.035), "matern52", 0.15, batch=3, name="2d_ragged_m52_b3_f32"),
    C.case(2, (12, 9), 3, (1 / 12, 1 / 9), "matern52", 0.1, chart="logradial2d", batch=2,
           name="2d_chart_oddx_b2_f32"),
    # the forward stops where the one-launch smallest levels end (16^2 -> 28^2 in one launch,
    # then the fused 28^2 -> 52^2 level), and the adjoint starts there
    C.from_workload("icr2d_se_16to1540_b16", depth=2, batch=2, name="2d_se_16to52_b2_f32"),
    # an odd level-0 size: the fused level (and the sweeps) with element accesses
    C.case(2, (11, 11), 4, (0.04, 0.04), "matern32", 0.15, batch=2, name="2d_odd11_b2_f32"),
    # depth 1: level 0, then the fused 24^2 -> 44^2 level
    C.from_workload("icr2d_chart_24to1284", depth=1, batch=2, name="2d_chart_24to44_b2_f32"),
    # a 3-D plan takes the two sweeps (the same kernels with and without the w and +v
    # epilogues)
    C.from_workload("icr3d_m52_10to388", depth=3, batch=2, name="3d_m52_10to52_b2_f32"),
]


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_fused_metric_equals_the_two_sweeps(c):
    import torch
    from paper_2402_16683_amd import icr as B
    plan = C.gpu_plan(c)
    info = plan.info
    batch = c["batch"]
    print(f"[case] {c['name']} batch {batch}", flush=True)
    v = C.to_device(W.standard_normal(info["n_xi"], seed=12, batch=batch), plan)
    w = torch.from_numpy(W.bernoulli_mask(info["n_out"], 0.7, seed=13) / 0.1 ** 2).to("cuda", plan.acc_dtype)
    out = B.icr_metric_apply(plan, w, v, out=C.nan_like((batch, info["n_xi"]), plan),
                             workspace=C.nan_like((batch, info["metric_workspace_elems"]), plan))
    s = B.icr_forward(plan, v, s=C.nan_like((batch, info["n_out"]), plan))
    y = (w * s.to(plan.acc_dtype)).to(plan.dtype)
    xib = B.icr_adjoint(plan, y, xi_bar=C.nan_like((batch, info["n_xi"]), plan))
    ref = (xib.to(plan.acc_dtype) + v.to(plan.acc_dtype)).to(plan.dtype)
    torch.cuda.synchronize()
    got = C.to_numpy(out)
    assert np.all(np.isfinite(got)), "metric output has unwritten/non-finite values"
    rms, mx = C.rel_errors(got, C.to_numpy(ref))
    print(f"[errors] {c['name']}: rel-RMS {rms:.2e} rel-max {mx:.2e} bitwise {torch.equal(out, ref)}")
    tol_rms, tol_max = (1e-6, 1e-5) if c["precision"] == "f32" else C.TOL[c["precision"]]
    assert rms <= tol_rms and mx <= tol_max, f"rel-RMS {rms:.3g}, rel-max {mx:.3g}"
