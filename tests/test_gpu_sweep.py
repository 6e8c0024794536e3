"""Sweep parity with identical matrices: the oracle's FP64 R, sqrtD and L00 are
loaded into the device plan (icr_plan_set_*), so only the HIP sweep kernels are
compared with the oracle's sweep, level by level. This covers the
ill-conditioned squared-exponential workloads, whose FP64 builds legitimately
differ (checked by residuals in test_gpu_build.py), and the full-size workloads in
the launch configuration the benchmark times.
"""

import numpy as np
import pytest

import workloads as W
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

CASES = [
    C.case(1, (7,), 6, (0.1,), "sqexp", 0.4, batch=4, name="1d_se_deep_f32"),
    C.from_workload("icr2d_se_16to1540_b16", batch=2, name="2d_se_full_b2_f32"),
    C.from_workload("icr2d_se_16to1540_b16", batch=2, precision="bf16", name="2d_se_full_b2_bf16"),
    # the 2-D workload at its benchmarked batch of 16: the 2-D kernels size their row marches
    # by the batch and the level, so the last three levels march 6, 13 and 4 rows per
    # wavefront (batch 2 marches 4, 2 and 1 rows there)
    C.from_workload("icr2d_se_16to1540_b16", name="2d_se_full_b16_f32"),
    C.from_workload("icr2d_se_16to1540_b16", precision="bf16", name="2d_se_full_b16_bf16"),
    # a large batch of small grids: every level in two chunks per sample (marches of 7 to
    # 50 rows); ragged last chunks are covered by the batch-16 case (770 rows in marches of
    # 6, 386 in marches of 13)
    C.from_workload("icr2d_se_16to1540_b16", depth=4, batch=1024, name="2d_se_16to196_b1024_f32"),
    C.from_workload("icr2d_se_16to1540_b16", depth=5, precision="f64", name="2d_se_16to388_f64"),
    C.from_workload("icr3d_m52_10to388", depth=4, batch=2, name="3d_m52_10to100_b2_f32"),
    C.from_workload("icr3d_m52_10to388", depth=4, precision="bf16", name="3d_m52_10to100_bf16"),
    C.from_workload("icr2d_chart_24to1284", depth=4, name="2d_chart_24to324_f32"),
    # shell rows: marches of at most 10 block rows take their matrix rows from LDS, longer
    # ones read the table row by row; at batch 4096 the 44^2 -> 84^2 level marches all its
    # 42 rows (44 in the adjoint) in one wavefront per sample (forward, adjoint and the
    # metric's fused level)
    C.from_workload("icr2d_chart_24to1284", depth=2, batch=4096, name="2d_chart_24to84_b4096_f32"),
    C.from_workload("icr3d_chart_10to388", depth=4, batch=2, name="3d_chart_10to100_b2_f32"),
    C.from_workload("icr3d_chart_10to388", depth=3, precision="bf16", name="3d_chart_10to52_bf16"),
    C.from_workload("icr3d_chart_10to388", depth=3, precision="f64", name="3d_chart_10to52_f64"),
    C.case(3, (4, 5, 6), 3, (0.2, 0.15, 0.1), "sqexp", 0.5, precision="f64", name="3d_se_ragged_f64"),
]

_cache = {}


def _setup(c):
    if c["name"] not in _cache:
        model = C.oracle_model(c)
        plan = C.gpu_plan(c)
        C.upload_oracle_matrices(plan, model)
        _cache[c["name"]] = (model, plan)
    return _cache[c["name"]]


def _check_levels(got_levels, ref_levels, prec, what):
    tol_rms, tol_max = C.TOL[prec]
    for l, (g, r) in enumerate(zip(got_levels, ref_levels)):
        assert np.all(np.isfinite(g)), f"{what} level {l}: non-finite values"
        rms, mx = C.rel_errors(g, r)
        assert rms <= tol_rms and mx <= tol_max, f"{what} level {l}: rel-RMS {rms:.3g}, rel-max {mx:.3g}"


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_sweep_forward_with_identical_matrices(c):
    import torch
    from paper_2402_16683_amd import icr as Bd
    model, plan = _setup(c)
    info = plan.info
    xi = W.standard_normal(info["n_xi"], seed=0, batch=c["batch"])
    ws = torch.full((c["batch"], max(info["workspace_elems"], 1)), float("nan"), dtype=plan.dtype,
                    device="cuda")
    s = Bd.icr_forward(plan, C.to_device(xi, plan), s=C.nan_like((c["batch"], info["n_out"]), plan), workspace=ws)
    torch.cuda.synchronize()
    _, ref = model.forward(C.stored_values(xi, c["precision"]), return_levels=True)
    got = C.level_views(C.to_numpy(ws), info["level_offsets"], c["depth"]) + [C.to_numpy(s)]
    _check_levels(got, ref, c["precision"], "s")


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_sweep_adjoint_with_identical_matrices(c):
    import torch
    from paper_2402_16683_amd import icr as Bd
    model, plan = _setup(c)
    info = plan.info
    y = W.standard_normal(info["n_out"], seed=1, batch=c["batch"])
    ws = torch.full((c["batch"], max(info["workspace_elems"], 1)), float("nan"), dtype=plan.dtype,
                    device="cuda")
    xib = Bd.icr_adjoint(plan, C.to_device(y, plan), xi_bar=C.nan_like((c["batch"], info["n_xi"]), plan),
                         workspace=ws)
    torch.cuda.synchronize()
    ref, ref_cot = model.adjoint(C.stored_values(y, c["precision"]), return_levels=True)
    offs = info["level_offsets"]
    got = C.to_numpy(xib)
    _check_levels(C.level_views(got, offs, c["depth"] + 1), C.level_views(ref, offs, c["depth"] + 1),
                  c["precision"], "xi_bar")
    _check_levels(C.level_views(C.to_numpy(ws), offs, c["depth"]), ref_cot[:-1], c["precision"], "s_bar")


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_sweep_metric_with_identical_matrices(c):
    import torch
    from paper_2402_16683_amd import icr as Bd
    model, plan = _setup(c)
    info = plan.info
    v = W.standard_normal(info["n_xi"], seed=2, batch=c["batch"])
    w = W.bernoulli_mask(info["n_out"], 0.7, seed=4) / 0.1 ** 2
    out = Bd.icr_metric_apply(plan, torch.from_numpy(w).to("cuda", plan.acc_dtype), C.to_device(v, plan),
                              out=C.nan_like((c["batch"], info["n_xi"]), plan),
                              workspace=C.nan_like((c["batch"], info["metric_workspace_elems"]), plan))
    torch.cuda.synchronize()
    assert np.all(np.isfinite(C.to_numpy(out))), "metric output has unwritten/non-finite values"
    ref = model.metric(w, C.stored_values(v, c["precision"]))
    rms, mx = C.rel_errors(C.to_numpy(out), ref)
    tol_rms, tol_max = C.TOL[c["precision"]]
    assert rms <= tol_rms and mx <= tol_max, f"rel-RMS {rms:.3g}, rel-max {mx:.3g}"
