"""End-to-end parity of the HIP ICR path (device FP64 build + sweep) with the
FP64 oracle, level by level, on well-conditioned cases.

Both sides get the same seeded inputs (the values the device stores, up-cast
exactly for the oracle) and each builds its own matrices in FP64. Outputs and
workspaces start as NaN, so a pixel a kernel never writes fails the comparison. Results are
compared per level by rel-RMS and relative max error against the tolerance of
the precision (FP32 1e-5, BF16 storage 1e-2 rel-RMS; FP64 1e-10, the agreement
two FP64 builds of R = K_fc K_cc^-1 can reach at cond(K_cc) ~ 1e5).
Ill-conditioned builds (squared exponential at small delta/length) are checked
by residuals in test_gpu_build.py and their sweeps with identical matrices in
test_gpu_sweep.py.
"""

import numpy as np
import pytest

import workloads as W
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

CASES = [
    C.from_workload("icr1d_m32_12to260", batch=3, name="1d_m32_full_f64"),
    C.from_workload("icr1d_m32_12to260", precision="f32", name="1d_m32_full_f32"),
    C.from_workload("icr1d_m32_12to260", precision="bf16", name="1d_m32_full_bf16"),
    C.from_workload("icr2d_se_16to1540_b16", depth=4, batch=2, name="2d_se_16to196_b2_f32"),
    C.from_workload("icr2d_se_16to1540_b16", depth=3, precision="f64", name="2d_se_16to100_f64"),
    C.from_workload("icr3d_m52_10to388", name="3d_m52_full_f32"),
    C.from_workload("icr3d_m52_10to388", precision="bf16", name="3d_m52_full_bf16"),
    C.from_workload("icr3d_m52_10to388", depth=3, name="3d_m52_10to52_f32"),
    C.from_workload("icr3d_m52_10to388", depth=2, precision="bf16", name="3d_m52_10to28_bf16"),
    C.from_workload("icr3d_m52_10to388", depth=2, precision="f64", name="3d_m52_10to28_f64"),
    C.case(3, (5, 7, 6), 2, (0.1, 0.12, 0.09), "matern32", 0.3, batch=2, name="3d_ragged_f32"),
    C.case(2, (9, 5), 3, (0.05, 0.07), "matern12", 0.2, precision="f64", name="2d_ragged_m12_f64"),
    # odd rows, even row length at every level: the 2-D fast adjoint on all levels
    C.case(2, (11, 8), 4, (0.03, 0.035), "matern52", 0.15, batch=3, name="2d_ragged_m52_f32"),
    # odd row length at level 0 (generic kernel), even above (fast adjoint)
    C.case(2, (8, 9), 4, (0.04, 0.03), "matern32", 0.2, batch=2, precision="bf16", name="2d_ragged_m32_bf16"),
    C.case(1, (7,), 4, (0.1,), "sqexp", 0.4, batch=4, name="1d_se_f32"),
    C.from_workload("icr2d_chart_24to1284", depth=3, name="2d_chart_24to164_f32"),
    # the charted workload at its stated size, 24^2 -> 1284^2 over six levels
    C.from_workload("icr2d_chart_24to1284", name="2d_chart_full_f32"),
    C.from_workload("icr2d_chart_24to1284", precision="bf16", batch=2, name="2d_chart_full_b2_bf16"),
    C.from_workload("icr2d_chart_24to1284", depth=2, precision="f64", name="2d_chart_24to84_f64"),
    # 2-D chart, one set per radial shell: the 2-D fast kernels read a row per coarse row;
    # an odd row length at level 0 sends that level to the generic kernels
    C.case(2, (9, 12), 3, (1 / 9, 1 / 12), "matern32", 0.08, chart="logradial2d", batch=2, precision="bf16",
           name="2d_chart_ragged_b2_bf16"),
    C.case(2, (12, 9), 3, (1 / 12, 1 / 9), "matern52", 0.1, chart="logradial2d", batch=2,
           name="2d_chart_oddx_b2_f32"),
    C.from_workload("icr3d_chart_10to388", depth=3, name="3d_chart_10to52_f32"),
    C.from_workload("icr3d_chart_10to388", depth=3, precision="bf16", name="3d_chart_10to52_bf16"),
    C.from_workload("icr3d_chart_10to388", depth=2, precision="f64", name="3d_chart_10to28_f64"),
    C.case(3, (6, 7, 5), 2, (1 / 6, 1 / 7, 1 / 5), "matern52", 0.2, chart="logradial_cyl3d",
           chart_params=(0.2, 1.5, 1.2, 0.7), batch=2, name="3d_chart_ragged_f32"),
    # odd level-0 sizes: every later level's slice (and every sample, the batch stride n_xi
    # being odd) starts 1-3 elements off a vector boundary, so the fast 2-D and 3-D kernels
    # run with element accesses (their level-0 refinement, of odd row length, is generic)
    C.case(3, (9, 9, 9), 3, (0.06, 0.06, 0.06), "matern52", 0.2, batch=2, name="3d_odd9_b2_f32"),
    C.case(3, (9, 9, 9), 3, (0.06, 0.06, 0.06), "matern52", 0.2, batch=2, precision="bf16", name="3d_odd9_b2_bf16"),
    C.case(2, (11, 11), 4, (0.04, 0.04), "matern32", 0.15, batch=3, name="2d_odd11_b3_f32"),
    C.case(2, (11, 13), 3, (0.05, 0.04), "matern52", 0.2, batch=2, precision="bf16", name="2d_odd11x13_b2_bf16"),
    C.case(2, (11, 11), 3, (1 / 11, 1 / 11), "matern32", 0.1, chart="logradial2d", batch=2,
           name="2d_chart_odd11_b2_f32"),
    C.case(2, (6, 6), 0, (0.2, 0.2), "matern52", 0.5, batch=2, name="2d_depth0_f32"),
    C.case(3, (3, 3, 3), 1, (0.2, 0.2, 0.2), "matern52", 0.5, precision="f64", name="3d_min_f64"),
]

_cache = {}


def _setup(c):
    if c["name"] not in _cache:
        model = C.oracle_model(c)
        plan = C.gpu_plan(c)
        _cache[c["name"]] = (model, plan)
    return _cache[c["name"]]


def _levels(flat, info, upto):
    offs = info["level_offsets"]
    return [flat[..., offs[l]:offs[l + 1]] for l in range(upto)]


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_forward_matches_oracle_per_level(c):
    import torch
    model, plan = _setup(c)
    info = plan.info
    B = c["batch"]
    xi = W.standard_normal(info["n_xi"], seed=0, batch=B)
    xi_dev = C.to_device(xi, plan)
    ws = torch.full((B, max(info["workspace_elems"], 1)), float("nan"), dtype=plan.dtype, device="cuda")
    from paper_2402_16683_amd import icr as Bd
    s = Bd.icr_forward(plan, xi_dev, s=C.nan_like((B, info["n_out"]), plan), workspace=ws)
    torch.cuda.synchronize()
    _, ref_levels = model.forward(C.stored_values(xi, c["precision"]), return_levels=True)
    got_levels = _levels(C.to_numpy(ws), info, c["depth"]) + [C.to_numpy(s)]
    tol_rms, tol_max = C.TOL[c["precision"]]
    for l, (g, r) in enumerate(zip(got_levels, ref_levels)):
        rms, mx = C.rel_errors(g, r)
        print(f"[errors] {c['name']} forward s level {l}: rel-RMS {rms:.2e} rel-max {mx:.2e}")
        assert np.all(np.isfinite(g)), f"level {l} has unwritten/non-finite values"
        assert rms <= tol_rms and mx <= tol_max, f"level {l}: rel-RMS {rms:.3g}, rel-max {mx:.3g}"
    if c["precision"] == "bf16":
        # against the oracle on the un-rounded excitations too
        rms, _ = C.rel_errors(got_levels[-1], model.forward(xi))
        assert rms <= tol_rms


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_adjoint_matches_oracle_per_level(c):
    import torch
    model, plan = _setup(c)
    info = plan.info
    B = c["batch"]
    y = W.standard_normal(info["n_out"], seed=1, batch=B)
    ws = torch.full((B, max(info["workspace_elems"], 1)), float("nan"), dtype=plan.dtype, device="cuda")
    from paper_2402_16683_amd import icr as Bd
    xib = Bd.icr_adjoint(plan, C.to_device(y, plan), xi_bar=C.nan_like((B, info["n_xi"]), plan), workspace=ws)
    torch.cuda.synchronize()
    ref, ref_cot = model.adjoint(C.stored_values(y, c["precision"]), return_levels=True)
    got = C.to_numpy(xib)
    assert np.all(np.isfinite(got)), "xi_bar has unwritten/non-finite values"
    tol_rms, tol_max = C.TOL[c["precision"]]
    offs = info["level_offsets"]
    for l in range(c["depth"] + 1):
        rms, mx = C.rel_errors(got[..., offs[l]:offs[l + 1]], ref[..., offs[l]:offs[l + 1]])
        print(f"[errors] {c['name']} adjoint xi_bar level {l}: rel-RMS {rms:.2e} rel-max {mx:.2e}")
        assert rms <= tol_rms and mx <= tol_max, f"xi_bar level {l}: rel-RMS {rms:.3g}, rel-max {mx:.3g}"
    cot = _levels(C.to_numpy(ws), info, c["depth"])
    for l in range(c["depth"]):
        rms, mx = C.rel_errors(cot[l], ref_cot[l])
        assert rms <= tol_rms and mx <= tol_max, f"s_bar level {l}: rel-RMS {rms:.3g}, rel-max {mx:.3g}"


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_metric_matches_oracle(c):
    import torch
    model, plan = _setup(c)
    info = plan.info
    B = c["batch"]
    v = W.standard_normal(info["n_xi"], seed=2, batch=B)
    mask = W.bernoulli_mask(info["n_out"], 0.7, seed=4)
    w = mask / 0.1 ** 2
    from paper_2402_16683_amd import icr as Bd
    w_dev = torch.from_numpy(w).to(device="cuda", dtype=plan.acc_dtype)
    ws = C.nan_like((B, info["metric_workspace_elems"]), plan)
    out = Bd.icr_metric_apply(plan, w_dev, C.to_device(v, plan), out=C.nan_like((B, info["n_xi"]), plan),
                              workspace=ws)
    torch.cuda.synchronize()
    ref = model.metric(w, C.stored_values(v, c["precision"]))
    assert np.all(np.isfinite(C.to_numpy(out))), "metric output has unwritten/non-finite values"
    rms, mx = C.rel_errors(C.to_numpy(out), ref)
    tol_rms, tol_max = C.TOL[c["precision"]]
    assert rms <= tol_rms and mx <= tol_max, f"rel-RMS {rms:.3g}, rel-max {mx:.3g}"


@pytest.mark.parametrize("c", CASES, ids=[c["name"] for c in CASES])
def test_adjoint_identity_and_determinism(c):
    """<L xi, y> = <xi, L^T y> on the device results (dots in FP64), and a repeat
    of each call is bitwise identical."""
    import torch
    _, plan = _setup(c)
    info = plan.info
    B = c["batch"]
    from paper_2402_16683_amd import icr as Bd
    xi = C.to_device(W.standard_normal(info["n_xi"], seed=5, batch=B), plan)
    y = C.to_device(W.standard_normal(info["n_out"], seed=6, batch=B), plan)
    s1 = Bd.icr_forward(plan, xi)
    s2 = Bd.icr_forward(plan, xi)
    a1 = Bd.icr_adjoint(plan, y)
    a2 = Bd.icr_adjoint(plan, y)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2) and torch.equal(a1, a2)
    lhs = np.sum(C.to_numpy(s1) * C.to_numpy(y), axis=-1)
    rhs = np.sum(C.to_numpy(xi) * C.to_numpy(a1), axis=-1)
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}[c["precision"]]
    scale = np.linalg.norm(C.to_numpy(s1), axis=-1) * np.linalg.norm(C.to_numpy(y), axis=-1)
    assert np.all(np.abs(lhs - rhs) <= tol * scale)
