"""icr_metric_apply_static, the metric without a workspace argument (its workspace is the
library's static device scratch), called through the C ABI: equal bit for bit to
icr_metric_apply (the same kernels in the same order) on two calls in a row, the second
with a smaller input; outputs start as NaN so an unwritten element fails; a call that
needs more than the 64 MiB scratch is refused before any launch."""

import ctypes

import numpy as np
import pytest

import workloads as W
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

BIG = C.from_workload("icr3d_m52_10to388", depth=4, batch=3, name="static_3d_10to100_b3")   # 14 MB of workspace
SMALL = C.case(2, (11, 8), 4, (0.03, 0.035), "matern52", 0.15, batch=2, name="static_2d_ragged_b2")


def _call_static(plan, w, w_stride, v, out):
    import torch
    from paper_2402_16683_amd import icr as B
    lib = B.load_library()
    st = torch.cuda.current_stream().cuda_stream
    return lib.icr_metric_apply_static(plan.handle, v.shape[0], ctypes.c_void_p(w.data_ptr()), w_stride,
                                       ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(st))


def _inputs(plan, c, seed, per_sample_w):
    import torch
    info = plan.info
    v = C.to_device(W.standard_normal(info["n_xi"], seed=seed, batch=c["batch"]), plan)
    if per_sample_w:
        w = np.stack([W.bernoulli_mask(info["n_out"], 0.7, seed=seed + 1 + k) / 0.01 for k in range(c["batch"])])
        stride = info["n_out"]
    else:
        w = W.bernoulli_mask(info["n_out"], 0.7, seed=seed + 1) / 0.01
        stride = 0
    return v, torch.from_numpy(w).to("cuda", plan.acc_dtype), stride


def test_static_scratch_metric_equals_the_workspace_metric_on_consecutive_calls():
    import torch
    from paper_2402_16683_amd import icr as B
    plans = {c["name"]: C.gpu_plan(c) for c in (BIG, SMALL)}
    # two calls in a row, the second smaller; then the large one again over the smaller
    # one's leftovers in the shared scratch
    for c, seed, per_sample in ((BIG, 30, False), (SMALL, 40, True), (BIG, 50, True)):
        plan = plans[c["name"]]
        v, w, stride = _inputs(plan, c, seed, per_sample)
        out = C.nan_like(tuple(v.shape), plan)
        rc = _call_static(plan, w, stride, v, out)
        assert rc == 0, B.icr_last_error()
        ref = B.icr_metric_apply(plan, w, v)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all(), c["name"]
        assert torch.equal(out, ref), c["name"]
    # the Python binding of the same entry point
    plan = plans[SMALL["name"]]
    v, w, _ = _inputs(plan, SMALL, 60, False)
    got = B.icr_metric_apply_static(plan, w, v)
    torch.cuda.synchronize()
    assert torch.equal(got, B.icr_metric_apply(plan, w, v))


def test_static_scratch_refuses_a_call_beyond_its_size():
    import torch
    from paper_2402_16683_amd import icr as B
    c = C.from_workload("icr3d_m52_10to388", name="static_3d_full")      # 268 MB of workspace
    plan = C.gpu_plan(c)
    v = torch.zeros((1, plan.info["n_xi"]), dtype=plan.dtype, device="cuda")
    w = torch.ones(plan.info["n_out"], dtype=plan.acc_dtype, device="cuda")
    out = C.nan_like(tuple(v.shape), plan)
    rc = _call_static(plan, w, 0, v, out)
    assert rc == 1 and "static" in B.icr_last_error()
    torch.cuda.synchronize()
    assert torch.isnan(out).all()          # nothing was launched
