"""The forward and adjoint sweeps replayed from a captured HIP graph.

The sweep calls allocate nothing and launch only on the caller's stream, so a caller can
capture them (torch.cuda.CUDAGraph drives hipStreamBeginCapture) and replay the launch
sequence without host work per launch. Each replay, with eager work and synchronisation
in between, must reproduce the eager result bit for bit (the same kernels run in the
same order), including the fused small-level launch and the 2-D and 3-D fast kernels.
"""

import numpy as np
import pytest

import workloads as W
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

CASES = [
    C.from_workload("icr1d_m32_12to260", batch=2, name="g1d_f64"),
    C.case(2, (12, 10), 4, (0.03, 0.035), "matern52", 0.15, batch=3, name="g2d_f32"),
    C.case(3, (8, 8, 8), 3, (0.06, 0.06, 0.06), "matern52", 0.2, batch=2, name="g3d_f32"),
    C.case(3, (8, 8, 8), 3, (0.06, 0.06, 0.06), "matern52", 0.2, batch=1, precision="bf16", name="g3d_bf16"),
]


@pytest.mark.parametrize("c", CASES, ids=lambda c: c["name"])
def test_graph_replays_equal_eager(c):
    import torch
    from paper_2402_16683_amd import icr as B
    plan = C.gpu_plan(c)
    info = plan.info
    nb = c["batch"]
    xi = C.to_device(W.standard_normal(info["n_xi"], seed=41, batch=nb), plan)
    y = C.to_device(W.standard_normal(info["n_out"], seed=42, batch=nb), plan)
    ws_f = torch.empty((nb, info["workspace_elems"]), dtype=plan.dtype, device="cuda")
    ws_a = torch.empty_like(ws_f)
    s_eager = B.icr_forward(plan, xi)
    xb_eager = B.icr_adjoint(plan, y)
    s = torch.empty_like(s_eager)
    xb = torch.empty_like(xb_eager)
    B.icr_forward(plan, xi, s, ws_f)   # warm-up outside the capture
    B.icr_adjoint(plan, y, xb, ws_a)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.icr_forward(plan, xi, s, ws_f)
        B.icr_adjoint(plan, y, xb, ws_a)
    for rep in range(3):
        s.fill_(float("nan"))
        xb.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(s, s_eager), rep
        assert torch.equal(xb, xb_eager), rep
        # eager work between replays, on the same buffers
        B.icr_forward(plan, xi * 2, s, ws_f)
        torch.cuda.synchronize()
        assert not torch.equal(s, s_eager) or bool((xi == 0).all())
