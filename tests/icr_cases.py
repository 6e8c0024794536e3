"""Workload cases for the tests and helpers that hand the same parameters and the
same seeded inputs to the FP64 oracle and to the HIP library."""

from __future__ import annotations

import math

import numpy as np

import workloads as W
from oracle import icr_oracle as O

# Tolerances on rel-RMS = ||x - x_oracle|| / ||x_oracle|| per level, and on
# max|x - x_oracle| / max|x_oracle|. FP32 and BF16 storage: the stated accuracy
# bars. FP64: both sides build R in FP64 independently, and R = K_fc K_cc^-1 is
# only determined to about cond(K_cc) eps64 (cond up to ~1e5 at the tested
# levels), so the sweeps can differ by ~1e-11 relative.
TOL = {"f64": (1e-10, 1e-9), "f32": (1e-5, 1e-4), "bf16": (1e-2, 4e-2)}


def case(ndim, shape0, depth, delta0, kernel, length, precision="f32", scale=1.0, chart="regular",
         chart_params=(0.1, math.log(10.0), 0.5 * math.pi), batch=1, clamp=True, name=None):
    return dict(ndim=ndim, shape0=tuple(shape0), depth=depth, delta0=tuple(delta0), kernel=kernel,
                length=length, precision=precision, scale=scale, chart=chart,
                chart_params=tuple(chart_params), batch=batch, clamp=clamp,
                name=name or f"{ndim}d_{kernel}_{'x'.join(map(str, shape0))}_L{depth}_{precision}")


def from_workload(key, **over):
    w = dict(W.WORKLOADS[key])
    w.update(over)
    return case(w["ndim"], w["shape0"], w["depth"], w["delta0"], w["kernel"], w["length"],
                precision=w["precision"], scale=w["scale"], chart=w["chart"],
                chart_params=w.get("chart_params", (0.1, math.log(10.0), 0.5 * math.pi)),
                batch=w["batch"], name=over.get("name", key))


def oracle_model(c) -> O.ICROracle:
    return O.build(O.ICRConfig(ndim=c["ndim"], shape0=c["shape0"], depth=c["depth"],
                               delta0=c["delta0"], kernel=c["kernel"], scale=c["scale"],
                               length=c["length"], chart=c["chart"], chart_params=c["chart_params"],
                               clamp=c["clamp"]))


def gpu_plan(c, precision=None):
    from paper_2402_16683_amd import icr as B
    cfg = B.make_config(c["ndim"], c["shape0"], c["depth"], c["delta0"], kernel=c["kernel"],
                        scale=c["scale"], length=c["length"], chart=c["chart"],
                        chart_params=c["chart_params"], precision=precision or c["precision"],
                        clamp=c["clamp"])
    return B.icr_build_matrices(cfg)


def chart_positions(c, pts: np.ndarray) -> np.ndarray:
    """Physical positions of index-space points under the case's chart (oracle maps)."""
    if c["chart"] == "regular":
        return pts
    if c["chart"] == "logradial2d":
        return O.logradial_chart(pts, c["chart_params"])
    if c["chart"] == "logradial_cyl3d":
        return O.logradial_cylinder_chart(pts, c["chart_params"])
    raise ValueError(c["chart"])


def is_shell(model) -> bool:
    """Charted models: the device keeps one matrix set per radial shell (first axis)."""
    return model.cfg.chart in ("logradial2d", "logradial_cyl3d")


def shell_sets(mat: np.ndarray, ndim: int) -> np.ndarray:
    """The per-pixel stack's sets at pixel (u, 1, ...) of every shell: (n_u, ...)."""
    return mat[(slice(None),) + (0,) * (ndim - 1)]


def rel_errors(got: np.ndarray, ref: np.ndarray):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nrm = np.linalg.norm(ref)
    rms = np.linalg.norm(got - ref) / nrm if nrm > 0 else np.linalg.norm(got)
    mx = np.max(np.abs(ref)) if ref.size else 0.0
    mxe = np.max(np.abs(got - ref)) / mx if ref.size and mx > 0 else 0.0
    return float(rms), float(mxe)


def to_numpy(t) -> np.ndarray:
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def nan_like(shape, plan):
    """A device buffer of the plan's storage type filled with NaN: an output element a
    kernel never writes stays NaN and fails the finiteness checks."""
    import torch
    return torch.full(shape, float("nan"), dtype=plan.dtype, device="cuda")


def to_device(a: np.ndarray, plan):
    """Host FP64 array -> device tensor of the plan's storage dtype."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda").to(plan.dtype)


def stored_values(a: np.ndarray, precision: str) -> np.ndarray:
    """The values a device tensor of this precision holds for host array a (FP64)."""
    if precision == "f64":
        return np.asarray(a, dtype=np.float64)
    if precision == "f32":
        return np.asarray(a, dtype=np.float32).astype(np.float64)
    return W.round_to_bf16(a).astype(np.float64)


def upload_oracle_matrices(plan, model):
    """Give the device plan the oracle's FP64 matrices (sweep-only comparisons).

    For a charted model the device holds one set per radial shell: it gets the oracle's
    set at pixel (u, 1, ...) of each shell, and the model's per-pixel sets are replaced by
    those shell sets broadcast along the other axes, so that both sides apply identical
    matrices."""
    from paper_2402_16683_amd import icr as B
    B.icr_plan_set_level0(plan, model.l00)
    d = model.cfg.ndim
    for l in range(model.cfg.depth):
        if is_shell(model):
            r_sh = shell_sets(model.r_mats[l], d)
            s_sh = shell_sets(model.sqrt_ds[l], d)
            grow = (slice(None),) + (None,) * (d - 1)
            model.r_mats[l] = np.ascontiguousarray(np.broadcast_to(r_sh[grow], model.r_mats[l].shape))
            model.sqrt_ds[l] = np.ascontiguousarray(np.broadcast_to(s_sh[grow], model.sqrt_ds[l].shape))
            r, s = r_sh, s_sh
        else:
            r = np.reshape(model.r_mats[l], (-1, 2 ** d, 3 ** d))
            s = np.reshape(model.sqrt_ds[l], (-1, 2 ** d, 2 ** d))
        B.icr_plan_set_refinement(plan, l, r, s)


def level_views(flat, offsets, upto):
    return [flat[..., offsets[l]:offsets[l + 1]] for l in range(upto)]
