"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
function include/icr.h declares, the Python structs match the C layout, and
argument errors are reported before any device work."""

import ctypes
import os
import subprocess
import sys

import pytest

from paper_2402_16683_amd import icr as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    lib = B.load_library()
    names = B.declared_functions()
    assert {"icr_build_matrices", "icr_forward", "icr_adjoint", "icr_metric_apply"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert set(names) <= exported
    assert B.icr_version() >= 100


def test_struct_layout_matches_the_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "icr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(icr_config), offsetof(icr_config, distances0),
         offsetof(icr_config, chart_params), sizeof(icr_plan_info), offsetof(icr_plan_info, n_xi));
  printf("%zu %zu %zu\n", offsetof(icr_plan_info, level_offsets), offsetof(icr_plan_info, device_bytes),
         offsetof(icr_plan_info, level_sets));
  return 0;
}''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(B.IcrConfig), B.IcrConfig.distances0.offset,
                    B.IcrConfig.chart_params.offset, ctypes.sizeof(B.IcrPlanInfo), B.IcrPlanInfo.n_xi.offset,
                    B.IcrPlanInfo.level_offsets.offset, B.IcrPlanInfo.device_bytes.offset,
                    B.IcrPlanInfo.level_sets.offset]


def _build_status(**over):
    params = dict(ndim=2, shape0=(6, 6), depth=2, distances0=(0.1, 0.1), kernel="matern32", length=0.2)
    params.update(over)
    cfg = B.make_config(**params)
    out = ctypes.c_void_p(123)
    st = B.load_library().icr_build_matrices(ctypes.byref(cfg), None, ctypes.byref(out))
    return st, out.value, B.icr_last_error()


@pytest.mark.parametrize("over,needle", [
    (dict(ndim=4, shape0=(6,) * 4, distances0=(0.1,) * 4), "ndim"),
    (dict(depth=-1), "depth"),
    (dict(depth=16), "depth"),
    (dict(shape0=(2, 6)), "fewer than 3"),
    (dict(shape0=(6, 0)), "shape0"),
    (dict(distances0=(0.1, -1.0)), "distances0"),
    (dict(length=0.0), "scale and length"),
    (dict(kernel=7), "kernel"),
    (dict(chart=5), "chart"),
    (dict(ndim=3, shape0=(5, 5, 5), distances0=(0.1,) * 3, chart="logradial2d"), "log-radial"),
    (dict(chart="logradial_cyl3d", chart_params=(0.1, 2.3, 1.5, 1.0)), "cylinder chart needs ndim == 3"),
    (dict(ndim=3, shape0=(5, 5, 5), distances0=(0.1,) * 3, chart="logradial_cyl3d",
          chart_params=(0.1, 2.3, 1.5, 0.0)), "height scale"),
    (dict(precision=9), "precision"),
])
def test_invalid_configs_are_rejected_before_any_device_work(over, needle):
    st, plan, msg = _build_status(**over)
    assert st == 1 and plan is None and needle in msg


def test_oversized_level0_is_unsupported():
    st, plan, msg = _build_status(ndim=2, shape0=(65, 65), depth=0)
    assert st == 5 and plan is None and "4096" in msg


def test_hot_calls_reject_a_null_plan_and_negative_batch():
    lib = B.load_library()
    assert lib.icr_forward(None, 1, None, None, None, None) == 1
    assert "plan" in B.icr_last_error()
    assert lib.icr_adjoint(None, 1, None, None, None, None) == 1
    assert lib.icr_metric_apply(None, 1, None, 0, None, None, None, None) == 1
    assert lib.icr_hyper_grad(None, 1, None, None, None, None, None, None, None, None) == 1
    assert lib.icr_plan_destroy(None) == 0 and B.icr_last_error() == ""
    info = B.IcrPlanInfo()
    assert lib.icr_plan_get_info(None, ctypes.byref(info)) == 1


def test_a_missing_library_fails_loudly():
    """No CPU fallback: without libicr.so the binding raises instead of computing."""
    code = ("from paper_2402_16683_amd import icr\n"
            "try:\n"
            "    icr.load_library('/nonexistent/libicr.so')\n"
            "except RuntimeError as e:\n"
            "    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0 and "raised" in r.stdout and "missing" in r.stdout


def test_hot_calls_refuse_host_tensors():
    import torch
    plan = B.Plan.__new__(B.Plan)  # no device plan is needed to reach the argument check
    plan.handle, plan.cfg = None, B.make_config(1, (12,), 1, (0.1,), precision="f32")
    plan.info = {"n_xi": 32, "n_out": 20}
    with pytest.raises(ValueError):
        B.icr_forward(plan, torch.zeros(32))
