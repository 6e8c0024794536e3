"""The correlated-field model and its Poisson Fisher metric M_p on the device (FP32)
against the FP64 oracle on the same inputs, at sizes from 32^2 to 4096^2.

Tolerances: the rel-RMS and relative max errors of FP32 FFTs grow like eps32 times
log2(n) with random rounding; 1e-5 rel-RMS and 1e-4 relative max (the FP32 accuracy
bar of the ICR sweeps) hold with margin at every size."""

import numpy as np
import pytest

import workloads as W
from oracle import cf_oracle as F
from tests import icr_cases as C

pytestmark = pytest.mark.gpu

# every path: one workgroup (32, 64), three passes with radix 4 (128 .. 1024; 512 ends on a
# radix-2 stage), radix 16 (2048 ends on a radix-8 stage, 4096)
SIZES = [32, 64, 128, 256, 512, 1024, 2048, 4096]
PARAMS = dict(amplitude=1.0, zero_mode=0.1, length=0.05, slope=3.0, offset_mean=2.0)


def _field(n, seed, scale=1.0):
    return (scale * W.standard_normal_f32(n * n, seed=seed)).reshape(n, n)


@pytest.mark.parametrize("n", SIZES)
def test_transform_rate_and_metric_match_the_oracle(n):
    import torch
    from paper_2402_16683_amd.cf import CorrelatedField
    cf = CorrelatedField(n, **PARAMS)
    amp = F.amplitude(n, PARAMS["amplitude"], PARAMS["zero_mode"], PARAMS["length"], PARAMS["slope"])
    np.testing.assert_allclose(cf.amplitude(), amp, rtol=1e-6)
    amp32 = cf.amplitude().astype(np.float64)
    x = _field(n, 70)
    p = _field(n, 71, 0.5)
    v = _field(n, 72)
    xd, pd, vd = (torch.from_numpy(a).cuda() for a in (x, p, v))
    y = cf.transform(xd)
    lam = cf.rate(pd)
    mv = cf.metric_apply(lam, vd)
    torch.cuda.synchronize()
    ref_y = F.transform(x.astype(np.float64))
    ref_lam = F.rate(amp32, p.astype(np.float64), PARAMS["offset_mean"])
    # the metric with the device's rate (its own FP32 rounding), so this checks M_p alone
    lam_h = lam.cpu().numpy().astype(np.float64)
    ref_mv = F.metric_apply(amp32, lam_h, v.astype(np.float64))
    for name, got, ref in (("T x", y, ref_y), ("lambda", lam, ref_lam), ("M_p v", mv, ref_mv)):
        rms, mx = C.rel_errors(got.cpu().numpy(), ref)
        print(f"[errors] cf n={n} {name}: rel-RMS {rms:.2e} rel-max {mx:.2e}")
        assert rms <= 1e-5 and mx <= 1e-4, name


def test_transform_is_its_own_inverse_and_the_metric_is_symmetric():
    import torch
    from paper_2402_16683_amd.cf import CorrelatedField
    n = 512
    cf = CorrelatedField(n, **PARAMS)
    x = torch.from_numpy(_field(n, 73)).cuda()
    back = cf.transform(cf.transform(x))
    rms, _ = C.rel_errors(back.cpu().numpy(), x.cpu().numpy())
    assert rms <= 1e-6
    lam = cf.rate(torch.from_numpy(_field(n, 74, 0.5)).cuda())
    u = torch.from_numpy(_field(n, 75)).cuda()
    v = torch.from_numpy(_field(n, 76)).cuda()
    a = float(torch.sum(u.double() * cf.metric_apply(lam, v).double()))
    b = float(torch.sum(cf.metric_apply(lam, u).double() * v.double()))
    assert abs(a - b) <= 1e-5 * (abs(a) + abs(b))


def test_invalid_sizes_are_rejected():
    from paper_2402_16683_amd import icr as B
    from paper_2402_16683_amd.cf import CorrelatedField
    for n in (16, 48, 8192):
        with pytest.raises(B.ICRError) as exc:
            CorrelatedField(n)
        assert exc.value.status == 1 and "power of two" in str(exc.value)


def test_misaligned_buffers_are_rejected():
    import torch
    from paper_2402_16683_amd import icr as B
    from paper_2402_16683_amd.cf import CorrelatedField
    n = 64
    cf = CorrelatedField(n, **PARAMS)
    x = torch.zeros(n * n + 1, dtype=torch.float32, device="cuda")[1:].reshape(n, n)  # 4 bytes off
    with pytest.raises(B.ICRError) as exc:
        cf.transform(x)
    assert exc.value.status == 1 and "aligned" in str(exc.value)
