"""The Python binding enforces buffer sizes before calling the C ABI, which sees only
pointers: a weight vector, output, input or workspace of the wrong size is refused with
ValueError and nothing is launched. Runs on the CPU: host tensors stand in for device
tensors (the `device` fixture makes them pass the device check), and a host tensor of
the right shape is refused without it."""

import pytest
import torch

from paper_2402_16683_amd import icr as B


class FakePlan:
    """Just what the binding's checks read: sizes and element types (no device plan)."""

    def __init__(self):
        self.handle = None
        self.info = dict(n_xi=100, n_out=64, workspace_elems=36, metric_workspace_elems=100, depth=1,
                         level_offsets=[0, 36, 100], hypergrad_workspace_elems=10)

    dtype = torch.float32
    acc_dtype = torch.float32


P = FakePlan()


@pytest.fixture
def device(monkeypatch):
    monkeypatch.setattr(torch.Tensor, "is_cuda", property(lambda self: True))


def _t(*shape, dtype=torch.float32):
    return torch.zeros(shape, dtype=dtype)


def test_host_tensors_are_refused():
    with pytest.raises(ValueError, match="device"):
        B.icr_forward(P, _t(2, 100), s=_t(2, 64), workspace=_t(2, 36))


def test_forward_and_adjoint_sizes(device):
    with pytest.raises(ValueError, match="batch"):
        B.icr_forward(P, _t(2, 99))
    with pytest.raises(ValueError, match="shape"):
        B.icr_forward(P, _t(2, 100), s=_t(1, 64), workspace=_t(2, 36))
    with pytest.raises(ValueError, match="shape"):
        B.icr_adjoint(P, _t(3, 64), xi_bar=_t(3, 64), workspace=_t(3, 36))
    with pytest.raises(ValueError, match="shape"):
        B.icr_adjoint(P, _t(64), xi_bar=_t(1, 100), workspace=_t(36))


def test_workspace_too_small_is_refused(device):
    with pytest.raises(ValueError, match="at least 72"):
        B.icr_forward(P, _t(2, 100), s=_t(2, 64), workspace=_t(2, 35))
    with pytest.raises(ValueError, match="at least 72"):
        B.icr_adjoint(P, _t(2, 64), xi_bar=_t(2, 100), workspace=_t(71))
    with pytest.raises(ValueError, match="at least 200"):
        B.icr_metric_apply(P, _t(64), _t(2, 100), out=_t(2, 100), workspace=_t(199))
    with pytest.raises(ValueError, match="at least 200"):
        B.icr_weighted_adjoint(P, _t(64), _t(2, 64), out=_t(2, 100), workspace=_t(2, 99))


@pytest.mark.parametrize("shape", [(63,), (65,), (1, 64), (3, 64), (2, 63)])
def test_weights_of_the_wrong_size_are_refused(device, shape):
    # (n_out,) is shared by all samples; (batch, n_out) is per sample; anything else would
    # make the kernels read past the weights
    with pytest.raises(ValueError, match="w must have"):
        B._weights(P, _t(*shape), batch=2)


def test_weight_strides(device):
    assert B._weights(P, _t(64), batch=2) == 0
    assert B._weights(P, _t(2, 64), batch=2) == 64
    assert B._weights(P, _t(1, 64), batch=1) == 64


def test_metric_cg_mgvi_shapes(device):
    with pytest.raises(ValueError, match="w must have"):
        B.icr_metric_apply(P, _t(1, 64), _t(2, 100))
    with pytest.raises(ValueError, match="w must have"):
        B.icr_cg_metric(P, _t(60), _t(1, 100), 5)
    with pytest.raises(ValueError, match="w must have"):
        B.icr_weighted_adjoint(P, _t(3, 64), _t(2, 64))
    with pytest.raises(ValueError, match="shape"):
        B.icr_weighted_adjoint(P, _t(64), _t(2, 64), add=_t(2, 99))
    with pytest.raises(ValueError, match="shape"):
        B.icr_mgvi_newton_step(P, _t(64), _t(1, 100), _t(2, 100), 3)


def test_level_views_are_checked(device):
    with pytest.raises(ValueError, match="level must be"):
        B.icr_forward_level(P, 1, _t(1, 36), _t(1, 64), _t(1, 64))
    with pytest.raises(ValueError, match="xi_fine"):
        B.icr_forward_level(P, 0, _t(1, 36), _t(1, 63), _t(1, 64))
    with pytest.raises(ValueError, match="s_coarse"):
        B.icr_forward_level(P, 0, _t(1, 35), _t(1, 64), _t(1, 64))
    with pytest.raises(ValueError, match="s_bar_coarse"):
        B.icr_adjoint_level(P, 0, _t(2, 64), _t(2, 64), _t(1, 36))
    with pytest.raises(ValueError, match="y_fine"):
        B.icr_adjoint_level(P, -1, _t(2, 35), _t(2, 36), None)
