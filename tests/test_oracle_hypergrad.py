"""Pins of the oracle's hyperparameter gradients.

Every derivative is checked against central finite differences of a function that
is pinned elsewhere (the kernels against their Bessel and Gaussian forms, the
Cholesky factor against LAPACK, the conditioning matrices and the sweep against
closed forms and covariances), so a dropped term, a wrong sign or a transposed
operand in the derivative formulas shows up as a mismatch.
"""

import math

import numpy as np
import pytest

from oracle import icr_oracle as O


def _fd(f, x, h):
    return (f(x + h) - f(x - h)) / (2.0 * h)


@pytest.mark.parametrize("kind", O.KERNELS)
def test_kernel_length_derivative_matches_finite_differences(kind):
    r = np.linspace(0.0, 1.5, 61)
    ell, sigma = 0.3, 1.4
    fd = _fd(lambda v: O.kernel_values(kind, r, sigma, v), ell, 1e-6)
    np.testing.assert_allclose(O.kernel_length_derivative(kind, r, sigma, ell), fd, rtol=1e-7, atol=1e-10)


def test_cholesky_derivative_matches_finite_differences_of_lapack():
    rng = np.random.default_rng(3)
    for n in (1, 3, 8, 27):
        b = rng.standard_normal((n, n))
        a = b @ b.T + n * np.eye(n)
        e = rng.standard_normal((n, n))
        da = e + e.T
        fd = _fd(lambda t: np.linalg.cholesky(a + t * da), 0.0, 1e-6)
        np.testing.assert_allclose(O.cholesky_derivative(np.linalg.cholesky(a), da), fd, rtol=1e-6, atol=1e-8)


def test_cholesky_derivative_refuses_a_clamped_column():
    low = np.array([[1.0, 0.0], [0.5, 0.0]])
    with pytest.raises(O.NotPositiveDefinite):
        O.cholesky_derivative(low, np.eye(2))


@pytest.mark.parametrize("ndim,kind,dl", [(1, "matern32", 0.11), (2, "sqexp", 0.3), (3, "matern52", 0.3),
                                          (2, "matern12", 0.11)])
def test_conditioning_matrix_derivatives_match_finite_differences(ndim, kind, dl):
    """Well-conditioned windows, so that the central differences resolve the derivative."""
    wins = O.window_offsets(ndim) * dl
    kids = (O.child_offsets(ndim) - 0.5) * dl / 2
    ell, h = 0.4, 1e-6
    tau = O.pivot_threshold(ndim, 1.0)

    def mats(v):
        r, s, _ = O.conditional_matrices(kind, 1.0, v, wins, kids, tau)
        return r, s

    r, s = mats(ell)
    dr, ds = O.conditional_matrices_length_derivative(kind, 1.0, ell, wins, kids, r, s)
    rp, sp = mats(ell + h)
    rm, sm = mats(ell - h)
    np.testing.assert_allclose(dr, (rp - rm) / (2 * h), rtol=1e-5, atol=1e-6 * np.abs(dr).max())
    np.testing.assert_allclose(ds, (sp - sm) / (2 * h), rtol=1e-5, atol=1e-6 * np.abs(ds).max())


CFGS = [
    O.ICRConfig(ndim=1, shape0=(10,), depth=3, delta0=(0.1,), kernel="matern32", length=0.3),
    O.ICRConfig(ndim=2, shape0=(6, 5), depth=2, delta0=(0.15, 0.12), kernel="matern52", scale=1.7, length=0.35),
    O.ICRConfig(ndim=3, shape0=(5, 4, 5), depth=1, delta0=(0.2, 0.25, 0.2), kernel="matern52", scale=0.6,
                length=0.5),
    O.ICRConfig(ndim=2, shape0=(5, 6), depth=2, delta0=(0.2, 1 / 6), kernel="matern32", length=0.1,
                chart="logradial2d"),
    O.ICRConfig(ndim=3, shape0=(5, 5, 4), depth=1, delta0=(0.2, 0.2, 0.25), kernel="matern32", length=0.2,
                chart="logradial_cyl3d", chart_params=(0.1, math.log(10.0), math.pi / 2, 1.0)),
]


@pytest.mark.parametrize("cfg", CFGS, ids=["1d", "2d", "3d", "chart2d", "chart3d"])
def test_hyper_grad_matches_finite_differences_of_the_sample(cfg):
    """dE/dtheta of E = <ybar, L(theta) xi>, each model rebuilt at theta +- h."""
    m = O.build(cfg)
    rng = np.random.default_rng(21)
    xi = rng.standard_normal((2, m.n_xi))
    y = rng.standard_normal((2, m.out_size))
    g = O.hyper_grad(m, xi, y)

    def energy(**over):
        kw = dict(cfg.__dict__)
        kw.update(over)
        return np.sum(y * O.build(O.ICRConfig(**kw)).forward(xi), axis=-1)

    hs = 1e-6 * cfg.scale
    fd_sigma = (energy(scale=cfg.scale + hs) - energy(scale=cfg.scale - hs)) / (2 * hs)
    hl = 1e-6 * cfg.length
    fd_len = (energy(length=cfg.length + hl) - energy(length=cfg.length - hl)) / (2 * hl)
    np.testing.assert_allclose(g[:, 0], fd_sigma, rtol=1e-6)
    np.testing.assert_allclose(g[:, 1], fd_len, rtol=2e-5, atol=1e-6 * np.abs(fd_len).max())
