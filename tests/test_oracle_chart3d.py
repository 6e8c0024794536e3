"""Pins of the oracle's three-dimensional chart: the log-radial cylinder.

Index point (u, v, w) sits at (r cos(a v), r sin(a v), h w) with r = r0 exp(g u).
Expected values come from the chart's closed form (known points), the law of
cosines for distances between charted points, GP conditioning on the charted
positions (block covariances exact at depth one), the symmetries of the chart
(rotation about and translation along its axis) and the stationary model that the
per-pixel path must reduce to under an identity chart.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import icr_oracle as O
from tests.test_oracle_pins import _joint_dense, _positions_nd

PARAMS = (0.1, math.log(10.0), math.pi / 2, 1.0)


def _cosine_law_distance(a, b, params):
    """Distances between charted index points from the law of cosines in the plane
    of the radial and angular axes plus the height difference."""
    r0, g, ang, h = params
    ra = r0 * np.exp(g * a[:, None, 0])
    rb = r0 * np.exp(g * b[None, :, 0])
    dth = ang * (a[:, None, 1] - b[None, :, 1])
    dz = h * (a[:, None, 2] - b[None, :, 2])
    sq = ra ** 2 + rb ** 2 - 2.0 * ra * rb * np.cos(dth) + dz ** 2
    return np.sqrt(np.maximum(sq, 0.0))


def test_cylinder_chart_maps_known_points():
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5, 0.5, 0.25]])
    p = O.logradial_cylinder_chart(pts, (0.1, math.log(10.0), math.pi / 2, 2.0))
    np.testing.assert_allclose(p[0], [0.1, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(p[1], [0.0, 1.0, 2.0], atol=1e-15)
    r = 0.1 * math.sqrt(10.0)
    np.testing.assert_allclose(p[2], [r / math.sqrt(2), r / math.sqrt(2), 0.5], atol=1e-15)


def test_cylinder_chart_distances_follow_the_law_of_cosines():
    rng = np.random.default_rng(4)
    a = rng.random((40, 3))
    b = rng.random((30, 3))
    ref = _cosine_law_distance(a, b, PARAMS)
    got = O.pairwise_distance(O.logradial_cylinder_chart(a, PARAMS), O.logradial_cylinder_chart(b, PARAMS))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_cylinder_chart_needs_four_parameters_and_three_axes():
    with pytest.raises(ValueError):
        O.logradial_cylinder_chart(np.zeros((1, 3)), PARAMS[:3])
    with pytest.raises(ValueError):
        O.build(O.ICRConfig(ndim=2, shape0=(5, 5), depth=1, delta0=(0.2, 0.2), chart="logradial_cyl3d",
                            chart_params=PARAMS))


def _model(shape0, depth, kind="matern32", length=0.05, params=PARAMS, **kw):
    return O.build(O.ICRConfig(ndim=3, shape0=tuple(shape0), depth=depth,
                               delta0=tuple(1.0 / n for n in shape0), kernel=kind, length=length,
                               chart="logradial_cyl3d", chart_params=params, **kw))


def test_cylinder_matrices_depend_only_on_the_radial_index():
    """Distances between charted points depend on (u1, u2, v1 - v2, w1 - w2) only, so
    every level's per-pixel matrices are constant along the angular and height axes:
    one set per radial shell describes a level exactly."""
    m = _model((7, 6, 5), 2)
    for r_mat, s_mat in zip(m.r_mats, m.sqrt_ds):
        scale_r = np.max(np.abs(r_mat))
        np.testing.assert_allclose(r_mat, np.broadcast_to(r_mat[:, :1, :1], r_mat.shape), atol=1e-10 * scale_r)
        np.testing.assert_allclose(s_mat, np.broadcast_to(s_mat[:, :1, :1], s_mat.shape), atol=1e-12)
        # and they do change from shell to shell
        assert np.max(np.abs(r_mat[0, 0, 0] - r_mat[-1, 0, 0])) > 1e-3


def test_cylinder_depth_one_block_covariances_are_exact():
    """Cov(fine block) = K_ff and Cov(fine block, coarse window) = K_fc with the
    kernel of law-of-cosines distances between the charted pixel positions."""
    n0, sigma, length = 5, 1.2, 0.3
    m = _model((n0,) * 3, 1, kind="matern52", length=length, scale=sigma)
    l0, l1 = _joint_dense(m)
    pos0, pos1 = _positions_nd((n0,) * 3, 1, (1.0 / n0,) * 3)
    k = lambda a, b: O.kernel_values("matern52", _cosine_law_distance(a, b, PARAMS), sigma, length)
    c11 = l1 @ l1.T
    c10 = l1 @ l0.T
    np.testing.assert_allclose(np.diag(c11), sigma ** 2, atol=1e-12)
    np.testing.assert_allclose(l0 @ l0.T, k(pos0, pos0), atol=1e-12)
    n1 = 2 * (n0 - 2)
    fine_idx = np.arange(n1 ** 3).reshape((n1,) * 3)
    coarse_idx = np.arange(n0 ** 3).reshape((n0,) * 3)
    for c in itertools.product(range(1, n0 - 1), repeat=3):
        blk = fine_idx[tuple(slice(2 * (ci - 1), 2 * ci) for ci in c)].ravel()
        win = coarse_idx[tuple(slice(ci - 1, ci + 2) for ci in c)].ravel()
        np.testing.assert_allclose(c11[np.ix_(blk, blk)], k(pos1[blk], pos1[blk]), atol=1e-12)
        np.testing.assert_allclose(c10[np.ix_(blk, win)], k(pos1[blk], pos0[win]), atol=1e-12)


def test_cylinder_matrices_use_the_positions_of_the_refined_pixels():
    """At every level a coarse pixel's window is the charted positions of its 27
    neighbours and its children those of the 8 fine pixels it spawns."""
    shape0, depth, length = (5, 6, 5), 2, 0.2
    m = _model(shape0, depth, length=length)
    pos = _positions_nd(shape0, depth, tuple(1.0 / n for n in shape0))
    tau = O.pivot_threshold(3, 1.0)
    for l in range(depth):
        n = m.shapes[l]
        nf = m.shapes[l + 1]
        grid = pos[l].reshape(n + (3,))
        fine = pos[l + 1].reshape(nf + (3,))
        for c in [(1, 1, 1), (n[0] - 2, 1, n[2] - 2), (n[0] // 2, n[1] - 2, 1)]:
            win = np.array([grid[c[0] + a, c[1] + b, c[2] + e]
                            for a, b, e in itertools.product((-1, 0, 1), repeat=3)])
            kid = np.array([fine[2 * (c[0] - 1) + a, 2 * (c[1] - 1) + b, 2 * (c[2] - 1) + e]
                            for a, b, e in itertools.product((0, 1), repeat=3)])
            kcc = O.kernel_values("matern32", _cosine_law_distance(win, win, PARAMS), 1.0, length)
            kfc = O.kernel_values("matern32", _cosine_law_distance(kid, win, PARAMS), 1.0, length)
            kff = O.kernel_values("matern32", _cosine_law_distance(kid, kid, PARAMS), 1.0, length)
            r_ref = np.linalg.solve(kcc, kfc.T).T
            d_ref = kff - r_ref @ kfc.T
            got_r = m.r_mats[l][c[0] - 1, c[1] - 1, c[2] - 1]
            got_s = m.sqrt_ds[l][c[0] - 1, c[1] - 1, c[2] - 1]
            np.testing.assert_allclose(got_r, r_ref, atol=1e-9)
            np.testing.assert_allclose(got_s @ got_s.T, d_ref, atol=1e-12)
            assert np.all(np.triu(got_s, 1) == 0.0)


def test_cylinder_per_pixel_path_with_an_identity_chart_equals_the_stationary_path(monkeypatch):
    """With the chart replaced by the identity the 3-D per-pixel build and sweep
    reduce to the stationary ones (pins the 3-D per-pixel indexing)."""
    base = dict(ndim=3, shape0=(5, 6, 4), depth=2, delta0=(0.12, 0.1, 0.15), kernel="matern52", length=0.3)
    stat = O.build(O.ICRConfig(**base))
    monkeypatch.setattr(O, "_positions", lambda c, pts: pts)
    chart = O.build(O.ICRConfig(chart="logradial_cyl3d", chart_params=PARAMS, **base))
    for l in range(2):
        np.testing.assert_allclose(chart.r_mats[l], np.broadcast_to(stat.r_mats[l], chart.r_mats[l].shape),
                                   atol=1e-9)
    xi = np.random.default_rng(2).standard_normal(stat.n_xi)
    np.testing.assert_allclose(chart.forward(xi), stat.forward(xi), atol=1e-10)
    y = np.random.default_rng(3).standard_normal(stat.out_size)
    np.testing.assert_allclose(chart.adjoint(y), stat.adjoint(y), atol=1e-10)


def test_cylinder_adjoint_is_the_transpose():
    m = _model((5, 5, 4), 1, length=0.1)
    np.testing.assert_allclose(m.dense_adjoint(), m.dense().T, atol=1e-13)
    rng = np.random.default_rng(12)
    xi = rng.standard_normal((2, m.n_xi))
    y = rng.standard_normal((2, m.out_size))
    np.testing.assert_allclose(np.sum(m.forward(xi) * y, -1), np.sum(xi * m.adjoint(y), -1), rtol=1e-12)
