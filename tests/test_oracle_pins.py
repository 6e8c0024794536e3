"""Pins of the FP64 oracle against closed forms, invariants and library routines.

None of these compares the oracle with itself: each expected value comes from
mathematics that fixes it independently (textbook GP conditioning, the Markov
property of the Ornstein-Uhlenbeck process, Kronecker structure of separable
kernels, LAPACK, scipy's Bessel functions) or from the level sizes printed with
the workload definitions.
"""

import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.special
import scipy.stats

from oracle import icr_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cfg(ndim, n0, depth, kernel, length, delta=None, **kw):
    delta = delta if delta is not None else 1.0 / n0
    return O.ICRConfig(ndim=ndim, shape0=(n0,) * ndim, depth=depth, delta0=(delta,) * ndim,
                       kernel=kernel, length=length, **kw)


# --------------------------------------------------------------------------- sizes

def test_level_sizes_match_the_printed_workloads():
    rows = [ln for ln in open(os.path.join(GOLDEN, "level_sizes.txt")) if not ln.startswith("#")]
    assert len(rows) == 4
    for row in rows:
        head, sizes = row.split(":")
        n0, depth = (int(v) for v in head.split())
        expect = [int(v) for v in sizes.split()]
        got = [s[0] for s in O.level_shapes((n0,), depth)]
        assert got == expect


def test_level_sizes_reject_levels_without_interior():
    with pytest.raises(ValueError):
        O.level_shapes((2, 5), 1)


# --------------------------------------------------------------------------- kernels

def _matern_bessel(nu, r, length):
    """General Matern covariance through the modified Bessel function K_nu."""
    x = math.sqrt(2 * nu) * np.maximum(r, 1e-300) / length
    return 2 ** (1 - nu) / scipy.special.gamma(nu) * x ** nu * scipy.special.kv(nu, x)


@pytest.mark.parametrize("kind,nu", [("matern12", 0.5), ("matern32", 1.5), ("matern52", 2.5)])
def test_matern_kernels_match_the_bessel_form(kind, nu):
    r = np.linspace(1e-3, 2.0, 301)
    ref = _matern_bessel(nu, r, 0.3)
    np.testing.assert_allclose(O.kernel_values(kind, r, 1.0, 0.3), ref, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(O.kernel_values(kind, r, 2.0, 0.3), 4.0 * ref, rtol=1e-12)
    assert O.kernel_values(kind, 0.0, 1.5, 0.3) == pytest.approx(2.25, abs=1e-15)


def test_squared_exponential_matches_the_normal_density():
    r = np.linspace(0, 1, 101)
    ref = scipy.stats.norm.pdf(r, scale=0.2) * math.sqrt(2 * math.pi) * 0.2
    np.testing.assert_allclose(O.kernel_values("sqexp", r, 1.0, 0.2), ref, rtol=1e-13)


# --------------------------------------------------------------------------- cholesky

def test_clamped_cholesky_equals_lapack_on_positive_definite_stacks():
    rng = np.random.default_rng(7)
    mats = []
    for n in (1, 4, 9, 27):
        b = rng.standard_normal((3, n, n))
        a = b @ np.swapaxes(b, -1, -2) + n * np.eye(n)
        low, cnt = O.clamped_cholesky(a, 1e-14)
        assert np.all(cnt == 0)
        for k in range(3):
            np.testing.assert_allclose(low[k], scipy.linalg.cholesky(a[k], lower=True),
                                       rtol=1e-12, atol=1e-12)
        mats.append(a)


def test_clamped_cholesky_clamps_rank_deficient_matrices():
    rng = np.random.default_rng(8)
    b = rng.standard_normal((8, 5))
    a = b @ b.T                      # rank 5 of 8: three pivots vanish
    low, cnt = O.clamped_cholesky(a, 1e-10)
    assert int(cnt) == 3
    assert np.allclose(np.triu(low, 1), 0.0)
    np.testing.assert_allclose(low @ low.T, a, atol=1e-9)
    with pytest.raises(O.NotPositiveDefinite):
        O.clamped_cholesky(a, 1e-10, clamp=False)


def test_clamp_boundary_is_the_pivot_threshold():
    """tau = 3^d eps k(0): a diagonal matrix (its own Schur complements) with pivots
    just above and just below tau keeps exactly the ones above."""
    for ndim, scale in ((1, 1.0), (2, 2.5), (3, 0.4)):
        tau = O.pivot_threshold(ndim, scale)
        assert tau == 3.0 ** ndim * np.finfo(np.float64).eps * scale ** 2
        piv = np.array([scale ** 2, 1.5 * tau, 0.9 * tau, 4.0 * tau, tau])
        low, cnt = O.clamped_cholesky(np.diag(piv), tau)
        assert int(cnt) == 2
        np.testing.assert_allclose(np.diag(low), [scale, np.sqrt(1.5 * tau), 0.0, 2.0 * np.sqrt(tau), 0.0],
                                   rtol=1e-15)


# --------------------------------------------------------------------------- conditioning

@pytest.mark.parametrize("h", [0.05, 0.4, 1.7])
def test_ornstein_uhlenbeck_bridge_closed_form(h):
    """Matern-1/2 in 1-D is Markov: a child only sees its two bracketing coarse pixels.

    Child at x_c - delta/4 lies 3 delta/4 right of x_{c-1} and delta/4 left of x_c;
    the bridge weights are sinh(h/4)/sinh(h) and sinh(3h/4)/sinh(h) with h = delta/l,
    and the bridge variance is (1-e^{-3h/2})(1-e^{-h/2})/(1-e^{-2h}).
    """
    length = 0.3
    delta = h * length
    wins = O.window_offsets(1) * delta
    kids = (O.child_offsets(1) - 0.5) * delta / 2
    r_mat, sqrt_d, cnt = O.conditional_matrices("matern12", 1.0, length, wins.astype(float),
                                                kids.astype(float), 1e-300)
    w_far, w_near = math.sinh(h / 4) / math.sinh(h), math.sinh(3 * h / 4) / math.sinh(h)
    np.testing.assert_allclose(r_mat, [[w_far, w_near, 0.0], [0.0, w_near, w_far]], atol=1e-13)
    v = (1 - math.exp(-1.5 * h)) * (1 - math.exp(-0.5 * h)) / (1 - math.exp(-2 * h))
    np.testing.assert_allclose(sqrt_d @ sqrt_d.T, np.diag([v, v]), atol=1e-14)
    np.testing.assert_allclose(sqrt_d, np.diag([math.sqrt(v)] * 2), atol=1e-13)
    assert int(cnt) == 0


@pytest.mark.parametrize("ndim,kind", [(1, "matern32"), (2, "sqexp"), (3, "matern52")])
def test_conditioning_residuals(ndim, kind):
    """R K_cc = K_fc, D + R K_cf = K_ff, sqrtD sqrtD^T = D, sqrtD lower with diag >= 0."""
    delta = np.array([0.11, 0.07, 0.09][:ndim])
    wins = O.window_offsets(ndim) * delta
    kids = (O.child_offsets(ndim) - 0.5) * delta / 2
    length = 0.35
    r_mat, sqrt_d, _ = O.conditional_matrices(kind, 1.0, length, wins, kids, 1e-300)
    k = lambda a, b: O.kernel_values(kind, O.pairwise_distance(a, b), 1.0, length)
    kcc, kfc, kff = k(wins, wins), k(kids, wins), k(kids, kids)
    scale = np.linalg.cond(kcc) * 1e-15
    np.testing.assert_allclose(r_mat @ kcc, kfc, atol=scale)
    d_mat = kff - r_mat @ kfc.T
    np.testing.assert_allclose(sqrt_d @ sqrt_d.T, d_mat, atol=1e-13)
    assert np.allclose(np.triu(sqrt_d, 1), 0.0) and np.all(np.diag(sqrt_d) >= 0)


def test_squared_exponential_refinement_is_a_kronecker_product():
    """SE is separable, so the 2-D window/children geometry gives R = R_x kron R_y.

    This pins the lexicographic (last axis fastest) ordering of windows and children.
    """
    dx, dy = 0.1, 0.07
    length = 0.25
    def one_d(delta):
        w = O.window_offsets(1) * delta
        c = (O.child_offsets(1) - 0.5) * delta / 2
        return O.conditional_matrices("sqexp", 1.0, length, w.astype(float), c.astype(float), 0.0)[0]
    d = np.array([dx, dy])
    r2, _, _ = O.conditional_matrices("sqexp", 1.0, length, O.window_offsets(2) * d,
                                      (O.child_offsets(2) - 0.5) * d / 2, 0.0)
    np.testing.assert_allclose(r2, np.kron(one_d(dx), one_d(dy)), atol=1e-10)
    d3 = np.array([dx, dy, 0.13])
    r3, _, _ = O.conditional_matrices("sqexp", 1.0, length, O.window_offsets(3) * d3,
                                      (O.child_offsets(3) - 0.5) * d3 / 2, 0.0)
    np.testing.assert_allclose(r3, np.kron(np.kron(one_d(dx), one_d(dy)), one_d(0.13)), atol=1e-9)


def test_level0_covariance_is_a_kronecker_product_for_squared_exponential():
    """K_00 over the C-ordered 2-D grid of a separable kernel equals K_x kron K_y."""
    m = O.build(O.ICRConfig(ndim=2, shape0=(4, 5), depth=0, delta0=(0.2, 0.3), kernel="sqexp",
                            length=0.5))
    kx = O.kernel_values("sqexp", np.abs(np.subtract.outer(np.arange(4) * 0.2, np.arange(4) * 0.2)), 1, 0.5)
    ky = O.kernel_values("sqexp", np.abs(np.subtract.outer(np.arange(5) * 0.3, np.arange(5) * 0.3)), 1, 0.5)
    np.testing.assert_allclose(m.l00 @ m.l00.T, np.kron(kx, ky), atol=1e-13)
    # the Cholesky factor of a Kronecker product is the product of the factors
    np.testing.assert_allclose(m.l00, np.kron(np.linalg.cholesky(kx), np.linalg.cholesky(ky)),
                               atol=1e-12)


# --------------------------------------------------------------------------- covariance of samples

def _positions_1d(n0, depth, delta0):
    """Pixel positions of every level from the child placement: fine pixel f is child
    f mod 2 of coarse pixel f//2 + 1, offset by (f mod 2 - 1/2) delta/2."""
    pos = [np.arange(n0) * delta0]
    delta = delta0
    for _ in range(depth):
        prev = pos[-1]
        nf = 2 * (len(prev) - 2)
        f = np.arange(nf)
        pos.append(prev[f // 2 + 1] + (f % 2 - 0.5) * delta / 2)
        delta /= 2
    return pos


def _positions_nd(shape0, depth, delta0):
    per_axis = [_positions_1d(n, depth, d) for n, d in zip(shape0, delta0)]
    out = []
    for l in range(depth + 1):
        axes = [p[l] for p in per_axis]
        grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
        out.append(grid.reshape(-1, len(shape0)))
    return out


def _joint_dense(model):
    """Dense maps xi -> s_l for every level, stacked (sum_l n_l^d x N_xi)."""
    _, levels = model.forward(np.eye(model.n_xi), return_levels=True)
    return [lv.T for lv in levels]


def test_depth_zero_samples_have_the_kernel_covariance():
    m = O.build(cfg(2, 5, 0, "matern32", 0.3))
    lmat = m.dense()
    pos = _positions_nd((5, 5), 0, (0.2, 0.2))[0]
    kref = O.kernel_values("matern32", O.pairwise_distance(pos, pos), 1.0, 0.3)
    np.testing.assert_allclose(lmat @ lmat.T, kref, atol=1e-13)


@pytest.mark.parametrize("ndim,n0,kind,length,chart", [
    (1, 9, "matern32", 0.2, None), (1, 7, "matern12", 0.5, None), (2, 5, "sqexp", 0.4, None),
    (3, 4, "matern52", 0.5, None), (2, 6, "matern32", 0.08, (0.1, math.log(10.0), math.pi / 2))])
def test_depth_one_block_covariances_are_exact(ndim, n0, kind, length, chart):
    """Cov(fine block) = K_ff, Cov(fine block, coarse window) = K_fc, Var = sigma^2.

    With a chart the kernel sees the charted positions of the pixels, so this also
    pins where the fine grid sits in index space (its origin and spacing)."""
    sigma = 1.3
    extra = dict(chart="logradial2d", chart_params=chart) if chart else {}
    m = O.build(cfg(ndim, n0, 1, kind, length, scale=sigma, **extra))
    l0, l1 = _joint_dense(m)
    pos0, pos1 = _positions_nd((n0,) * ndim, 1, (1.0 / n0,) * ndim)
    if chart:
        pos0, pos1 = O.logradial_chart(pos0, chart), O.logradial_chart(pos1, chart)
    k = lambda a, b: O.kernel_values(kind, O.pairwise_distance(a, b), sigma, length)
    c11 = l1 @ l1.T
    c10 = l1 @ l0.T
    np.testing.assert_allclose(np.diag(c11), sigma ** 2, atol=1e-12)
    np.testing.assert_allclose(np.diag(l0 @ l0.T), sigma ** 2, atol=1e-12)
    n1 = 2 * (n0 - 2)
    fine_idx = np.arange(n1 ** ndim).reshape((n1,) * ndim)
    coarse_idx = np.arange(n0 ** ndim).reshape((n0,) * ndim)
    for c in itertools.product(range(1, n0 - 1), repeat=ndim):
        blk = fine_idx[tuple(slice(2 * (ci - 1), 2 * ci) for ci in c)].ravel()
        win = coarse_idx[tuple(slice(ci - 1, ci + 2) for ci in c)].ravel()
        np.testing.assert_allclose(c11[np.ix_(blk, blk)], k(pos1[blk], pos1[blk]), atol=1e-12)
        np.testing.assert_allclose(c10[np.ix_(blk, win)], k(pos1[blk], pos0[win]), atol=1e-12)
    np.testing.assert_allclose(l0 @ l0.T, k(pos0, pos0), atol=1e-12)


def test_markov_process_cross_covariance_is_exact_everywhere():
    """For Matern-1/2 in 1-D every fine pixel's conditional mean given all coarse
    pixels depends only on its bracketing pair, so Cov(s_1, s_0) = K for all pairs;
    Matern-3/2 is not Markov and misses it (discriminates the placement)."""
    n0 = 10
    for kind, exact in (("matern12", True), ("matern32", False)):
        m = O.build(cfg(1, n0, 1, kind, 0.3))
        l0, l1 = _joint_dense(m)
        pos0, pos1 = _positions_1d(n0, 1, 1.0 / n0)
        kref = O.kernel_values(kind, np.abs(np.subtract.outer(pos1, pos0)), 1.0, 0.3)
        err = np.max(np.abs(l1 @ l0.T - kref))
        assert (err < 1e-13) if exact else (err > 1e-4)


@pytest.mark.parametrize("ndim,n0,depth,kind,length", [
    (1, 12, 3, "matern32", 0.2), (2, 6, 2, "sqexp", 0.3), (3, 5, 1, "matern52", 0.4)])
def test_icr_covariance_approximates_the_kernel(ndim, n0, depth, kind, length):
    """ICR is an approximation: L L^T is close to, not equal to, K on the final grid."""
    m = O.build(cfg(ndim, n0, depth, kind, length))
    lmat = m.dense()
    pos = _positions_nd((n0,) * ndim, depth, (1.0 / n0,) * ndim)[-1]
    kref = O.kernel_values(kind, O.pairwise_distance(pos, pos), 1.0, length)
    rel = np.linalg.norm(lmat @ lmat.T - kref) / np.linalg.norm(kref)
    assert rel < 0.1


def test_separable_sweep_equals_the_outer_product_of_one_dimensional_sweeps():
    """With a separable kernel, a separable level-0 excitation and zero fresh
    excitations, the 2-D and 3-D sweeps are outer products of 1-D sweeps. This pins
    the multi-dimensional indexing of the sweep to the 1-D one."""
    length, depth = 0.3, 2
    shapes0, deltas = (6, 7, 5), (0.15, 0.11, 0.13)
    rng = np.random.default_rng(3)
    ones = []
    seeds = []
    for n, d in zip(shapes0, deltas):
        m1 = O.build(O.ICRConfig(ndim=1, shape0=(n,), depth=depth, delta0=(d,), kernel="sqexp",
                                 length=length))
        a = rng.standard_normal(n)
        xi = np.zeros(m1.n_xi)
        xi[:n] = a
        ones.append(m1.forward(xi))
        seeds.append(a)
    for nd in (2, 3):
        m = O.build(O.ICRConfig(ndim=nd, shape0=shapes0[:nd], depth=depth, delta0=deltas[:nd],
                                kernel="sqexp", length=length))
        xi = np.zeros(m.n_xi)
        x0 = seeds[0]
        for a in seeds[1:nd]:
            x0 = np.kron(x0, a)
        xi[: x0.size] = x0
        ref = ones[0]
        for v in ones[1:nd]:
            ref = np.kron(ref, v)
        np.testing.assert_allclose(m.forward(xi), ref, atol=1e-10)


# --------------------------------------------------------------------------- adjoint / metric

MODELS = [
    cfg(1, 12, 4, "matern32", 0.2),
    cfg(2, 6, 2, "sqexp", 0.3),
    cfg(3, 5, 2, "matern52", 0.4),
    O.ICRConfig(ndim=2, shape0=(6, 6), depth=2, delta0=(1 / 6, 1 / 6), kernel="matern32",
                length=0.05, chart="logradial2d"),
]


@pytest.mark.parametrize("c", MODELS, ids=["1d", "2d", "3d", "chart"])
def test_adjoint_dot_product_identity(c):
    m = O.build(c)
    rng = np.random.default_rng(11)
    xi = rng.standard_normal((3, m.n_xi))
    y = rng.standard_normal((3, m.out_size))
    lhs = np.sum(m.forward(xi) * y, axis=-1)
    rhs = np.sum(xi * m.adjoint(y), axis=-1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("c", MODELS[:2] + MODELS[3:], ids=["1d", "2d", "chart"])
def test_dense_adjoint_is_the_transpose(c):
    m = O.build(c)
    np.testing.assert_allclose(m.dense_adjoint(), m.dense().T, atol=1e-13)


def test_forward_is_linear_and_batched():
    m = O.build(MODELS[1])
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, m.n_xi))
    np.testing.assert_allclose(m.forward(2.0 * a - 3.0 * b), 2.0 * m.forward(a) - 3.0 * m.forward(b),
                               atol=1e-12)
    both = m.forward(np.stack([a, b]))
    np.testing.assert_allclose(both[1], m.forward(b), atol=1e-15)


def test_metric_is_symmetric_bounded_below_and_solvable_by_cg():
    m = O.build(MODELS[1])
    rng = np.random.default_rng(9)
    w = (rng.random(m.out_size) < 0.7) / 0.1 ** 2
    mat = np.stack([m.metric(w, e) for e in np.eye(m.n_xi)], axis=1)
    np.testing.assert_allclose(mat, mat.T, atol=1e-10)
    assert np.min(np.linalg.eigvalsh(0.5 * (mat + mat.T))) >= 1.0 - 1e-10
    lmat = m.dense()
    np.testing.assert_allclose(mat, lmat.T @ (w[:, None] * lmat) + np.eye(m.n_xi), atol=1e-10)
    b = rng.standard_normal(m.n_xi)
    x = scipy.sparse.linalg.cg(scipy.sparse.linalg.LinearOperator(
        (m.n_xi, m.n_xi), matvec=lambda v: m.metric(w, v)), b, rtol=1e-12, maxiter=2000)[0]
    np.testing.assert_allclose(x, np.linalg.solve(mat, b), rtol=1e-8, atol=1e-9)


# --------------------------------------------------------------------------- chart

def test_logradial_chart_maps_known_points():
    p = O.logradial_chart(np.array([[0.0, 0.0], [1.0, 1.0], [0.5, 0.5]]),
                          (0.1, math.log(10.0), math.pi / 2))
    np.testing.assert_allclose(p[0], [0.1, 0.0], atol=1e-15)
    np.testing.assert_allclose(p[1], [0.0, 1.0], atol=1e-15)
    r = 0.1 * math.sqrt(10.0)
    np.testing.assert_allclose(p[2], [r / math.sqrt(2), r / math.sqrt(2)], atol=1e-15)


def test_chart_matrices_do_not_depend_on_the_angle():
    """The log-radial chart is a rotation along its angular axis, so per-pixel
    matrices only depend on the radial index."""
    m = O.build(O.ICRConfig(ndim=2, shape0=(8, 8), depth=2, delta0=(1 / 8, 1 / 8),
                            kernel="matern32", length=0.05, chart="logradial2d"))
    for r_mat, s_mat in zip(m.r_mats, m.sqrt_ds):
        np.testing.assert_allclose(r_mat, np.broadcast_to(r_mat[:, :1], r_mat.shape), atol=1e-10)
        np.testing.assert_allclose(s_mat, np.broadcast_to(s_mat[:, :1], s_mat.shape), atol=1e-12)


def test_chart_matrices_use_the_positions_of_the_refined_pixels():
    """At every level, a coarse pixel's window is the charted positions of its 3^d
    neighbours and its children are the charted positions of the fine pixels it
    spawns (fine f is a child of coarse f//2 + 1), as placed level by level."""
    params = (0.1, math.log(10.0), math.pi / 2)
    n0, depth = 5, 3
    m = O.build(O.ICRConfig(ndim=2, shape0=(n0, n0), depth=depth, delta0=(1 / n0, 1 / n0),
                            kernel="matern32", length=0.05, chart="logradial2d",
                            chart_params=params))
    pos = _positions_nd((n0, n0), depth, (1 / n0, 1 / n0))
    tau = O.pivot_threshold(2, 1.0)
    for l in range(depth):
        n = m.shapes[l][0]
        nf = m.shapes[l + 1][0]
        grid = pos[l].reshape(n, n, 2)
        fine = pos[l + 1].reshape(nf, nf, 2)
        for c in [(1, 1), (n - 2, 1), (1, n - 2), (n // 2, n // 2 - 1), (n - 2, n - 2)]:
            win = np.array([grid[c[0] + a, c[1] + b] for a in (-1, 0, 1) for b in (-1, 0, 1)])
            kid = np.array([fine[2 * (c[0] - 1) + a, 2 * (c[1] - 1) + b] for a in (0, 1) for b in (0, 1)])
            r_ref, s_ref, _ = O.conditional_matrices("matern32", 1.0, 0.05, O.logradial_chart(win, params),
                                                     O.logradial_chart(kid, params), tau)
            np.testing.assert_allclose(m.r_mats[l][c[0] - 1, c[1] - 1], r_ref, atol=1e-9)
            np.testing.assert_allclose(m.sqrt_ds[l][c[0] - 1, c[1] - 1], s_ref, atol=1e-11)


def test_per_pixel_path_with_an_identity_chart_equals_the_stationary_path(monkeypatch):
    """The charted (per-pixel matrix) build and sweep reduce to the stationary ones
    when the chart is the identity: pins the per-pixel geometry and indexing."""
    base = dict(ndim=2, shape0=(6, 7), depth=2, delta0=(0.12, 0.1), kernel="matern52", length=0.3)
    stat = O.build(O.ICRConfig(**base))
    monkeypatch.setattr(O, "_positions", lambda c, pts: pts)
    chart = O.build(O.ICRConfig(chart="logradial2d", **base))
    for l in range(2):
        np.testing.assert_allclose(chart.r_mats[l], np.broadcast_to(stat.r_mats[l], chart.r_mats[l].shape),
                                   atol=1e-9)
    xi = np.random.default_rng(2).standard_normal(stat.n_xi)
    np.testing.assert_allclose(chart.forward(xi), stat.forward(xi), atol=1e-10)
    y = np.random.default_rng(3).standard_normal(stat.out_size)
    np.testing.assert_allclose(chart.adjoint(y), stat.adjoint(y), atol=1e-10)


def test_unbuildable_configurations_raise():
    with pytest.raises(O.NotPositiveDefinite):
        # SE with a long length scale: K_00 and D are numerically indefinite
        O.build(cfg(2, 5, 1, "sqexp", 8.0, clamp=False))
    m = O.build(cfg(2, 5, 1, "sqexp", 8.0))
    assert m.clamped[0] > 0 and m.clamped[1] > 0
    with pytest.raises(O.NotPositiveDefinite):
        # so long that the window covariance itself is singular: never clamped
        O.build(cfg(2, 5, 1, "sqexp", 50.0))
