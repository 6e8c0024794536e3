"""Plain FP64 CPU oracle of Iterative Charted Refinement (ICR).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark import this module. The library (HIP kernels behind the C ABI)
never calls it, and it shares no code with the library.

What it computes (NIFTy.re, section "Gaussian Processes"; the paper defers the
details of ICR to Edenhofer et al. 2022). A Gaussian-process sample s = L xi is
drawn from standard-normal excitations xi (section "Standardization": the prior
of every latent parameter is N(0, 1)) level by level:

  * level 0: s_0 = chol(K_00) xi_0 over the n_0^d pixels of the coarsest grid;
  * level l -> l+1: every interior coarse pixel c (all of whose 3^d neighbours
    exist) spawns 2^d fine pixels. Their values are the GP conditional mean given
    the 3^d window, R_l s_l[c + W], plus sqrt(D_l) times fresh excitations, with
    R_l = K_fc K_cc^-1 and D_l = K_ff - K_fc K_cc^-1 K_cf (textbook GP
    conditioning, Rasmussen & Williams 2006, eq. 2.19).

The adjoint L^T is the exact transpose of that sweep, and the metric of a
Gaussian likelihood in standardized coordinates is M = L^T N^-1 L + 1 (section
"Performance of NIFTy.re compared to NIFTy": the Fisher metric plus the identity).
The gradient of <ybar, L xi> with respect to the kernel's scale and length scale
(hyper_grad) follows the level recursion by the chain rule, with the derivatives of
R = K_fc K_cc^-1, D and their Cholesky factors written out in closed form (the
paper values automatic differentiation of the model, section "Gaussian Processes").

Readings where the paper is silent:
  * children sit at +-delta/4 per axis around their coarse pixel, so the fine grid
    has spacing delta/2 and n_{l+1} = 2 (n_l - 2); border coarse pixels only take
    part in windows;
  * windows W = {-1,0,1}^d and children {0,1}^d are ordered lexicographically with
    the last axis fastest; xi is stored level by level, each level in C order;
  * sqrt(D) is the lower Cholesky factor, and a pivot <= tau = 3^d eps k(0) is
    clamped (its column set to zero and counted) instead of failing;
  * the log-radial chart maps index coordinates (u, v) to
    (r0 e^(g u) cos(a v), r0 e^(g u) sin(a v)); the log-radial cylinder chart maps
    (u, v, w) to (r0 e^(g u) cos(a v), r0 e^(g u) sin(a v), h w).

Every function here is pinned by a test in tests/test_oracle_*.py against closed
forms, invariants or library routines; none is "parity unpinned".
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

EPS64 = float(np.finfo(np.float64).eps)

KERNELS = ("matern12", "matern32", "matern52", "sqexp")
CHARTS = ("regular", "logradial2d", "logradial_cyl3d")


class NotPositiveDefinite(ValueError):
    """A factorisation met a non-positive pivot where clamping is not allowed."""


# ---------------------------------------------------------------------------
# Kernels (standard stationary forms, Rasmussen & Williams 2006, section 4.2)
# ---------------------------------------------------------------------------

def kernel_values(kind: str, r, scale: float, length: float) -> np.ndarray:
    """Covariance k(r) for Euclidean distance r; k(0) = scale**2."""
    t = np.asarray(r, dtype=np.float64) / float(length)
    if kind == "matern12":
        k = np.exp(-t)
    elif kind == "matern32":
        a = math.sqrt(3.0) * t
        k = (1.0 + a) * np.exp(-a)
    elif kind == "matern52":
        a = math.sqrt(5.0) * t
        k = (1.0 + a + a * a / 3.0) * np.exp(-a)
    elif kind == "sqexp":
        k = np.exp(-0.5 * t * t)
    else:
        raise ValueError(f"unknown kernel {kind!r}")
    return float(scale) ** 2 * k


def pairwise_distance(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Euclidean distances between point sets a (..., m, dim) and b (..., n, dim)."""
    diff = a[..., :, None, :] - b[..., None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=-1))


# ---------------------------------------------------------------------------
# Geometry
# ---------------------------------------------------------------------------

def level_shapes(shape0, depth: int) -> list[tuple[int, ...]]:
    """Grid shape of every level: n_{l+1} = 2 (n_l - 2) per axis."""
    shapes = [tuple(int(n) for n in shape0)]
    for _ in range(depth):
        prev = shapes[-1]
        if min(prev) < 3:
            raise ValueError(f"a level of shape {prev} has no interior pixel to refine")
        shapes.append(tuple(2 * (n - 2) for n in prev))
    return shapes


def level_spacings(delta0, depth: int) -> list[np.ndarray]:
    """Pixel spacing per axis at every level: delta_l = delta_0 / 2^l."""
    d0 = np.asarray(delta0, dtype=np.float64)
    return [d0 / 2.0 ** l for l in range(depth + 1)]


def level_origins(delta0, depth: int) -> list[np.ndarray]:
    """Position of pixel 0 at every level: o_0 = 0, o_{l+1} = o_l + 3/4 delta_l.

    Fine pixel 0 is the lower child of coarse pixel 1, which sits at
    o_l + delta_l - delta_l / 4.
    """
    spac = level_spacings(delta0, depth)
    org = [np.zeros_like(spac[0])]
    for l in range(depth):
        org.append(org[-1] + 0.75 * spac[l])
    return org


def window_offsets(ndim: int) -> np.ndarray:
    """The 3^d window offsets {-1,0,1}^d, lexicographic, last axis fastest."""
    return np.array(list(itertools.product((-1, 0, 1), repeat=ndim)), dtype=np.int64)


def child_offsets(ndim: int) -> np.ndarray:
    """The 2^d child offsets {0,1}^d, lexicographic, last axis fastest."""
    return np.array(list(itertools.product((0, 1), repeat=ndim)), dtype=np.int64)


def grid_indices(shape) -> np.ndarray:
    """All multi-indices of a grid in C order, shape (prod(shape), ndim)."""
    return np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"),
                    axis=-1).reshape(-1, len(shape))


def logradial_chart(points: np.ndarray, params) -> np.ndarray:
    """Map index-space points (u, v) to (r cos theta, r sin theta).

    r = r0 exp(g u) and theta = a v with params = (r0, g, a).
    """
    r0, g, a = float(params[0]), float(params[1]), float(params[2])
    r = r0 * np.exp(g * points[..., 0])
    th = a * points[..., 1]
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=-1)


def logradial_cylinder_chart(points: np.ndarray, params) -> np.ndarray:
    """Map index-space points (u, v, w) to (r cos theta, r sin theta, h w).

    r = r0 exp(g u), theta = a v and height h w with params = (r0, g, a, h): the
    log-radial chart of the plane extended by a linear axis.
    """
    if len(params) < 4:
        raise ValueError("the log-radial cylinder chart takes (r0, g, a, h)")
    r0, g, a, h = (float(v) for v in params[:4])
    r = r0 * np.exp(g * points[..., 0])
    th = a * points[..., 1]
    return np.stack([r * np.cos(th), r * np.sin(th), h * points[..., 2]], axis=-1)


# ---------------------------------------------------------------------------
# Clamped Cholesky
# ---------------------------------------------------------------------------

def clamped_cholesky(a: np.ndarray, tau: float, clamp: bool = True):
    """Lower Cholesky factor of symmetric a (..., n, n), column by column.

    Column j of the Schur complement is a[j:, j] - L[j:, :j] L[j, :j]^T. A pivot
    at or below tau makes column j of L zero (and is counted) when clamp is True,
    else NotPositiveDefinite is raised. Returns (L, number of clamped pivots).
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[-1]
    low = np.zeros_like(a)
    count = np.zeros(a.shape[:-2], dtype=np.int64)
    for j in range(n):
        col = a[..., j:, j] - (low[..., j:, :j] @ low[..., j, :j][..., None])[..., 0]
        piv = col[..., 0]
        bad = ~(piv > tau)
        if np.any(bad) and not clamp:
            raise NotPositiveDefinite(f"pivot {j} is {np.min(piv)!r} <= {tau!r}")
        root = np.sqrt(np.where(bad, 1.0, piv))
        low[..., j:, j] = np.where(bad[..., None], 0.0, col / root[..., None])
        count += bad
    return low, count


def pivot_threshold(ndim: int, scale: float) -> float:
    """Clamp threshold tau = 3^d eps_64 k(0)."""
    return 3.0 ** ndim * EPS64 * float(scale) ** 2


# ---------------------------------------------------------------------------
# Conditioning matrices: R = K_fc K_cc^-1, D = K_ff - R K_cf, sqrt(D)
# ---------------------------------------------------------------------------

def conditional_matrices(kind, scale, length, win_pos, child_pos, tau, clamp=True):
    """Refinement matrix and lower sqrt of the conditional covariance.

    win_pos: (..., 3^d, dim) physical window positions; child_pos: (..., 2^d, dim).
    Returns R (..., 2^d, 3^d), sqrtD (..., 2^d, 2^d), clamped-pivot counts (...).
    """
    k_cc = kernel_values(kind, pairwise_distance(win_pos, win_pos), scale, length)
    k_fc = kernel_values(kind, pairwise_distance(child_pos, win_pos), scale, length)
    k_ff = kernel_values(kind, pairwise_distance(child_pos, child_pos), scale, length)
    try:
        np.linalg.cholesky(k_cc)  # K_cc must be positive definite for the solve
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite("window covariance K_cc is not positive definite") from exc
    # R K_cc = K_fc  <=>  K_cc R^T = K_cf (K_cc symmetric)
    r_mat = np.swapaxes(np.linalg.solve(k_cc, np.swapaxes(k_fc, -1, -2)), -1, -2)
    d_mat = k_ff - r_mat @ np.swapaxes(k_fc, -1, -2)
    d_mat = 0.5 * (d_mat + np.swapaxes(d_mat, -1, -2))
    sqrt_d, count = clamped_cholesky(d_mat, tau, clamp)
    return r_mat, sqrt_d, count


# ---------------------------------------------------------------------------
# The ICR model
# ---------------------------------------------------------------------------

@dataclass
class ICRConfig:
    """Parameters of one ICR prior (all lengths in the chart's index units)."""
    ndim: int
    shape0: tuple
    depth: int
    delta0: tuple
    kernel: str = "matern32"
    scale: float = 1.0
    length: float = 0.1
    chart: str = "regular"
    chart_params: tuple = (0.1, math.log(10.0), 0.5 * math.pi)
    clamp: bool = True


@dataclass
class ICROracle:
    cfg: ICRConfig
    shapes: list = field(default_factory=list)
    offsets: list = field(default_factory=list)
    n_xi: int = 0
    l00: np.ndarray | None = None
    r_mats: list = field(default_factory=list)      # per level: (2^d,3^d) or (*n_int, 2^d, 3^d)
    sqrt_ds: list = field(default_factory=list)     # per level: (2^d,2^d) or (*n_int, 2^d, 2^d)
    clamped: list = field(default_factory=list)     # per level (and level 0 first)

    # -- sizes ---------------------------------------------------------------
    @property
    def out_size(self) -> int:
        return int(np.prod(self.shapes[-1]))

    def level_slice(self, l: int) -> slice:
        return slice(self.offsets[l], self.offsets[l] + int(np.prod(self.shapes[l])))

    # -- forward -------------------------------------------------------------
    def forward(self, xi: np.ndarray, return_levels: bool = False):
        """s = L xi for xi of shape (..., N_xi); returns s_L (..., prod(n_L))."""
        d = self.cfg.ndim
        xi = np.asarray(xi, dtype=np.float64)
        batch = xi.shape[:-1]
        s = (xi[..., self.level_slice(0)] @ self.l00.T).reshape(batch + self.shapes[0])
        levels = [s]
        for l in range(self.cfg.depth):
            xi_f = xi[..., self.level_slice(l + 1)].reshape(batch + self.shapes[l + 1])
            s = refine(s, xi_f, self.r_mats[l], self.sqrt_ds[l], d)
            levels.append(s)
        flat = [v.reshape(batch + (-1,)) for v in levels]
        return (flat[-1], flat) if return_levels else flat[-1]

    # -- adjoint -------------------------------------------------------------
    def adjoint(self, ybar: np.ndarray, return_levels: bool = False):
        """xi_bar = L^T ybar for ybar of shape (..., prod(n_L)); returns (..., N_xi)."""
        d = self.cfg.ndim
        ybar = np.asarray(ybar, dtype=np.float64)
        batch = ybar.shape[:-1]
        out = np.zeros(batch + (self.n_xi,))
        y = ybar.reshape(batch + self.shapes[-1])
        cot = [None] * (self.cfg.depth + 1)
        cot[-1] = y
        for l in reversed(range(self.cfg.depth)):
            xi_bar_f, y = refine_adjoint(y, self.r_mats[l], self.sqrt_ds[l], d, self.shapes[l])
            out[..., self.level_slice(l + 1)] = xi_bar_f.reshape(batch + (-1,))
            cot[l] = y
        out[..., self.level_slice(0)] = y.reshape(batch + (-1,)) @ self.l00
        if return_levels:
            return out, [c.reshape(batch + (-1,)) for c in cot]
        return out

    # -- metric --------------------------------------------------------------
    def metric(self, w: np.ndarray, v: np.ndarray) -> np.ndarray:
        """M v = L^T (w * (L v)) + v, with w the inverse noise variance per pixel."""
        return self.adjoint(np.asarray(w, dtype=np.float64) * self.forward(v)) + v

    # -- dense ---------------------------------------------------------------
    def dense(self) -> np.ndarray:
        """Dense L (prod(n_L) x N_xi) built column by column from the forward."""
        return self.forward(np.eye(self.n_xi)).T

    def dense_adjoint(self) -> np.ndarray:
        """Dense L^T (N_xi x prod(n_L)) built column by column from the adjoint."""
        return self.adjoint(np.eye(self.out_size)).T


def refine(s: np.ndarray, xi_f: np.ndarray, r_mat, sqrt_d, ndim: int) -> np.ndarray:
    """One forward level: fine = R s[window] + sqrt(D) xi for every interior coarse pixel.

    s: (..., n_c...), xi_f: (..., 2(n_c - 2)...). r_mat is (2^d, 3^d) for a stationary
    level or (*n_int, 2^d, 3^d) per interior coarse pixel (charted); same for sqrt_d.
    """
    batch = s.shape[:-ndim]
    nc = s.shape[-ndim:]
    wins = window_offsets(ndim)
    kids = child_offsets(ndim)
    out = np.empty(batch + tuple(2 * (n - 2) for n in nc))
    lead = (Ellipsis,)
    for ib, b in enumerate(kids):
        acc = np.zeros(batch + tuple(n - 2 for n in nc))
        for iw, w in enumerate(wins):
            window = s[lead + tuple(slice(1 + w[a], nc[a] - 1 + w[a]) for a in range(ndim))]
            acc = acc + _coef(r_mat, ib, iw) * window
        for jb, bp in enumerate(kids):
            fresh = xi_f[lead + tuple(slice(bp[a], None, 2) for a in range(ndim))]
            acc = acc + _coef(sqrt_d, ib, jb) * fresh
        out[lead + tuple(slice(b[a], None, 2) for a in range(ndim))] = acc
    return out


def refine_adjoint(ybar_f: np.ndarray, r_mat, sqrt_d, ndim: int, nc):
    """Transpose of `refine`: returns (xi_bar of the fine level, s_bar of the coarse level).

    The coarse cotangent is accumulated by scatter-add in FP64, the plain reading of
    the transpose.
    """
    batch = ybar_f.shape[:-ndim]
    wins = window_offsets(ndim)
    kids = child_offsets(ndim)
    lead = (Ellipsis,)
    blocks = [ybar_f[lead + tuple(slice(b[a], None, 2) for a in range(ndim))] for b in kids]
    xi_bar = np.empty_like(ybar_f)
    for jb, bp in enumerate(kids):
        acc = sum(_coef(sqrt_d, ib, jb) * blocks[ib] for ib in range(len(kids)))
        xi_bar[lead + tuple(slice(bp[a], None, 2) for a in range(ndim))] = acc
    s_bar = np.zeros(batch + tuple(nc))
    for iw, w in enumerate(wins):
        acc = sum(_coef(r_mat, ib, iw) * blocks[ib] for ib in range(len(kids)))
        s_bar[lead + tuple(slice(1 + w[a], nc[a] - 1 + w[a]) for a in range(ndim))] += acc
    return xi_bar, s_bar


def _coef(mat, i, j):
    """Entry (i, j) of a shared matrix, or the per-pixel field of entries of a stack."""
    return mat[..., i, j]


# ---------------------------------------------------------------------------
# Building a model
# ---------------------------------------------------------------------------

def _positions(cfg: ICRConfig, idx_points: np.ndarray) -> np.ndarray:
    if cfg.chart == "regular":
        return idx_points
    if cfg.chart == "logradial2d":
        if cfg.ndim != 2:
            raise ValueError("the log-radial chart is two-dimensional")
        return logradial_chart(idx_points, cfg.chart_params)
    if cfg.chart == "logradial_cyl3d":
        if cfg.ndim != 3:
            raise ValueError("the log-radial cylinder chart is three-dimensional")
        return logradial_cylinder_chart(idx_points, cfg.chart_params)
    raise ValueError(f"unknown chart {cfg.chart!r}")


def _level0_positions(cfg: ICRConfig, shape0) -> np.ndarray:
    """Physical positions of the level-0 pixels in C order."""
    spac = level_spacings(cfg.delta0, 0)[0]
    return _positions(cfg, grid_indices(shape0) * spac)


def _window_positions(cfg: ICRConfig, shapes, l: int):
    """Physical window (3^d) and child (2^d) positions of every matrix set of level l.

    Stationary grid: one set, relative to the coarse pixel, shapes (1, 3^d, d) and
    (1, 2^d, d). Chart: one set per interior coarse pixel in C order.
    """
    d = cfg.ndim
    dl = level_spacings(cfg.delta0, cfg.depth)[l]
    wins = window_offsets(d).astype(np.float64)
    kids = child_offsets(d).astype(np.float64)
    if cfg.chart == "regular":
        # stationary: one set per level, geometry relative to the coarse pixel
        return (wins * dl)[None], ((kids - 0.5) * dl / 2.0)[None]
    org = level_origins(cfg.delta0, cfg.depth)[l]
    n_int = tuple(n - 2 for n in shapes[l])
    centre = org + (grid_indices(n_int) + 1) * dl                # (P, d)
    win_idx = centre[:, None, :] + wins[None] * dl               # (P, 3^d, d)
    kid_idx = centre[:, None, :] + (kids[None] - 0.5) * dl / 2.0
    return _positions(cfg, win_idx), _positions(cfg, kid_idx)


def _set_shape(cfg: ICRConfig, shapes, l: int, mat: np.ndarray) -> np.ndarray:
    """A level's stack of sets as stored: (2^d, .) when stationary, else per pixel."""
    if cfg.chart == "regular":
        return mat[0]
    n_int = tuple(n - 2 for n in shapes[l])
    return mat.reshape(n_int + mat.shape[-2:])


def build(cfg: ICRConfig) -> ICROracle:
    """Level sizes, level-0 Cholesky factor and per-level R, sqrt(D) in FP64."""
    if cfg.ndim not in (1, 2, 3):
        raise ValueError("ndim must be 1, 2 or 3")
    if cfg.kernel not in KERNELS:
        raise ValueError(f"unknown kernel {cfg.kernel!r}")
    d = cfg.ndim
    model = ICROracle(cfg)
    model.shapes = level_shapes(cfg.shape0, cfg.depth)
    sizes = [int(np.prod(s)) for s in model.shapes]
    model.offsets = [int(v) for v in np.concatenate([[0], np.cumsum(sizes)[:-1]])]
    model.n_xi = int(sum(sizes))
    tau = pivot_threshold(d, cfg.scale)

    # level 0: dense Cholesky of the kernel over all n_0^d pixels, C order
    x0 = _level0_positions(cfg, model.shapes[0])
    k00 = kernel_values(cfg.kernel, pairwise_distance(x0, x0), cfg.scale, cfg.length)
    model.l00, c0 = clamped_cholesky(k00, tau, cfg.clamp)
    model.clamped = [int(c0)]

    for l in range(cfg.depth):
        win_pos, child_pos = _window_positions(cfg, model.shapes, l)
        r_mat, sqrt_d, cnt = conditional_matrices(cfg.kernel, cfg.scale, cfg.length,
                                                  win_pos, child_pos, tau, cfg.clamp)
        model.r_mats.append(_set_shape(cfg, model.shapes, l, r_mat))
        model.sqrt_ds.append(_set_shape(cfg, model.shapes, l, sqrt_d))
        model.clamped.append(int(np.sum(cnt)))
    return model


# ---------------------------------------------------------------------------
# Gradients with respect to the kernel hyperparameters (scale sigma, length l)
# ---------------------------------------------------------------------------
#
# L depends on theta = (sigma, l) through K_00 and every level's R and sqrt(D). For
# E = <ybar, L xi> the chain rule through the level recursion
#   s_0 = L_00 xi_0,   s_{l+1} = R_l s_l[window] + sqrt(D_l) xi_{l+1}
# gives dE/dtheta = sum_l <sbar_{l+1}, dR_l s_l[window] + d sqrt(D_l) xi_{l+1}>
#                   + <sbar_0, dL_00 xi_0>,
# with sbar_l the level cotangents of the adjoint sweep. Every covariance is
# proportional to sigma^2, so R does not depend on sigma, sqrt(D) and L_00 are
# proportional to sigma, and dE/dsigma = <ybar, L xi> / sigma.

def kernel_length_derivative(kind: str, r, scale: float, length: float) -> np.ndarray:
    """d k(r) / d length of the kernels of kernel_values (closed forms)."""
    t = np.asarray(r, dtype=np.float64) / float(length)
    if kind == "matern12":
        dk = np.exp(-t) * t
    elif kind == "matern32":
        a = math.sqrt(3.0) * t
        dk = a * a * np.exp(-a)
    elif kind == "matern52":
        a = math.sqrt(5.0) * t
        dk = a * a * (1.0 + a) / 3.0 * np.exp(-a)
    elif kind == "sqexp":
        dk = t * t * np.exp(-0.5 * t * t)
    else:
        raise ValueError(f"unknown kernel {kind!r}")
    return float(scale) ** 2 * dk / float(length)


def cholesky_derivative(low: np.ndarray, da: np.ndarray) -> np.ndarray:
    """Directional derivative of the lower Cholesky factor L of A along symmetric dA.

    From dA = dL L^T + L dL^T with dL lower: L^-1 dA L^-T = Phi + Phi^T where
    Phi = L^-1 dL is lower, so Phi is the lower triangle of X = L^-1 dA L^-T with its
    diagonal halved and dL = L Phi. A clamped (zero) column makes L singular; its
    derivative is undefined and NotPositiveDefinite is raised.
    """
    low = np.asarray(low, dtype=np.float64)
    if np.any(np.diagonal(low, axis1=-2, axis2=-1) <= 0.0):
        raise NotPositiveDefinite("the factor has a clamped column: no derivative")
    x = np.linalg.solve(low, da)                                   # L^-1 dA
    x = np.linalg.solve(low, np.swapaxes(x, -1, -2))               # L^-1 (L^-1 dA)^T = L^-1 dA L^-T
    x = 0.5 * (x + np.swapaxes(x, -1, -2))
    n = low.shape[-1]
    phi = np.tril(x) - 0.5 * np.eye(n) * np.diagonal(x, axis1=-2, axis2=-1)[..., None, :]
    return low @ phi


def conditional_matrices_length_derivative(kind, scale, length, win_pos, child_pos, r_mat, sqrt_d):
    """d R / d length and d sqrt(D) / d length of conditional_matrices' results.

    R K_cc = K_fc gives dR = (dK_fc - R dK_cc) K_cc^-1, and D = K_ff - R K_cf gives
    dD = dK_ff - dR K_cf - R dK_cf (symmetrised); sqrt(D) follows cholesky_derivative.
    """
    dist_cc = pairwise_distance(win_pos, win_pos)
    dist_fc = pairwise_distance(child_pos, win_pos)
    dist_ff = pairwise_distance(child_pos, child_pos)
    k_cc = kernel_values(kind, dist_cc, scale, length)
    k_fc = kernel_values(kind, dist_fc, scale, length)
    dk_cc = kernel_length_derivative(kind, dist_cc, scale, length)
    dk_fc = kernel_length_derivative(kind, dist_fc, scale, length)
    dk_ff = kernel_length_derivative(kind, dist_ff, scale, length)
    rhs = np.swapaxes(dk_fc - r_mat @ dk_cc, -1, -2)
    d_r = np.swapaxes(np.linalg.solve(k_cc, rhs), -1, -2)
    d_d = dk_ff - d_r @ np.swapaxes(k_fc, -1, -2) - r_mat @ np.swapaxes(dk_fc, -1, -2)
    d_d = 0.5 * (d_d + np.swapaxes(d_d, -1, -2))
    return d_r, cholesky_derivative(sqrt_d, d_d)


def length_derivatives(model: ICROracle):
    """d L_00, [d R_l], [d sqrt(D_l)] with respect to the length scale, shaped as stored."""
    cfg = model.cfg
    x0 = _level0_positions(cfg, model.shapes[0])
    dist0 = pairwise_distance(x0, x0)
    d_l00 = cholesky_derivative(model.l00, kernel_length_derivative(cfg.kernel, dist0, cfg.scale, cfg.length))
    d_r, d_s = [], []
    for l in range(cfg.depth):
        win_pos, child_pos = _window_positions(cfg, model.shapes, l)
        nset = win_pos.shape[0]
        r_mat = np.reshape(model.r_mats[l], (nset,) + model.r_mats[l].shape[-2:])
        s_mat = np.reshape(model.sqrt_ds[l], (nset,) + model.sqrt_ds[l].shape[-2:])
        dr, ds = conditional_matrices_length_derivative(cfg.kernel, cfg.scale, cfg.length, win_pos,
                                                        child_pos, r_mat, s_mat)
        d_r.append(_set_shape(cfg, model.shapes, l, dr))
        d_s.append(_set_shape(cfg, model.shapes, l, ds))
    return d_l00, d_r, d_s


def hyper_grad(model: ICROracle, xi: np.ndarray, ybar: np.ndarray) -> np.ndarray:
    """(dE/dsigma, dE/dlength) of E = <ybar, L xi> per sample, shape (..., 2)."""
    d = model.cfg.ndim
    xi = np.asarray(xi, dtype=np.float64)
    ybar = np.asarray(ybar, dtype=np.float64)
    batch = xi.shape[:-1]
    s_final, s_levels = model.forward(xi, return_levels=True)
    _, cot = model.adjoint(ybar, return_levels=True)
    g_sigma = np.sum(ybar * s_final, axis=-1) / model.cfg.scale
    d_l00, d_r, d_s = length_derivatives(model)
    g_len = np.sum(cot[0] * (xi[..., model.level_slice(0)] @ d_l00.T), axis=-1)
    for l in range(model.cfg.depth):
        s_l = s_levels[l].reshape(batch + model.shapes[l])
        xi_f = xi[..., model.level_slice(l + 1)].reshape(batch + model.shapes[l + 1])
        t = refine(s_l, xi_f, d_r[l], d_s[l], d).reshape(batch + (-1,))
        g_len = g_len + np.sum(cot[l + 1] * t, axis=-1)
    return np.stack([g_sigma, g_len], axis=-1)


# ---------------------------------------------------------------------------
# Metric Gaussian Variational Inference around the ICR prior
# ---------------------------------------------------------------------------
#
# Section "Variational Inference": MGVI approximates the posterior by samples drawn
# around an expansion point with the Fisher metric plus the prior curvature, and
# alternates between drawing samples and minimising the KL divergence over the
# expansion point (antithetically mirrored samples, CG for the samples, a Newton-CG
# minimiser for the KL). Here the likelihood is Gaussian with inverse noise variance
# w per final pixel, so the energy H(xi) = 1/2 (d - L xi)^T W (d - L xi) + 1/2 xi^T xi
# has gradient M xi - L^T W d and the metric M = L^T W L + 1 everywhere:
#  * a sample: r = eta + L^T (sqrt(w) * eta') with eta, eta' standard normal has
#    covariance M, so delta = M^-1 r (CG) has covariance M^-1, and mean +- delta is an
#    antithetic pair;
#  * the KL over antithetic pairs has gradient mean over the pairs of grad H(mean +- delta)
#    = M mean - L^T W d, and one Newton step mean - M^-1 (M mean - L^T W d) (CG).

def conjugate_gradient(apply, b: np.ndarray, iterations: int) -> np.ndarray:
    """Textbook CG from x_0 = 0 for exactly `iterations` steps (Hestenes & Stiefel 1952)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    for _ in range(iterations):
        if rr == 0.0:
            break
        q = apply(p)
        alpha = rr / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def cg_energy(mx: np.ndarray, b: np.ndarray, x: np.ndarray) -> float:
    """The CG energy E(x) = x.Mx / 2 - b.x, given Mx."""
    return 0.5 * float(x @ mx) - float(b @ x)


def conjugate_gradient_sl(apply, b: np.ndarray, absdelta: float, maxiter: int):
    """CG from x_0 = 0 stopped by the change of its energy (section "Variational
    Inference": the linear samples are drawn by CG with an absolute energy tolerance and
    an iteration limit). Each step is the textbook one; after it, E(x) = x.Mx / 2 - b.x
    is evaluated from its definition (Mx carried along by linearity) and CG stops once a
    step lowered E by less than absdelta, keeping that step, or after maxiter steps, or
    at a zero residual. Returns (x, steps, per-step energy decreases)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    mx = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(r @ r)
    energy = cg_energy(mx, b, x)
    decreases = []
    while len(decreases) < maxiter and rr != 0.0:
        q = apply(p)
        alpha = rr / float(p @ q)
        x = x + alpha * p
        mx = mx + alpha * q
        r = r - alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        new_energy = cg_energy(mx, b, x)
        decreases.append(energy - new_energy)
        energy = new_energy
        if decreases[-1] < absdelta:
            break
    return x, len(decreases), np.array(decreases)


def weighted_adjoint(model: ICROracle, w: np.ndarray, power: float, y: np.ndarray, add=None) -> np.ndarray:
    """L^T (w^power * y) (+ add)."""
    out = model.adjoint(np.asarray(w, dtype=np.float64) ** power * np.asarray(y, dtype=np.float64))
    return out if add is None else out + np.asarray(add, dtype=np.float64)


def mgvi_draw(model: ICROracle, w: np.ndarray, eta_xi: np.ndarray, eta_data: np.ndarray, iterations: int):
    """One MGVI sample displacement delta = M^-1 (eta + L^T (sqrt(w) eta')) by CG; mean +- delta."""
    r = weighted_adjoint(model, w, 0.5, eta_data, add=eta_xi)
    return conjugate_gradient(lambda v: model.metric(w, v), r, iterations)


def energy_gradient(model: ICROracle, w: np.ndarray, d: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """grad H(xi) = L^T W (L xi - d) + xi."""
    return model.adjoint(np.asarray(w) * (model.forward(xi) - np.asarray(d))) + xi


def mgvi_newton_step(model: ICROracle, w: np.ndarray, b: np.ndarray, mean: np.ndarray, iterations: int):
    """mean - M^-1 g with g = M mean - b, b = L^T W d (CG for M^-1 g)."""
    g = model.metric(w, mean) - b
    return mean - conjugate_gradient(lambda v: model.metric(w, v), g, iterations)
