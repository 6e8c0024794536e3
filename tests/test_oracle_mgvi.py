"""Pins of the oracle's MGVI pieces on tiny grids, against dense linear algebra.

The sample map (eta, eta') -> r must have covariance exactly M = I + L^T W L, CG must
reach the dense solve, the antithetic pair's mean gradient must equal the gradient at
the mean, and one Newton step must land on the dense posterior mean M^-1 L^T W d.
"""

import numpy as np

from oracle import icr_oracle as O

CFG = O.ICRConfig(ndim=2, shape0=(6, 5), depth=1, delta0=(1 / 6, 1 / 5), kernel="matern32", length=0.3)


def _setup():
    m = O.build(CFG)
    rng = np.random.default_rng(17)
    w = (rng.random(m.out_size) < 0.7) / 0.1 ** 2
    lmat = m.dense()
    mmat = lmat.T @ (w[:, None] * lmat) + np.eye(m.n_xi)
    return m, rng, w, lmat, mmat


def test_sample_right_hand_side_has_the_metric_as_covariance():
    m, rng, w, lmat, mmat = _setup()
    # the linear map (eta, eta') -> r, column by column
    cols = [O.weighted_adjoint(m, w, 0.5, np.zeros(m.out_size), add=e) for e in np.eye(m.n_xi)]
    cols += [O.weighted_adjoint(m, w, 0.5, e, add=np.zeros(m.n_xi)) for e in np.eye(m.out_size)]
    a = np.stack(cols, axis=1)
    np.testing.assert_allclose(a @ a.T, mmat, atol=1e-9 * np.abs(mmat).max())


def test_cg_reaches_the_dense_solve():
    m, rng, w, lmat, mmat = _setup()
    b = rng.standard_normal(m.n_xi)
    x = O.conjugate_gradient(lambda v: m.metric(w, v), b, 400)
    np.testing.assert_allclose(x, np.linalg.solve(mmat, b), rtol=1e-8, atol=1e-10)


def test_cg_iterates_minimise_the_energy_over_the_krylov_space():
    """After k steps from 0, CG's x_k is the minimiser of x.Mx/2 - b.x over
    span{b, Mb, ..., M^(k-1) b} (its defining property), computed densely from an
    orthonormal basis of that space."""
    m, rng, w, lmat, mmat = _setup()
    b = rng.standard_normal(m.n_xi)
    for k in (1, 2, 3, 5, 8):
        basis = [b]
        for _ in range(k - 1):
            basis.append(mmat @ basis[-1])
        q, _ = np.linalg.qr(np.stack(basis, axis=1))
        x_ref = q @ np.linalg.solve(q.T @ mmat @ q, q.T @ b)
        x = O.conjugate_gradient(lambda v: m.metric(w, v), b, k)
        np.testing.assert_allclose(x, x_ref, rtol=1e-7, atol=1e-9 * np.abs(x_ref).max())
        xs, steps, _ = O.conjugate_gradient_sl(lambda v: m.metric(w, v), b, -np.inf, k)
        assert steps == k
        np.testing.assert_allclose(xs, x_ref, rtol=1e-7, atol=1e-9 * np.abs(x_ref).max())


def test_drawn_sample_solves_the_metric_system():
    m, rng, w, lmat, mmat = _setup()
    eta, eta_d = rng.standard_normal(m.n_xi), rng.standard_normal(m.out_size)
    delta = O.mgvi_draw(m, w, eta, eta_d, 400)
    r = eta + lmat.T @ (np.sqrt(w) * eta_d)
    np.testing.assert_allclose(mmat @ delta, r, rtol=1e-8, atol=1e-8)


def test_antithetic_pair_gradient_equals_the_gradient_at_the_mean():
    m, rng, w, lmat, mmat = _setup()
    d = rng.standard_normal(m.out_size)
    mean, delta = rng.standard_normal((2, m.n_xi))
    g = 0.5 * (O.energy_gradient(m, w, d, mean + delta) + O.energy_gradient(m, w, d, mean - delta))
    dense = lmat.T @ (w * (lmat @ mean - d)) + mean
    np.testing.assert_allclose(g, dense, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g, mmat @ mean - lmat.T @ (w * d), rtol=1e-10, atol=1e-9)


def test_one_newton_step_reaches_the_posterior_mean():
    m, rng, w, lmat, mmat = _setup()
    d = rng.standard_normal(m.out_size)
    b = O.weighted_adjoint(m, w, 1.0, d)
    np.testing.assert_allclose(b, lmat.T @ (w * d), rtol=1e-10, atol=1e-10)
    mean = O.mgvi_newton_step(m, w, b, rng.standard_normal(m.n_xi), 400)
    np.testing.assert_allclose(mean, np.linalg.solve(mmat, lmat.T @ (w * d)), rtol=1e-8, atol=1e-9)


def test_energy_stopping_rule_against_dense_energies():
    """The energy-change rule: the energies the oracle evaluates equal x.Mx/2 - b.x with
    the dense M; a step's decrease equals alpha (r.r) / 2 (exact line search, the form
    the device uses); the rule stops at the first step whose decrease is below absdelta
    and the iterate is the plain CG iterate after that many steps."""
    m, rng, w, lmat, mmat = _setup()
    b = rng.standard_normal(m.n_xi)
    apply = lambda v: m.metric(w, v)
    n = 20
    _, steps, dec_all = O.conjugate_gradient_sl(apply, b, 0.0, n)
    assert steps == n and np.all(dec_all > 0)          # without a threshold: the limit
    energies = []
    for k in range(n + 1):
        xk = O.conjugate_gradient(apply, b, k)
        energies.append(0.5 * xk @ mmat @ xk - b @ xk)
    np.testing.assert_allclose(dec_all, -np.diff(energies), rtol=1e-7, atol=1e-12 * abs(energies[-1]))
    # closed form of a step's decrease
    x, r, p, rr = np.zeros_like(b), b.copy(), b.copy(), b @ b
    for k in range(10):
        q = mmat @ p
        alpha = rr / (p @ q)
        np.testing.assert_allclose(dec_all[k], 0.5 * alpha * rr, rtol=1e-7)
        x, r = x + alpha * p, r - alpha * q
        p, rr = r + (r @ r / rr) * p, r @ r
    # thresholds between the decreases: the rule stops after the first step below it
    for absdelta in (0.5 * dec_all[:6].min(), 0.9 * dec_all[:10].min(), 2.0 * dec_all[-1]):
        expect = next(k for k in range(n) if dec_all[k] < absdelta) + 1
        assert 1 < expect <= n
        x_sl, steps, _ = O.conjugate_gradient_sl(apply, b, absdelta, n)
        assert steps == expect
        np.testing.assert_allclose(x_sl, O.conjugate_gradient(apply, b, steps), rtol=1e-12, atol=1e-14)
    # a threshold above the first decrease stops after one step; the limit caps the steps
    assert O.conjugate_gradient_sl(apply, b, 2.0 * dec_all[0], n)[1] == 1
    assert O.conjugate_gradient_sl(apply, b, 1e-300, 5)[1] == 5
