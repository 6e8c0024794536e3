"""Pins of the correlated-field oracle: the Hartley transform against its definition
summed by brute force, its symmetry and involution, the stationary covariance of a
sample against the Wiener-Khinchin closed form, and the Fisher metric against finite
differences of the Poisson log-likelihood gradient (for the exponential link the
Hessian equals the Fisher metric)."""

import math

import numpy as np

from oracle import cf_oracle as F


def test_hartley_transform_matches_the_cas_sum():
    rng = np.random.default_rng(1)
    for n1, n2 in ((4, 4), (8, 6), (5, 7)):
        x = rng.standard_normal((n1, n2))
        m, n = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
        ref = np.empty((n1, n2))
        for k in range(n1):
            for l in range(n2):
                ang = 2 * math.pi * (k * m / n1 + l * n / n2)
                ref[k, l] = np.sum(x * (np.cos(ang) + np.sin(ang)))
        np.testing.assert_allclose(F.hartley2(x), ref, atol=1e-11)


def test_transform_is_symmetric_and_its_own_inverse():
    n = 8
    cols = np.stack([F.transform(e.reshape(n, n)).ravel() for e in np.eye(n * n)], axis=1)
    np.testing.assert_allclose(cols, cols.T, atol=1e-13)
    np.testing.assert_allclose(cols @ cols, np.eye(n * n), atol=1e-12)


def test_sample_covariance_is_stationary_with_the_amplitude_spectrum():
    """Cov(T(A xi)) = T diag(A^2) T is circulant, its first row the inverse DFT of A^2."""
    n = 8
    amp = F.amplitude(n, 1.3, 0.4, 0.3, 3.0)
    cols = np.stack([F.transform(amp * e.reshape(n, n)).ravel() for e in np.eye(n * n)], axis=1)
    cov = cols @ cols.T
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    k = np.stack([ii.ravel(), jj.ravel()], axis=1)
    for a in (0, 9, 27):
        for b in range(n * n):
            d = (k[b] - k[a]) % n
            ref = np.sum(amp ** 2 * np.cos(2 * math.pi * (ii * d[0] + jj * d[1]) / n)) / n ** 2
            assert abs(cov[a, b] - ref) < 1e-12


def test_amplitude_spectrum_closed_form():
    amp = F.amplitude(6, 2.0, 0.5, 0.25, 4.0)
    assert amp[0, 0] == 0.5
    np.testing.assert_allclose(amp[1, 0], 2.0 / (1 + 0.25 ** 2), rtol=1e-14)
    np.testing.assert_allclose(amp[5, 5], amp[1, 1], rtol=1e-14)   # shorter way round
    np.testing.assert_allclose(amp[3, 2], 2.0 / (1 + 13 * 0.25 ** 2), rtol=1e-14)


def test_metric_is_the_hessian_of_the_poisson_log_likelihood():
    n = 8
    rng = np.random.default_rng(3)
    amp = F.amplitude(n, 1.0, 0.3, 0.2, 3.0)
    p = 0.3 * rng.standard_normal((n, n))
    counts = rng.poisson(5.0, (n, n)).astype(np.float64)
    v = rng.standard_normal((n, n))
    lam = F.rate(amp, p, 1.5)
    h = 1e-6
    fd = (F.neg_log_likelihood_gradient(amp, p + h * v, 1.5, counts)
          - F.neg_log_likelihood_gradient(amp, p - h * v, 1.5, counts)) / (2 * h)
    np.testing.assert_allclose(F.metric_apply(amp, lam, v) - v, fd, rtol=1e-6, atol=1e-7)
    # symmetric, bounded below by 1
    cols = np.stack([F.metric_apply(amp, lam, e.reshape(n, n)).ravel() for e in np.eye(n * n)], axis=1)
    np.testing.assert_allclose(cols, cols.T, atol=1e-10)
    assert np.linalg.eigvalsh(0.5 * (cols + cols.T)).min() >= 1 - 1e-10
