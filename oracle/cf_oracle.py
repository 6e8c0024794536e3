"""Plain FP64 CPU oracle of the correlated-field model with a Poisson likelihood.

TEST INFRASTRUCTURE. Only the test suite and the benchmark's CPU-baseline leg import
this module. The library never calls it, and it shares no code with the library.

What it computes (NIFTy.re, section "Gaussian Processes", the correlated field; section
"Performance of NIFTy.re compared to NIFTy", the metric M_p it benchmarks). On an n x n
periodic grid of unit volume a realisation is s = FT(sqrt(P) xi) with xi standard
normal; the benchmark applies M_p = F_p + 1 with F_p the Fisher metric of a Poisson
likelihood at position p, written J^T N^-1 J with J the Jacobian of the forward model.

Readings where the paper is silent:
  * the field is real, so FT is the (real, symmetric) Hartley transform, normalised so
    that it is its own inverse: T x = (Re - Im)(FFT2 x) / n;
  * sqrt(P) is a fixed Matern-like amplitude spectrum
    A(k) = a (1 + (|k| l)^2)^(-g/4) over integer harmonic numbers |k| (the shorter way
    round the periodic grid), with the zero mode set to a0; the amplitude's own
    parameters are not excitations here;
  * the Poisson rate is lambda(xi) = exp(m + T(A xi)), so J = diag(lambda) T diag(A),
    N^-1 = diag(1 / lambda) and M_p v = v + A T(lambda(p) T(A v)).
"""

from __future__ import annotations

import numpy as np


def hartley2(x: np.ndarray) -> np.ndarray:
    """Unnormalised 2-D Hartley transform sum x[m, n] cas(2 pi (k m / n1 + l n / n2))."""
    f = np.fft.fft2(np.asarray(x, dtype=np.float64))
    return f.real - f.imag


def transform(x: np.ndarray) -> np.ndarray:
    """T x = hartley2(x) / sqrt(n1 n2): symmetric and its own inverse."""
    x = np.asarray(x, dtype=np.float64)
    return hartley2(x) / np.sqrt(x.shape[-2] * x.shape[-1])


def harmonic_norm(n: int) -> np.ndarray:
    """|k| of every harmonic mode of an n x n periodic grid (integer wave numbers)."""
    k = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
    return np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)


def amplitude(n: int, a: float, a0: float, length: float, slope: float) -> np.ndarray:
    """A(k) = a (1 + (|k| l)^2)^(-slope/4), A(0) = a0."""
    amp = a * (1.0 + (harmonic_norm(n) * length) ** 2) ** (-slope / 4.0)
    amp[0, 0] = a0
    return amp


def rate(amp: np.ndarray, p: np.ndarray, mean: float) -> np.ndarray:
    """lambda(p) = exp(m + T(A p))."""
    return np.exp(mean + transform(amp * p))


def metric_apply(amp: np.ndarray, lam: np.ndarray, v: np.ndarray) -> np.ndarray:
    """M_p v = v + A T(lambda T(A v))."""
    return v + amp * transform(lam * transform(amp * v))


def neg_log_likelihood_gradient(amp: np.ndarray, xi: np.ndarray, mean: float, counts: np.ndarray) -> np.ndarray:
    """Gradient of sum(lambda - d log lambda) over xi: A T(lambda - d) (T symmetric)."""
    lam = rate(amp, xi, mean)
    return amp * transform(lam - counts)
