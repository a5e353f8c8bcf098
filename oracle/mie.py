"""Mie series for plane-wave scattering by a PEC sphere (oracle check path).

Textbook series (Bohren & Huffman, Absorption and Scattering of Light by Small
Particles, 1983, Sec. 4.4, with the perfectly conducting limit of the
coefficients; also Harrington, Time-Harmonic Electromagnetic Fields, Sec. 6-9).
With x = ka, psi_n(x) = x j_n(x), xi_n(x) = x h_n^(1)(x):
    a_n = psi_n'(x)/xi_n'(x),     b_n = psi_n(x)/xi_n(x)
    S1(t) = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n)
    S2(t) = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n)
    pi_n = P_n^1(cos t)/sin t,  tau_n = d P_n^1(cos t)/dt
For incidence along +z polarised along x, at scattering angles (t, phi):
    sigma(t, phi) = (4 pi / k^2) (cos^2 phi |S2(t)|^2 + sin^2 phi |S1(t)|^2).
Magnitudes do not depend on the exp(+-j w t) convention.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def coefficients(x: float, nmax: int | None = None):
    if nmax is None:
        nmax = int(x + 4.05 * x ** (1.0 / 3.0) + 10)
    n = np.arange(1, nmax + 1)
    j = spherical_jn(n, x); jd = spherical_jn(n, x, derivative=True)
    y = spherical_yn(n, x); yd = spherical_yn(n, x, derivative=True)
    h = j + 1j * y; hd = jd + 1j * yd
    psi = x * j; dpsi = j + x * jd
    xi = x * h; dxi = h + x * hd
    return n, dpsi / dxi, psi / xi


def angular(n: np.ndarray, mu: float):
    nmax = int(n[-1])
    pi = np.zeros(nmax + 1); tau = np.zeros(nmax + 1)
    pi[1] = 1.0
    for k in range(2, nmax + 1):
        pi[k] = (2 * k - 1) / (k - 1) * mu * pi[k - 1] - k / (k - 1) * pi[k - 2]
    for k in range(1, nmax + 1):
        tau[k] = k * mu * pi[k] - (k + 1) * pi[k - 1]
    return pi[1:], tau[1:]


def amplitudes(ka: float, theta: np.ndarray):
    n, a, b = coefficients(ka)
    fac = (2 * n + 1) / (n * (n + 1))
    S1 = []; S2 = []
    for t in np.atleast_1d(theta):
        pi, tau = angular(n, math.cos(t))
        S1.append(np.sum(fac * (a * pi + b * tau)))
        S2.append(np.sum(fac * (a * tau + b * pi)))
    return np.array(S1), np.array(S2)


def rcs(k: float, a: float, theta, phi) -> np.ndarray:
    """Bistatic RCS (m^2); incidence along +z, polarisation along x."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    phi = np.broadcast_to(np.asarray(phi, dtype=np.float64), theta.shape)
    S1, S2 = amplitudes(k * a, theta)
    return 4 * math.pi / k ** 2 * (np.cos(phi) ** 2 * np.abs(S2) ** 2 + np.sin(phi) ** 2 * np.abs(S1) ** 2)


def backscatter_normalised(ka: float) -> float:
    """sigma_back / (pi a^2)."""
    n, a, b = coefficients(ka)
    s = np.sum((2 * n + 1) * (-1.0) ** n * (a - b))
    return float(abs(s) ** 2 / ka ** 2)


def q_sca(ka: float) -> float:
    n, a, b = coefficients(ka)
    return float(2 / ka ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2)))


def q_ext(ka: float) -> float:
    n, a, b = coefficients(ka)
    return float(2 / ka ** 2 * np.sum((2 * n + 1) * np.real(a + b)))
