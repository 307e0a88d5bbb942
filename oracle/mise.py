"""Closed-form MISE of the von Mises KDE (Sec. II.B, Eq. MISE).

Test infrastructure: see the package docstring. These formulas serve the
pins of the CV objective: Eq. (cv_def) plus the integral of f^2 is an
unbiased estimate of the MISE (Sec. II.B), so the seed-average of the CV
objective can be compared with the exact MISE of a known density.

For a density on [0, L) with Fourier coefficients ``f_m = E[exp(-i m Theta)]``
(so ``f(x) = (1/L) sum_m f_m exp(i m theta)``) and the von Mises kernel with
coefficients ``rho_m = I_m(kappa)/I_0(kappa)``, the estimate from n
independent samples has coefficients ``rho_m c_m`` with
``E c_m = f_m`` and ``E |c_m - f_m|^2 = (1 - |f_m|^2)/n``, hence

    MISE = (2/L) sum_{m>=1} [ |f_m|^2 (1 - rho_m)^2 + rho_m^2 (1 - |f_m|^2)/n ].

The same holds for any kernel, with its own coefficients in place of
``rho_m`` (``mise_from_coeffs``; the triangle of ``triangle`` has
``rho_m = sinc^2(pi m h / L)``).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize

from .vonmises import bessel_ratio


def mise(kappa, n, L, f_coeffs):
    """Exact MISE for true coefficients ``f_coeffs[m-1] = |f_m|`` (m >= 1;
    coefficients beyond the array are zero)."""
    a = np.asarray(f_coeffs, dtype=np.float64)
    m_max = max(len(a), int(math.ceil(10.0 * math.sqrt(float(kappa)) + 40.0)))
    m = np.arange(1, m_max + 1)
    rho = bessel_ratio(m, float(kappa))
    aa = np.zeros(m_max)
    aa[:len(a)] = a
    return (2.0 / L) * float(np.sum(aa * aa * (1.0 - rho) ** 2 + rho * rho * (1.0 - aa * aa) / n))


def mise_from_coeffs(rho, n, L, f_coeffs):
    """The same MISE for any kernel with Fourier coefficients ``rho[m-1]``
    (m = 1..len(rho); the kernel's coefficients beyond are taken as zero,
    so ``rho`` must run until they are negligible)."""
    rho = np.asarray(rho, dtype=np.float64)
    a = np.asarray(f_coeffs, dtype=np.float64)
    aa = np.zeros(max(len(rho), len(a)))
    aa[:len(a)] = a
    rr = np.zeros_like(aa)
    rr[:len(rho)] = rho
    return (2.0 / L) * float(np.sum(aa * aa * (1.0 - rr) ** 2 + rr * rr * (1.0 - aa * aa) / n))


def int_f_squared(L, f_coeffs):
    """``int f^2 = (1/L)(1 + 2 sum |f_m|^2)``."""
    a = np.asarray(f_coeffs, dtype=np.float64)
    return (1.0 + 2.0 * float(np.sum(a * a))) / L


def expected_cv(kappa, n, L, f_coeffs):
    """``E[CV(kappa)] = MISE(kappa) - int f^2``."""
    return mise(kappa, n, L, f_coeffs) - int_f_squared(L, f_coeffs)


def cosine_coeffs(alpha):
    """Coefficients of ``(1 + alpha cos theta)/L``: only ``|f_1| = alpha/2``."""
    return np.array([alpha / 2.0])


def vonmises_coeffs(kappa_f, m_max=None):
    """Coefficients of a von Mises truth VM(mu, kappa_f): ``I_m/I_0(kappa_f)``."""
    if m_max is None:
        m_max = int(math.ceil(10.0 * math.sqrt(kappa_f) + 40.0))
    return bessel_ratio(np.arange(1, m_max + 1), float(kappa_f))


def kappa_opt(n, L, f_coeffs, lo=1e-3, hi=1e7):
    """The concentration that minimises the exact MISE (bounded search on
    log kappa)."""
    res = optimize.minimize_scalar(lambda t: mise(math.exp(t), n, L, f_coeffs),
                                   bounds=(math.log(lo), math.log(hi)), method="bounded",
                                   options={"xatol": 1e-9})
    return math.exp(res.x)
