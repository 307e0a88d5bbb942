"""Anderson-Darling test of uniform positions (Sec. II.D).

Test infrastructure: see the package docstring.

The width-update rule asks whether the particle positions are still
consistent with a uniform distribution on [0, L), using the
Anderson-Darling statistic and its p-value.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

_CLAMP = 2.0 ** -53


def ad_statistic(x, L):
    """``A^2 = -n - (1/n) sum_{k=1}^{n} (2k-1) [ln u_(k) + ln(1 - u_(n+1-k))]``
    for the sorted ``u = x/L`` (origin at x = 0), each clamped to
    [2^-53, 1 - 2^-53] so that the logarithms exist."""
    u = np.sort(np.asarray(x, dtype=np.float64) / L)
    u = np.clip(u, _CLAMP, 1.0 - _CLAMP)
    n = u.shape[0]
    k = np.arange(1, n + 1, dtype=np.float64)
    s = np.sum((2.0 * k - 1.0) * (np.log(u) + np.log1p(-u[::-1])))
    return -n - s / n


def _ad_cdf_term(j, z):
    """Term j of Anderson and Darling's series for the limiting law of A^2."""
    a = 4 * j + 1
    coef = special.binom(-0.5, j) * a * math.exp(-(a * a) * math.pi ** 2 / (8.0 * z))

    def integrand(w):
        return math.exp(z / (8.0 * (w * w + 1.0)) - (a * a) * math.pi ** 2 * w * w / (8.0 * z))

    val, _ = integrate.quad(integrand, 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=200)
    return coef * val


def ad_cdf(z, terms=40):
    """Limiting distribution ``P(A^2 <= z)`` of the statistic for a fully
    specified continuous law, from the series of Anderson and Darling (1954):

        (sqrt(2 pi)/z) sum_{j>=0} binom(-1/2, j) (4j+1) exp(-(4j+1)^2 pi^2/(8z))
            * int_0^inf exp(z/(8(w^2+1)) - (4j+1)^2 pi^2 w^2/(8z)) dw.
    """
    if z <= 0.0:
        return 0.0
    total = 0.0
    for j in range(terms):
        t = _ad_cdf_term(j, z)
        total += t
        if j > 3 and abs(t) < 1e-18:
            break
    return min(1.0, max(0.0, math.sqrt(2.0 * math.pi) / z * total))


def ad_pvalue(a2):
    """Upper-tail p-value ``1 - P(A^2 <= a2)`` under the limiting law."""
    return 1.0 - ad_cdf(float(a2))
