"""Von Mises kernel on a periodic domain (Sec. II.A, Eq. vonMises).

Test infrastructure: see the package docstring.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def wrap(x, L):
    """Map positions into [0, L): ``x - L*floor(x/L)``; a result equal to L
    (possible by rounding for tiny negative x) becomes 0."""
    x = np.asarray(x, dtype=np.float64)
    y = x - L * np.floor(x / L)
    return np.where(y >= L, 0.0, y)


def i0e(k):
    """Exponentially scaled modified Bessel function ``exp(-|k|) I0(k)``
    (the normaliser of Eq. vonMises), from SciPy."""
    return special.i0e(np.asarray(k, dtype=np.float64))


def bessel_ratio(m, k):
    """``I_m(k) / I_0(k)``: the m-th Fourier coefficient of the von Mises
    law (its characteristic function), from SciPy's scaled ``ive``."""
    k = np.asarray(k, dtype=np.float64)
    return special.ive(m, k) / special.ive(0, k)


def kernel(d, kappa, L):
    """``K_kappa(d)``: the von Mises density of Eq. (vonMises), centred at 0,
    written as a density in x on [0, L) (Jacobian 2*pi/L):

        K(d) = exp(-2 kappa sin^2(pi d / L)) / (L * I0e(kappa)).

    ``kappa`` may be a scalar or broadcast against ``d``. kappa = 0 gives the
    uniform density 1/L.
    """
    d = np.asarray(d, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    s = np.sin(math.pi * d / L)
    return np.exp(-2.0 * kappa * s * s) / (L * i0e(kappa))


def conv2(d, kappa, L):
    """Two-fold convolution ``Kbar(d) = int_0^L K(t - d) K(t) dt`` used by the
    first term of Eq. (cv_def).

    For the von Mises kernel the integral is closed form: the product of two
    von Mises exponentials centred a distance d apart is a von Mises
    exponential of concentration ``2 kappa |cos(pi d/L)|``, so

        Kbar(d) = I0(2 kappa c) / (L I0(kappa)^2),   c = |cos(pi d / L)|.

    It is evaluated without cancellation as

        exp(-2 kappa s^2 / (1 + c)) * I0e(2 kappa c) / (L I0e(kappa)^2),

    s = sin(pi d / L), using 1 - c = s^2 / (1 + c).
    """
    d = np.asarray(d, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    ang = math.pi * d / L
    s = np.sin(ang)
    c = np.abs(np.cos(ang))
    e = np.exp(-2.0 * kappa * s * s / (1.0 + c))
    ik = i0e(kappa)
    return e * i0e(2.0 * kappa * c) / (L * ik * ik)


def conv2_at_zero(kappa, L):
    """``Kbar(0) = I0e(2 kappa) / (L I0e(kappa)^2)``."""
    kappa = np.asarray(kappa, dtype=np.float64)
    ik = i0e(kappa)
    return i0e(2.0 * kappa) / (L * ik * ik)


def kappa_from_width(h, L):
    """Width h on [0, L) to concentration: ``1/kappa`` plays the role of the
    squared width on the circle (Sec. II.A), so ``kappa = (L / (2 pi h))^2``."""
    return (L / (2.0 * math.pi * np.asarray(h, dtype=np.float64))) ** 2


def width_from_kappa(kappa, L):
    """Inverse of ``kappa_from_width``: ``h = (L / 2 pi) / sqrt(kappa)``."""
    return (L / (2.0 * math.pi)) / np.sqrt(np.asarray(kappa, dtype=np.float64))
