"""Least-squares cross-validation objective (Sec. II.B, Eq. cv_def).

Test infrastructure: see the package docstring.

With ``n`` samples, the objective of Eq. (cv_def) with the kernel and its
two-fold convolution written as densities in x is

    CV(kappa) = (1/n^2) sum_{i,j} Kbar(X_i - X_j)
              - (2/(n(n-1))) sum_{i != j} K(X_i - X_j).

The first double sum keeps i = j (it is the integral of the squared
estimate); the second is the leave-one-out term and excludes it. Both are
symmetric in (i, j), so with the unordered sums

    S1 = sum_{i<j} Kbar(X_i - X_j),   S2 = sum_{i<j} K(X_i - X_j)

the objective is ``(n Kbar(0) + 2 S1)/n^2 - 4 S2/(n(n-1))``.
"""
from __future__ import annotations

import math

import numpy as np

from .vonmises import conv2, conv2_at_zero, kernel, bessel_ratio


def pair_sums_rows(x, L, kappas, i0, i1):
    """The part of the unordered pair sums with the first index in rows
    [i0, i1): ``(S1[b], S2[b])`` over the pairs i in [i0, i1), j in (i, n)."""
    x = np.asarray(x, dtype=np.float64)
    kappas = np.atleast_1d(np.asarray(kappas, dtype=np.float64))
    n = x.shape[0]
    S1 = np.zeros(kappas.shape[0])
    S2 = np.zeros(kappas.shape[0])
    xi = x[i0:i1, None]
    xj = x[None, i0:]
    d = xi - xj
    mask = (np.arange(i0, n)[None, :] > np.arange(i0, i1)[:, None])
    dd = d[mask]
    if dd.size == 0:
        return S1, S2
    for b, k in enumerate(kappas):
        S1[b] = conv2(dd, k, L).sum()
        S2[b] = kernel(dd, k, L).sum()
    return S1, S2


def pair_sums(x, L, kappas, block=256):
    """Direct unordered pair sums ``(S1[b], S2[b])`` over all i < j, for each
    candidate ``kappas[b]``. O(n^2) per kappa, in row blocks of ``block``
    rows, added in row order."""
    x = np.asarray(x, dtype=np.float64)
    kappas = np.atleast_1d(np.asarray(kappas, dtype=np.float64))
    n = x.shape[0]
    S1 = np.zeros(kappas.shape[0])
    S2 = np.zeros(kappas.shape[0])
    for i0 in range(0, n, block):
        s1, s2 = pair_sums_rows(x, L, kappas, i0, min(n, i0 + block))
        S1 += s1
        S2 += s2
    return S1, S2


def cv_from_sums(n, L, kappas, S1, S2):
    """Objective from the unordered pair sums (see module docstring)."""
    kappas = np.atleast_1d(np.asarray(kappas, dtype=np.float64))
    n = float(n)
    first = (n * conv2_at_zero(kappas, L) + 2.0 * np.asarray(S1)) / (n * n)
    second = 4.0 * np.asarray(S2) / (n * (n - 1.0))
    return first - second


def cv_curve(x, L, kappas):
    """``(cv[b], S1[b], S2[b])`` by direct pair sums."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape[0] < 2:
        raise ValueError("the leave-one-out term needs n >= 2")
    S1, S2 = pair_sums(x, L, kappas)
    return cv_from_sums(x.shape[0], L, kappas, S1, S2), S1, S2


def cv_argmin(cv):
    """Index of the smallest objective value; the smallest index on ties."""
    cv = np.asarray(cv)
    return int(np.flatnonzero(cv == cv.min())[0])


def fourier_moments(x, L, m_max, block=65536):
    """``c_m = (1/n) sum_j exp(i m theta_j)`` for m = 1..m_max (complex)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    th = (2.0 * math.pi / L) * x
    m = np.arange(1, m_max + 1, dtype=np.float64)
    acc = np.zeros(m_max, dtype=np.complex128)
    for j0 in range(0, n, block):
        ph = np.outer(th[j0:j0 + block], m)
        acc += np.cos(ph).sum(axis=0) + 1j * np.sin(ph).sum(axis=0)
    return acc / n


def pair_sums_fourier(x, L, kappas):
    """The same ``(S1, S2)`` through the Fourier series of the kernels.

    On the circle ``K(d) = (1/L)(1 + 2 sum_m rho_m cos(m dtheta))`` with
    ``rho_m = I_m(kappa)/I_0(kappa)``, and the convolution squares the
    coefficients. Summing over all ordered pairs turns ``cos(m dtheta)`` into
    ``n^2 |c_m|^2``; removing the diagonal and halving gives the unordered
    sums. The series is cut where ``rho_m < exp(-50)`` (m beyond
    ``10 sqrt(kappa) + 40``). O(n * m_max) instead of O(n^2).
    """
    x = np.asarray(x, dtype=np.float64)
    kappas = np.atleast_1d(np.asarray(kappas, dtype=np.float64))
    n = float(x.shape[0])
    m_max = int(math.ceil(10.0 * math.sqrt(float(kappas.max())) + 40.0))
    c = fourier_moments(x, L, m_max)
    p = np.abs(c) ** 2
    m = np.arange(1, m_max + 1)
    S1 = np.zeros(kappas.shape[0])
    S2 = np.zeros(kappas.shape[0])
    for b, k in enumerate(kappas):
        rho = bessel_ratio(m, k)
        all_kbar = (n * n / L) * (1.0 + 2.0 * np.sum(rho * rho * p))
        all_k = (n * n / L) * (1.0 + 2.0 * np.sum(rho * p))
        S1[b] = 0.5 * (all_kbar - n * conv2_at_zero(k, L))
        S2[b] = 0.5 * (all_k - n * kernel(0.0, k, L))
    return S1, S2


def cv_curve_fourier(x, L, kappas):
    """``(cv[b], S1[b], S2[b])`` through ``pair_sums_fourier``."""
    S1, S2 = pair_sums_fourier(x, L, kappas)
    return cv_from_sums(np.asarray(x).shape[0], L, kappas, S1, S2), S1, S2


def cv_without_leave_one_out(x, L, kappas):
    """The objective of Appendix A: the same as Eq. (cv_def) but with the
    second sum over all (i, j), i = j included, and 1/n^2 in front of both.
    Its diagonal part ``(Kbar(0) - 2 K(0))/n`` is negative and grows without
    bound as the kernel narrows, which is why the leave-one-out form is used.
    """
    x = np.asarray(x, dtype=np.float64)
    kappas = np.atleast_1d(np.asarray(kappas, dtype=np.float64))
    n = float(x.shape[0])
    S1, S2 = pair_sums(x, L, kappas)
    first = (n * conv2_at_zero(kappas, L) + 2.0 * S1) / (n * n)
    second = 2.0 * (n * kernel(0.0, kappas, L) + 2.0 * S2) / (n * n)
    return first - second
