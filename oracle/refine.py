"""Continuous minimisation of the CV objective and the exact pilot at the
particles (Sec. II.B, the minimiser of Eq. cv_def; Sec. II.C, the pilot
estimate of the adaptive widths).

Test infrastructure: see the package docstring.

* The paper minimises the CV objective over the width with a Newton-type
  method. Here the minimiser is taken inside the bracket that a scan over a
  list of concentrations finds: with b* the first minimum of the list, the
  search runs over u = log(kappa) between the list's neighbours of b*
  (b* - 1 and b* + 1, clipped to the list). The minimiser is the
  stationary point of the objective there: the root of dCV/du, with the
  derivative written out by direct sums over the pairs (``cv_slope``; the
  kernels' kappa-derivatives are closed forms in I1/I0). The root search is
  a library step (SciPy's brentq). Where dCV/du keeps one sign over the
  bracket, the minimiser is the end with the lower objective.
* The pilot of Silverman's adaptive estimate is the fixed-width estimate
  itself; evaluated exactly at the particles it is
  ``f_i = (1/n) sum_j K_kappa(X_i - X_j)``, all j including i (the estimate
  at a sample point), instead of an interpolation of its grid values.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize, special

from . import cv as _cv
from .vonmises import conv2, conv2_at_zero, kernel


def cv_at(x, L, kappa):
    """The objective of Eq. (cv_def) at one concentration, by direct sums."""
    return float(_cv.cv_curve(x, L, [float(kappa)])[0][0])


def _ratio1(z):
    """I1(z) / I0(z) (SciPy's scaled Bessel functions)."""
    z = np.asarray(z, dtype=np.float64)
    return special.i1e(z) / special.i0e(z)


def cv_slope(x, L, kappa, block=256):
    """``dCV/du`` at ``u = log(kappa)``, by direct sums of the derivatives.

    With K = exp(-2 kappa s^2) / (L I0e(kappa)) and
    Kbar = I0(2 kappa c) / (L I0(kappa)^2) (s, c as in ``vonmises``):

        dK/dkappa    = K (1 - 2 s^2 - I1(kappa)/I0(kappa)),
        dKbar/dkappa = Kbar (2 c I1(2 kappa c)/I0(2 kappa c) - 2 I1(kappa)/I0(kappa)),

    and dCV/dkappa is Eq. (cv_def) with each kernel replaced by its
    derivative (the i = j term of the first sum included)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    k = float(kappa)
    r1 = float(_ratio1(k))
    dk_bar0 = float(conv2_at_zero(k, L)) * (2.0 * float(_ratio1(2.0 * k)) - 2.0 * r1)
    s1 = 0.0
    s2 = 0.0
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        d = x[i0:i1, None] - x[None, i0:]
        mask = np.arange(i0, n)[None, :] > np.arange(i0, i1)[:, None]
        dd = d[mask]
        if dd.size == 0:
            continue
        ang = math.pi * dd / L
        s = np.sin(ang)
        c = np.abs(np.cos(ang))
        s1 += float(np.sum(conv2(dd, k, L) * (2.0 * c * _ratio1(2.0 * k * c) - 2.0 * r1)))
        s2 += float(np.sum(kernel(dd, k, L) * (1.0 - 2.0 * s * s - r1)))
    dcv = (n * dk_bar0 + 2.0 * s1) / (n * n) - 4.0 * s2 / (n * (n - 1.0))
    return k * dcv


def bracket(kappas, b):
    """Concentrations around list index ``b``: ``(kappas[b-1], kappas[b+1])``
    clipped to the list."""
    k = np.asarray(kappas, dtype=np.float64)
    return float(k[max(b - 1, 0)]), float(k[min(b + 1, k.shape[0] - 1)])


def cv_minimise(x, L, kappas, xtol=1e-14):
    """Scan ``kappas`` (ascending), then find the stationary point of the
    objective in log(kappa) inside the bracket of the scan's first minimum
    (see the module docstring).

    Returns ``(kappa_min, cv_min, b_star, (lo, hi))``. A concentration of 0
    in the bracket is replaced by the smallest positive list value (log
    scale)."""
    x = np.asarray(x, dtype=np.float64)
    kappas = np.asarray(kappas, dtype=np.float64)
    grid, _, _ = _cv.cv_curve(x, L, kappas)
    b = _cv.cv_argmin(grid)
    lo, hi = bracket(kappas, b)
    if lo <= 0.0:
        lo = float(kappas[kappas > 0.0].min())
    if hi <= lo:
        return float(kappas[b]), float(grid[b]), b, (lo, hi)
    ua, ub = math.log(lo), math.log(hi)
    ga, gb = cv_slope(x, L, lo), cv_slope(x, L, hi)
    if ga < 0.0 < gb:
        u = optimize.brentq(lambda t: cv_slope(x, L, math.exp(t)), ua, ub, xtol=xtol, rtol=4 * np.finfo(float).eps,
                            maxiter=200)
        k = math.exp(u)
        return k, cv_at(x, L, k), b, (lo, hi)
    va, vb = cv_at(x, L, lo), cv_at(x, L, hi)
    return (lo, va, b, (lo, hi)) if va <= vb else (hi, vb, b, (lo, hi))


def pilot_exact(x, L, kappa, block=2048):
    """``f_i = (1/n) sum_j K_kappa(X_i - X_j)`` over all j (direct sums)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    out = np.empty(n)
    for i0 in range(0, n, block):
        d = x[i0:i0 + block, None] - x[None, :]
        out[i0:i0 + block] = kernel(d, float(kappa), L).sum(axis=1)
    return out / n


def adapt_widths_exact(x, L, kappa_star, alpha=0.5, floor=np.finfo(np.float64).tiny):
    """Particle-wise concentrations from the exact pilot at the particles:
    the steps of ``density.adapt_widths`` with ``f_i = pilot_exact(x, L,
    kappa_star)`` in place of the grid interpolation. Returns
    ``(kappa_i, log_g, n_floored)``."""
    f = pilot_exact(x, L, kappa_star)
    n_floored = int(np.count_nonzero(f < floor))
    f = np.maximum(f, floor)
    lf = np.log(f)
    log_g = float(np.mean(lf))
    return float(kappa_star) * np.exp(2.0 * alpha * (lf - log_g)), log_g, n_floored
