"""Continuous minimisation of the CV objective and the exact pilot at the
particles (Sec. II.B, the minimiser of Eq. cv_def; Sec. II.C, the pilot
estimate of the adaptive widths).

Test infrastructure: see the package docstring.

* The paper minimises the CV objective over the width with a Newton-type
  method. Here the minimiser is taken inside the bracket that a scan over a
  list of concentrations finds: with b* the first minimum of the list, the
  search runs over u = log(kappa) between the list's neighbours of b*
  (b* - 1 and b* + 1, clipped to the list), and the objective is the plain
  direct-sum definition (``cv.cv_curve``) at each trial kappa. The 1D
  search itself is a library step (SciPy's bounded Brent method).
* The pilot of Silverman's adaptive estimate is the fixed-width estimate
  itself; evaluated exactly at the particles it is
  ``f_i = (1/n) sum_j K_kappa(X_i - X_j)``, all j including i (the estimate
  at a sample point), instead of an interpolation of its grid values.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize

from . import cv as _cv
from .vonmises import kernel


def cv_at(x, L, kappa):
    """The objective of Eq. (cv_def) at one concentration, by direct sums."""
    return float(_cv.cv_curve(x, L, [float(kappa)])[0][0])


def bracket(kappas, b):
    """Concentrations around list index ``b``: ``(kappas[b-1], kappas[b+1])``
    clipped to the list."""
    k = np.asarray(kappas, dtype=np.float64)
    return float(k[max(b - 1, 0)]), float(k[min(b + 1, k.shape[0] - 1)])


def cv_minimise(x, L, kappas, xatol=1e-11):
    """Scan ``kappas`` (ascending), then minimise the objective over
    log(kappa) inside the bracket of the scan's first minimum.

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
    res = optimize.minimize_scalar(lambda u: cv_at(x, L, math.exp(u)), bounds=(math.log(lo), math.log(hi)),
                                   method="bounded", options={"xatol": xatol, "maxiter": 500})
    k = math.exp(res.x)
    val = cv_at(x, L, k)
    # the bounded search may stop short of an end point that is lower
    for e in (lo, hi):
        ve = cv_at(x, L, e)
        if ve < val:
            k, val = e, ve
    return k, val, b, (lo, hi)


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
