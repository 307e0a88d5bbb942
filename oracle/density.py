"""Deposit, gather and particle-wise adaptive widths (Sec. II.B Eq. kde,
Sec. II.C Eq. adaptive_width, Sec. III.A).

Test infrastructure: see the package docstring.
"""
from __future__ import annotations

import numpy as np

from .vonmises import kernel


def grid_nodes(L, M):
    """Node positions ``x_g = g L / M``, g = 0..M-1 (the finite-difference
    grid of Sec. III.A)."""
    return np.arange(M, dtype=np.float64) * (L / M)


def _per_particle_kappa(n, kappa, kappa_i):
    if kappa_i is None:
        return np.full(n, float(kappa))
    k = np.asarray(kappa_i, dtype=np.float64)
    if k.shape != (n,):
        raise ValueError("kappa_i must have one value per particle")
    return k


def deposit(x, L, M, kappa=None, kappa_i=None, block=4096):
    """Kernel density estimate at the grid nodes, Eq. (kde) with each
    particle's own normalised kernel (the adaptive estimate of Sec. II.C,
    step 3; a global kappa is the special case of equal widths):

        rho_g = (1/n) sum_i K_{kappa_i}(x_g - X_i).

    The result is a probability density (integral close to 1).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    k = _per_particle_kappa(n, kappa, kappa_i)
    xg = grid_nodes(L, M)
    rho = np.zeros(M)
    for i0 in range(0, n, block):
        d = xg[:, None] - x[None, i0:i0 + block]
        rho += kernel(d, k[None, i0:i0 + block], L).sum(axis=1)
    return rho / n


def gather(x, L, field, kappa=None, kappa_i=None, block=4096):
    """Interpolate a grid field back to the particles with the same kernel:

        G_i = dx * sum_g F_g K_{kappa_i}(x_g - X_i),  dx = L / M.

    This is the adjoint of ``deposit``: ``dx * sum_g F_g rho_g = mean_i G_i``.
    """
    x = np.asarray(x, dtype=np.float64)
    F = np.asarray(field, dtype=np.float64)
    M = F.shape[0]
    n = x.shape[0]
    k = _per_particle_kappa(n, kappa, kappa_i)
    xg = grid_nodes(L, M)
    out = np.empty(n)
    for i0 in range(0, n, block):
        d = xg[None, :] - x[i0:i0 + block, None]
        out[i0:i0 + block] = (kernel(d, k[i0:i0 + block, None], L) * F[None, :]).sum(axis=1)
    return out * (L / M)


def pilot_at_particles(x, L, pilot):
    """Pilot density at each particle by periodic linear interpolation of the
    pilot grid: with j = floor(x/dx) and t = x/dx - j,
    ``(1-t) pilot[j] + t pilot[(j+1) mod M]``."""
    x = np.asarray(x, dtype=np.float64)
    p = np.asarray(pilot, dtype=np.float64)
    M = p.shape[0]
    u = x / (L / M)
    j = np.floor(u).astype(np.int64)
    t = u - j
    j = np.mod(j, M)
    return (1.0 - t) * p[j] + t * p[(j + 1) % M]


def adapt_widths(x, L, pilot, kappa_star, alpha=0.5, floor=np.finfo(np.float64).tiny):
    """Silverman's particle-wise widths (Sec. II.C), in concentration form.

    1. ``f_i`` = pilot density at particle i (``pilot_at_particles``),
       floored at ``floor`` (the smallest positive normal number) so that its
       logarithm exists; the number of floored particles is returned.
    2. ``log g = mean_i log f_i`` (geometric mean, Sec. II.C step 2).
    3. The width factor ``lambda_i = (f_i/g)^(-alpha)`` multiplies the CV width
       h; with ``kappa = (L/(2 pi h))^2`` this is
       ``kappa_i = kappa_star * (f_i/g)^(2 alpha)``.

    Returns ``(kappa_i, log_g, n_floored)``.
    """
    f = pilot_at_particles(x, L, pilot)
    n_floored = int(np.count_nonzero(f < floor))
    f = np.maximum(f, floor)
    lf = np.log(f)
    log_g = float(np.mean(lf))
    kappa_i = float(kappa_star) * np.exp(2.0 * alpha * (lf - log_g))
    return kappa_i, log_g, n_floored
