"""Landau damping with standard PIC and with the KDE density (Sec. III.B).

Test infrastructure: see the package docstring.

* Standard PIC weights particles to the grid and the field back with the
  first-order (linear, "cloud-in-cell") shape: the triangle of half-width
  one cell (``triangle`` with h = dx). One step is the cycle of
  Sec. III.A with that shape in place of the von Mises kernel.
* The electric field energy at a step is ``W = (dx / 2) sum_g E_g^2``
  (eps0 = 1: the energy density E^2 / 2 integrated by the grid's
  rectangle rule, exact for the grid's trigonometric modes).
* The damping rate is read off the logarithm of W as the paper does: the
  slope of the line through the first two peaks after t = 0. A peak is a
  step n >= 1 with ``W[n-1] < W[n] >= W[n+1]``. The energy decays at twice
  the rate of the field amplitude, so this slope is 2 Im(omega).
* The theory is the root of the Vlasov-Poisson dispersion relation for a
  Maxwellian of thermal velocity v_th (plasma frequency 1):
  ``1 + (1 + zeta Z(zeta)) / (k v_th)^2 = 0``, ``zeta = omega / (sqrt(2) k v_th)``,
  with the plasma dispersion function ``Z(zeta) = i sqrt(pi) w(zeta)`` (SciPy's
  Faddeeva function w as the library step), solved by Newton's method. Only
  k v_th matters; the root is followed by continuation in k v_th from 0.2
  (started at the Bohm-Gross frequency, where the damping is negligible),
  since Newton from that start alone diverges once the damping is strong.
* A smoothing kernel used for both the deposit and the gather multiplies
  the force of mode k by the square of its Fourier coefficient, rho_1^2 for
  the von Mises kernel of concentration kappa at the box's fundamental
  mode (rho_1 = I_1/I_0). The mode then obeys the same relation with the
  susceptibility scaled by s = rho_1^2, ``1 + s (1 + zeta Z) / (k v_th)^2``,
  followed by continuation in s from 1 (``response``).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import triangle
from .pic import charge_from_density, efield_centered, poisson_fd, push


def field_step_standard(x, v, L, M, dt):
    """One standard-PIC step: linear weighting (half-width dx) for the
    deposit and the gather; Poisson, field and push as ``pic.field_step``.
    Returns ``(x_new, v_new, rho, E_grid)``."""
    dx = L / M
    rho = triangle.deposit(x, L, M, h=dx)
    phi = poisson_fd(charge_from_density(rho, L), dx)
    E = efield_centered(phi, dx)
    E_i = triangle.gather(x, L, E, h=dx)
    x_new, v_new = push(x, v, E_i, dt, L)
    return x_new, v_new, rho, E


def field_energy(E, L):
    """``W = (dx / 2) sum_g E_g^2``."""
    E = np.asarray(E, dtype=np.float64)
    return 0.5 * (L / E.shape[0]) * float(np.sum(E * E))


def first_two_peaks(W):
    """Indices of the first two local maxima of W after index 0, or None."""
    W = np.asarray(W, dtype=np.float64)
    peaks = []
    for n in range(1, W.shape[0] - 1):
        if W[n - 1] < W[n] >= W[n + 1]:
            peaks.append(n)
            if len(peaks) == 2:
                return peaks
    return None


def damping_rate(W, dt):
    """Slope of log W through its first two peaks after t = 0; NaN when
    there are fewer than two."""
    p = first_two_peaks(W)
    if p is None:
        return float("nan")
    W = np.asarray(W, dtype=np.float64)
    return (math.log(W[p[1]]) - math.log(W[p[0]])) / ((p[1] - p[0]) * dt)


def dispersion(omega, k, v_th, response=1.0):
    """``1 + s (1 + zeta Z(zeta)) / (k v_th)^2`` at complex omega, s = response."""
    zeta = omega / (math.sqrt(2.0) * k * v_th)
    Z = 1j * math.sqrt(math.pi) * special.wofz(zeta)
    return 1.0 + response * (1.0 + zeta * Z) / (k * v_th) ** 2


def _newton(w, kv, tol, resp=1.0):
    s = math.sqrt(2.0) * kv
    for _ in range(100):
        zeta = w / s
        Z = 1j * math.sqrt(math.pi) * special.wofz(zeta)
        f = 1.0 + resp * (1.0 + zeta * Z) / (kv * kv)
        dZ = -2.0 * (1.0 + zeta * Z)
        df = resp * (Z + zeta * dZ) / (kv * kv * s)
        step = f / df
        w -= step
        if abs(step) < tol * abs(w):
            break
    return w


def landau_root(k, v_th, response=1.0, tol=1e-14):
    """Least-damped root omega = omega_r + i gamma (gamma < 0) of
    ``dispersion``: Newton's method on the analytic function (derivative by
    Z'(zeta) = -2 (1 + zeta Z(zeta))), continued in k v_th from 0.2, then in
    the response from 1."""
    target = k * v_th
    kv = min(0.2, target)
    w = _newton(complex(math.sqrt(1.0 + 3.0 * kv * kv), 0.0), kv, tol)
    while kv < target:
        kv = min(target, kv + 0.02)
        w = _newton(w, kv, tol)
    for s in np.linspace(1.0, response, 41)[1:]:
        w = _newton(w, target, tol, float(s))
    return w


def kernel_response(kappa):
    """``rho_1(kappa)^2``: the factor a von Mises kernel of concentration
    kappa, used for the deposit and the gather, puts on the fundamental
    mode's force (SciPy's scaled Bessel functions)."""
    r1 = special.i1e(kappa) / special.i0e(kappa)
    return float(r1 * r1)
