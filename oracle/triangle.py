"""First-order (triangular) kernel of adjustable width on a periodic domain.

Test infrastructure: see the package docstring.

Standard PIC weights a particle onto the grid with a triangle whose total
width is twice the grid spacing (first-order weighting, Sec. I); the paper's
cheapest accurate strategy keeps that shape and chooses its width by the
least-squares CV objective (Sec. IV, the comparison of shapes and costs).
Here the width is the half-width h of the support, 0 < h <= L/2, so that
the support never meets its own periodic image; standard PIC is h = dx.

* Kernel:      T_h(d) = (1/h) max(0, 1 - |d|/h), |d| the periodic distance.
* Convolution: T_h is the self-convolution of a box of width h, so the
  two-fold convolution that enters the first CV term is the four-fold
  convolution of that box, the centred cubic B-spline B scaled to h:

      Tbar_h(d) = (1/h) sum_k B((d + k L) / h),
      B(u) = 2/3 - u^2 + |u|^3/2   for |u| <= 1,
             (2 - |u|)^3 / 6        for 1 <= |u| <= 2,
             0                      otherwise.

  With h <= L/2 the support of B(./h) is shorter than L, so for d in
  [0, L/2] only the images d and L - d can contribute.
* Fourier coefficients (for the MISE pin): the box of width h has
  coefficient sin(pi m h / L) / (pi m h / L), so T_h has its square.

The CV objective, its pair sums and its argmin are those of ``cv`` with T
and Tbar in place of the von Mises kernel and its convolution.
"""
from __future__ import annotations

import math

import numpy as np


def periodic_distance(d, L):
    """Distance on the circle of length L: ``min(|d| mod L, L - |d| mod L)``."""
    d = np.abs(np.asarray(d, dtype=np.float64)) % L
    return np.minimum(d, L - d)


def check_width(h, L):
    h = np.asarray(h, dtype=np.float64)
    if np.any(~np.isfinite(h)) or np.any(h <= 0.0) or np.any(h > 0.5 * L):
        raise ValueError("half-widths must lie in (0, L/2]")
    return h


def kernel(d, h, L):
    """``T_h(d) = max(0, 1 - |d|/h) / h`` at the periodic distance."""
    h = check_width(h, L)
    r = periodic_distance(d, L)
    return np.maximum(0.0, 1.0 - r / h) / h


def bspline3(u):
    """The centred cubic B-spline, piece by piece (the textbook form)."""
    a = np.abs(np.asarray(u, dtype=np.float64))
    out = np.zeros_like(a)
    inner = a <= 1.0
    outer = (a > 1.0) & (a < 2.0)
    out[inner] = 2.0 / 3.0 - a[inner] ** 2 + 0.5 * a[inner] ** 3
    out[outer] = (2.0 - a[outer]) ** 3 / 6.0
    return out


def conv2(d, h, L):
    """``Tbar_h(d) = int_0^L T_h(t - d) T_h(t) dt``: the scaled cubic B-spline
    at the periodic distance r and at its image L - r."""
    h = check_width(h, L)
    r = periodic_distance(d, L)
    return (bspline3(r / h) + bspline3((L - r) / h)) / h


def conv2_at_zero(h, L):
    """``Tbar_h(0) = (B(0) + B(L/h)) / h = 2 / (3 h)`` (B(L/h) = 0 for h <= L/2)."""
    h = check_width(h, L)
    return (bspline3(np.zeros_like(h)) + bspline3(L / h)) / h


def fourier_coeffs(m, h, L):
    """``rho_m = (sin(pi m h / L) / (pi m h / L))^2`` for m >= 1."""
    z = math.pi * np.asarray(m, dtype=np.float64) * float(h) / L
    return (np.sin(z) / z) ** 2


def pair_sums(x, L, widths, block=256):
    """Direct unordered pair sums ``(S1[b], S2[b]) = (sum_{i<j} Tbar, sum_{i<j} T)``
    for each half-width ``widths[b]``."""
    x = np.asarray(x, dtype=np.float64)
    widths = np.atleast_1d(check_width(widths, L))
    n = x.shape[0]
    S1 = np.zeros(widths.shape[0])
    S2 = np.zeros(widths.shape[0])
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        d = x[i0:i1, None] - x[None, i0:]
        rows = np.arange(i0, i1)[:, None]
        cols = np.arange(i0, n)[None, :]
        upper = cols > rows
        r = periodic_distance(d, L)[upper]
        for b, h in enumerate(widths):
            S1[b] += float(np.sum(conv2(r, h, L)))
            S2[b] += float(np.sum(kernel(r, h, L)))
    return S1, S2


def cv_from_sums(n, L, widths, S1, S2):
    """``(n Tbar(0) + 2 S1)/n^2 - 4 S2/(n (n - 1))`` (Eq. cv_def with T)."""
    widths = np.atleast_1d(np.asarray(widths, dtype=np.float64))
    n = float(n)
    first = (n * conv2_at_zero(widths, L) + 2.0 * np.asarray(S1)) / (n * n)
    second = 4.0 * np.asarray(S2) / (n * (n - 1.0))
    return first - second


def cv_curve(x, L, widths):
    """``(cv[b], S1[b], S2[b])`` by direct pair sums."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape[0] < 2:
        raise ValueError("the leave-one-out term needs n >= 2")
    S1, S2 = pair_sums(x, L, widths)
    return cv_from_sums(x.shape[0], L, widths, S1, S2), S1, S2


def deposit(x, L, M, h=None, h_i=None, block=4096):
    """``rho_g = (1/N) sum_i T_{h_i}(x_g - x_i)`` at the nodes ``x_g = g L / M``,
    with one half-width ``h`` or per-particle ``h_i``."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    hh = np.full(n, float(h)) if h_i is None else np.asarray(h_i, dtype=np.float64)
    check_width(hh, L)
    g = np.arange(M) * (L / M)
    rho = np.zeros(M)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        rho += np.sum(kernel(g[:, None] - x[None, i0:i1], hh[None, i0:i1], L), axis=1)
    return rho / n


def gather(x, L, field, h=None, h_i=None):
    """``G_i = dx sum_g F_g T_{h_i}(x_g - x_i)``."""
    x = np.asarray(x, dtype=np.float64)
    field = np.asarray(field, dtype=np.float64)
    M = field.shape[0]
    n = x.shape[0]
    hh = np.full(n, float(h)) if h_i is None else np.asarray(h_i, dtype=np.float64)
    check_width(hh, L)
    g = np.arange(M) * (L / M)
    w = kernel(g[None, :] - x[:, None], hh[:, None], L)
    return (L / M) * (w @ field)
