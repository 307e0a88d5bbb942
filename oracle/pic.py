"""One electrostatic PIC step with a KDE density (Sec. III.A).

Test infrastructure: see the package docstring.

Units follow the Birdsall convention the paper adopts (Sec. III.A): the
plasma frequency is 1 and e = m = eps0 = 1, with a uniform neutralising ion
background of density 1. Electrons carry charge -1.
"""
from __future__ import annotations

import math

import numpy as np

from .vonmises import wrap
from .density import deposit, gather


def charge_from_density(rho, L):
    """Electron number density ``n_e = L * rho`` (rho integrates to ~1 over
    [0, L), so the mean number density is 1) and net charge ``1 - n_e``."""
    return 1.0 - L * np.asarray(rho, dtype=np.float64)


def poisson_fd(rho_q, dx):
    """Solve the three-point periodic finite-difference Poisson equation of
    Sec. III.A, ``(phi[j-1] - 2 phi[j] + phi[j+1]) / dx^2 = -rho_q[j]``,
    exactly by the discrete Fourier transform: the stencil multiplies mode m
    by ``-(2 - 2 cos(2 pi m / M)) / dx^2``. The mean (m = 0) is not
    determined by a periodic problem and is set to zero, which also drops
    any net charge."""
    rho_q = np.asarray(rho_q, dtype=np.float64)
    M = rho_q.shape[0]
    rh = np.fft.fft(rho_q)
    m = np.arange(M)
    denom = 2.0 - 2.0 * np.cos(2.0 * math.pi * m / M)
    ph = np.zeros(M, dtype=np.complex128)
    ph[1:] = rh[1:] * dx * dx / denom[1:]
    return np.real(np.fft.ifft(ph))


def efield_centered(phi, dx):
    """Centred difference ``E_j = (phi[j-1] - phi[j+1]) / (2 dx)`` (Sec. III.A)."""
    phi = np.asarray(phi, dtype=np.float64)
    return (np.roll(phi, 1) - np.roll(phi, -1)) / (2.0 * dx)


def push(x, v, E_i, dt, L):
    """Leapfrog step as discretised in Sec. III.A, for electrons (q/m = -1):
    ``v <- v - E_i dt`` then ``x <- x + v dt``, then wrap into [0, L)."""
    v_new = np.asarray(v, dtype=np.float64) - np.asarray(E_i, dtype=np.float64) * dt
    x_new = wrap(np.asarray(x, dtype=np.float64) + v_new * dt, L)
    return x_new, v_new


def field_step(x, v, kappa_i, L, M, dt):
    """The deposit -> Poisson -> field -> gather -> push part of one step.

    Returns ``(x_new, v_new, rho, E_grid)`` where rho is the deposited
    probability density and E_grid the field on the nodes."""
    dx = L / M
    rho = deposit(x, L, M, kappa_i=kappa_i)
    phi = poisson_fd(charge_from_density(rho, L), dx)
    E = efield_centered(phi, dx)
    E_i = gather(x, L, E, kappa_i=kappa_i)
    x_new, v_new = push(x, v, E_i, dt, L)
    return x_new, v_new, rho, E
