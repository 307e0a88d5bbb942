"""CPU FP64 oracle for the von Mises KDE hot path (test infrastructure).

This package is the plain, slow, obviously correct statement of what the
GPU library computes. It exists to check that library and is never part of
it: only the tests, the package's ``smoke()`` check and the benchmark's
``cpu_baseline`` timing may import it. It imports nothing from the GPU
package, and the GPU package imports nothing from it.

Everything is float64 NumPy/SciPy. Library routines serve as single steps
(``scipy.special.i0e``/``ive`` for Bessel functions, ``numpy.fft`` for the
periodic Poisson solve, ``numpy.sort``); everything else is the definition
written out, citing the paper's section and equation.

Notation used throughout (the paper states the kernel on the circle,
Eq. (vonMises); the domain of the PIC problem is [0, L)):

* ``theta = 2*pi*x/L`` maps a position to the circle.
* The kernel as a density in x is ``K_kappa(d) = exp(kappa*(cos(2*pi*d/L)-1))
  / (L * I0e(kappa))`` with ``I0e(k) = exp(-k) I0(k)``; the exponent is
  evaluated as ``-2*kappa*sin(pi*d/L)**2``.
* The grid has M nodes ``x_g = g*L/M`` and the density is the estimate
  evaluated at the nodes (Sec. III.A, finite-difference grid).

Submodules:

* ``vonmises`` -- wrap, kernel, its two-fold convolution, width <-> kappa.
* ``cv``       -- pair sums, the least-squares CV objective, argmin.
* ``density``  -- deposit, gather, pilot interpolation, adaptive widths.
* ``pic``      -- Poisson solve, centred field, leapfrog push, session step.
* ``adtest``   -- Anderson-Darling statistic and its asymptotic p-value.
* ``mise``     -- closed-form MISE from Fourier coefficients (CV pins).
* ``triangle`` -- first-order (triangular) kernel of adjustable width: the
  kernel, its two-fold convolution (a scaled cubic B-spline), pair sums,
  CV, deposit and gather.
* ``update``   -- the width-update rule of Sec. II.D.
* ``landau``   -- the standard-PIC (linear weighting) step, the field
  energy, the two-peak damping rate and the Landau root of the Maxwellian
  dispersion relation (Sec. III.B).
* ``refine``   -- the continuous minimiser of the CV objective inside the
  scan's bracket, and the exact pilot at the particles with the adaptive
  widths taken from it.
"""
from . import vonmises, cv, density, pic, adtest, update, mise, triangle, refine, landau  # noqa: F401
