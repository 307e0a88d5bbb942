"""Planted mistakes in the oracle (CPU only): each plausible slip must make
one of the pins fail. The mutants are patched into the oracle for the
duration of one test and the corresponding pin is run against them."""
import math

import numpy as np
import pytest

from oracle import cv, density, vonmises as vm
import tests.test_oracle_cv as pins_cv
import tests.test_oracle_kernel as pins_k
import tests.test_oracle_adapt_pic as pins_a


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_dropped_half_angle_denominator_in_conv2(monkeypatch):
    def bad(d, kappa, L):
        ang = math.pi * np.asarray(d) / L
        s, c = np.sin(ang), np.abs(np.cos(ang))
        ik = vm.i0e(kappa)
        return np.exp(-2 * kappa * s * s) * vm.i0e(2 * kappa * c) / (L * ik * ik)
    monkeypatch.setattr(vm, "conv2", bad)
    monkeypatch.setattr(pins_k.vm, "conv2", bad)
    assert _fails(pins_k.test_conv2_equals_quadrature, 37.0, 0.25)


def test_signed_cosine_in_conv2(monkeypatch):
    def bad(d, kappa, L):
        ang = math.pi * np.asarray(d) / L
        s, c = np.sin(ang), np.cos(ang)
        ik = vm.i0e(kappa)
        return np.exp(-2 * kappa * s * s / (1 + c)) * vm.i0e(2 * kappa * np.abs(c)) / (L * ik * ik)
    monkeypatch.setattr(pins_k.vm, "conv2", bad)
    assert _fails(pins_k.test_conv2_equals_quadrature, 5.0, 0.77)


def test_full_angle_in_kernel(monkeypatch):
    def bad(d, kappa, L):
        s = np.sin(2 * math.pi * np.asarray(d) / L)
        return np.exp(-2.0 * kappa * s * s) / (L * vm.i0e(kappa))
    monkeypatch.setattr(pins_k.vm, "kernel", bad)
    assert _fails(pins_k.test_kernel_is_scipy_von_mises_law, 4.0)


def test_n_squared_in_leave_one_out_term(monkeypatch):
    orig = cv.cv_from_sums

    def bad(n, L, kappas, S1, S2):
        from oracle.vonmises import conv2_at_zero
        n = float(n)
        return (n * conv2_at_zero(np.atleast_1d(kappas), L) + 2 * np.asarray(S1)) / n ** 2 \
            - 4 * np.asarray(S2) / (n * n)
    monkeypatch.setattr(cv, "cv_from_sums", bad)
    assert _fails(pins_cv.test_two_particles_closed_form)
    monkeypatch.setattr(cv, "cv_from_sums", orig)


def test_missing_diagonal_in_first_term(monkeypatch):
    def bad(n, L, kappas, S1, S2):
        n = float(n)
        return 2 * np.asarray(S1) / n ** 2 - 4 * np.asarray(S2) / (n * (n - 1))
    monkeypatch.setattr(cv, "cv_from_sums", bad)
    assert _fails(pins_cv.test_uniform_kernel_limit)


def test_pair_sum_off_by_one_row(monkeypatch):
    def bad(x, L, kappas, block=256):
        x = np.asarray(x, dtype=np.float64)
        return cv.pair_sums.__wrapped__(x[1:], L, kappas) if hasattr(cv.pair_sums, "__wrapped__") \
            else _orig_pair_sums(x[1:], L, kappas)
    global _orig_pair_sums
    _orig_pair_sums = cv.pair_sums
    monkeypatch.setattr(cv, "pair_sums", bad)
    assert _fails(pins_cv.test_fourier_identity_matches_direct_sums, 50)


def test_wrong_adapt_exponent(monkeypatch):
    orig = density.adapt_widths

    def bad(x, L, pilot, kappa_star, alpha=0.5, floor=np.finfo(np.float64).tiny):
        return orig(x, L, pilot, kappa_star, -alpha, floor)
    monkeypatch.setattr(density, "adapt_widths", bad)
    assert _fails(pins_a.test_adapt_invariants)


def test_transposed_gather(monkeypatch):
    def bad(x, L, field, kappa=None, kappa_i=None, block=4096):
        F = np.asarray(field)[::-1]
        return _orig_gather(x, L, F, kappa=kappa, kappa_i=kappa_i)
    global _orig_gather
    _orig_gather = density.gather
    monkeypatch.setattr(density, "gather", bad)
    assert _fails(pins_k.test_gather_is_adjoint_of_deposit, 64)


# ---------------------------------------------------------- triangle shape

import tests.test_oracle_triangle as pins_t
from oracle import triangle as tri


def test_triangle_bspline_inner_piece_sign(monkeypatch):
    def bad(u):
        a = np.abs(np.asarray(u, dtype=np.float64))
        out = np.zeros_like(a)
        inner, outer = a <= 1.0, (a > 1.0) & (a < 2.0)
        out[inner] = 2.0 / 3.0 - a[inner] ** 2 - 0.5 * a[inner] ** 3
        out[outer] = (2.0 - a[outer]) ** 3 / 6.0
        return out
    monkeypatch.setattr(tri, "bspline3", bad)
    assert _fails(pins_t.test_conv2_equals_quadrature, 0.3, 0.17)


def test_triangle_missing_periodic_image(monkeypatch):
    def bad(d, h, L):
        r = tri.periodic_distance(d, L)
        return tri.bspline3(r / h) / h
    monkeypatch.setattr(tri, "conv2", bad)
    assert _fails(pins_t.test_conv2_equals_quadrature, 0.45 * pins_t.L0, 0.5 * pins_t.L0)


def test_triangle_kernel_without_normalisation(monkeypatch):
    def bad(d, h, L):
        return np.maximum(0.0, 1.0 - tri.periodic_distance(d, L) / h)
    monkeypatch.setattr(tri, "kernel", bad)
    assert _fails(pins_t.test_kernel_integrates_to_one, 0.7)


def test_triangle_full_width_read_as_half_width(monkeypatch):
    """Reading h as the full support width halves the triangle; the PIC
    special case (linear weighting at h = dx) catches it."""
    orig = tri.kernel

    def bad(d, h, L):
        return orig(d, 0.5 * np.asarray(h, dtype=np.float64), L)
    monkeypatch.setattr(tri, "kernel", bad)
    assert _fails(pins_t.test_width_dx_is_linear_weighting)


def test_triangle_conv_at_zero_in_cv(monkeypatch):
    """A wrong Tbar(0) in the first CV term shifts the objective by n Tbar(0)/n^2;
    the unbiasedness pin against the Fourier MISE catches it."""
    monkeypatch.setattr(tri, "conv2_at_zero", lambda h, L: 1.0 / np.asarray(h, dtype=np.float64))
    assert _fails(pins_t.test_cv_is_unbiased_for_mise_minus_int_f2, 0.35)
