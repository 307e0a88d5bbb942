"""Pins of the continuous CV minimiser and the exact pilot (oracle/refine.py),
CPU only.

Each pin comes from outside the code it checks: the two-particle objective
written with mpmath Bessel functions at 30 digits and minimised by mpmath's
root finder, SciPy's von Mises law for the pilot, the Fourier series of the
kernel (SciPy's scaled Bessel functions) as a second route, and the scale
invariances of the geometric-mean normalisation."""
import math

import mpmath
import numpy as np
import pytest
from scipy import special, stats

import workloads as W
from oracle import cv, refine
from oracle.vonmises import bessel_ratio

mpmath.mp.dps = 30


def _cv_two_mp(kappa, d, L):
    """n = 2 at distance d: (Kbar(0) + Kbar(d))/2 - 2 K(d), from I0 itself."""
    k = mpmath.mpf(kappa)
    i0k = mpmath.besseli(0, k)
    c = abs(mpmath.cos(mpmath.pi * d / L))
    kbar0 = mpmath.besseli(0, 2 * k) / (L * i0k ** 2)
    kbard = mpmath.besseli(0, 2 * k * c) / (L * i0k ** 2)
    kd = mpmath.exp(k * mpmath.cos(2 * mpmath.pi * d / L)) / (L * i0k)
    return (kbar0 + kbard) / 2 - 2 * kd


@pytest.mark.parametrize("d", [0.3, 0.9, 1.2])
def test_two_particle_minimiser_matches_mpmath(d):
    L = 2 * math.pi
    x = np.array([0.5, 0.5 + d])
    kappas = W.log_kappas(0.1, 1e3, 13)
    k_o, v_o, b, (lo, hi) = refine.cv_minimise(x, L, kappas)
    f = lambda u: mpmath.diff(lambda t: _cv_two_mp(mpmath.exp(t), d, L), u)
    u_mp = mpmath.findroot(f, math.log(k_o))
    assert math.log(lo) < float(u_mp) < math.log(hi)
    assert abs(k_o / float(mpmath.exp(u_mp)) - 1) < 1e-12
    assert abs(v_o - float(_cv_two_mp(mpmath.exp(u_mp), d, L))) < 1e-13


def test_two_particle_minimum_at_the_list_end():
    """Two particles far apart: the objective rises from the smallest listed
    concentration (mpmath slope > 0 there), so the minimiser is that end."""
    L, d = 2 * math.pi, 1.7
    kappas = W.log_kappas(0.1, 1e3, 13)
    k_o, v_o, b, _ = refine.cv_minimise(np.array([0.5, 0.5 + d]), L, kappas)
    slope = mpmath.diff(lambda t: _cv_two_mp(mpmath.exp(t), d, L), math.log(kappas[0]))
    assert b == 0 and slope > 0 and k_o == kappas[0]


@pytest.mark.parametrize("kappa", [0.7, 12.0, 300.0, 5000.0])
def test_slope_matches_central_differences(kappa):
    """The direct-sum derivative against fourth-order central differences of
    the direct-sum objective in log(kappa)."""
    L = 4 * math.pi
    rng = np.random.default_rng(46)
    x = W.cosine_positions(rng, 300, L, 0.5, 0.5)
    h = 2e-3
    f = [refine.cv_at(x, L, kappa * math.exp(j * h)) for j in (-2, -1, 1, 2)]
    fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
    g = refine.cv_slope(x, L, kappa)
    assert abs(g - fd) <= 1e-9 * max(1.0, abs(fd)) + 1e-9


def test_two_particle_slope_matches_mpmath():
    L, d = 2 * math.pi, 0.7
    x = np.array([1.0, 1.0 + d])
    for kappa in (0.3, 4.0, 60.0):
        ref = mpmath.diff(lambda t: _cv_two_mp(mpmath.exp(t), d, L), math.log(kappa))
        assert abs(refine.cv_slope(x, L, kappa) - float(ref)) < 1e-13


def test_minimum_is_below_the_scan_and_stationary():
    L = 4 * math.pi
    rng = np.random.default_rng(41)
    x = W.cosine_positions(rng, 400, L, 0.5, 0.5)
    kappas = W.log_kappas(1.0, 1e4, 12)
    k, v, b, (lo, hi) = refine.cv_minimise(x, L, kappas)
    grid, _, _ = cv.cv_curve(x, L, kappas)
    assert v <= grid.min() and lo < k < hi
    # central second-order differences in log(kappa): slope ~ 0 at the minimum
    h = 1e-3
    up, mid, dn = (refine.cv_at(x, L, k * math.exp(s)) for s in (h, 0.0, -h))
    slope = (up - dn) / (2 * h)
    curv = (up - 2 * mid + dn) / (h * h)
    assert curv > 0
    assert abs(slope) <= 1e-5 * curv


def test_minimiser_agrees_with_the_fourier_route():
    """Minimise the Fourier-series objective (SciPy ive) independently and
    compare the minimisers."""
    from scipy import optimize
    L = 4 * math.pi
    rng = np.random.default_rng(42)
    x = W.cosine_positions(rng, 700, L, 0.3, 0.5)
    kappas = W.log_kappas(1.0, 1e4, 16)
    k, v, b, (lo, hi) = refine.cv_minimise(x, L, kappas)
    res = optimize.minimize_scalar(lambda u: float(cv.cv_curve_fourier(x, L, [math.exp(u)])[0][0]),
                                   bounds=(math.log(lo), math.log(hi)), method="bounded",
                                   options={"xatol": 1e-11})
    assert abs(res.x - math.log(k)) < 1e-5
    assert abs(res.fun - v) < 1e-13
    assert abs(refine.cv_slope(x, L, k)) < 1e-14


@pytest.mark.parametrize("kappa", [0.0, 0.8, 30.0, 900.0])
def test_pilot_exact_is_the_von_mises_mixture(kappa):
    L = 4 * math.pi
    rng = np.random.default_rng(43)
    x = W.cosine_positions(rng, 300, L, 0.4, 0.5)
    f = refine.pilot_exact(x, L, kappa)
    th = 2 * math.pi * x / L
    ref = np.array([np.mean(stats.vonmises.pdf(t - th, kappa)) for t in th]) * (2 * math.pi / L)
    assert np.max(np.abs(f - ref) / ref) < 1e-12


def test_pilot_exact_fourier_series():
    """f(x) = (1/L)(1 + 2 sum_m rho_m Re(conj(c_m) e^{i m theta})), c_m the
    sample's Fourier moments, rho_m = I_m/I_0 (SciPy)."""
    L = 4 * math.pi
    kappa = 55.0
    rng = np.random.default_rng(44)
    x = W.cosine_positions(rng, 500, L, 0.5, 0.5)
    th = 2 * math.pi * x / L
    m = np.arange(1, 200)
    c = np.exp(1j * np.outer(th, m)).mean(axis=0)
    rho = special.ive(m, kappa) / special.ive(0, kappa)
    ref = (1 + 2 * np.real(np.exp(1j * np.outer(th, m)) @ (rho * np.conj(c)))) / L
    assert np.max(np.abs(refine.pilot_exact(x, L, kappa) - ref) / ref) < 1e-12
    assert np.allclose(rho, bessel_ratio(m, kappa), rtol=1e-14, atol=0)


def test_adapt_exact_invariants():
    L = 4 * math.pi
    rng = np.random.default_rng(45)
    x = W.cosine_positions(rng, 800, L, 0.5, 0.5)
    k, lg, nf = refine.adapt_widths_exact(x, L, 40.0, 0.5)
    assert nf == 0
    assert abs(np.mean(np.log(k / 40.0))) < 1e-13
    k0, _, _ = refine.adapt_widths_exact(x, L, 40.0, 0.0)
    assert np.all(k0 == 40.0)
    # kappa_i = kappa* f_i / g at alpha = 0.5: ratios follow the pilot
    f = refine.pilot_exact(x, L, 40.0)
    assert np.allclose(k / k[0], f / f[0], rtol=1e-12)
