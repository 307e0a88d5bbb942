"""Pins of the first-order (triangular) kernel oracle, CPU only.

Each pin comes from outside the oracle's own formulas: quadrature of the
defining integrals, the partition of unity of hat functions, linear
(cloud-in-cell) weighting as the h = dx special case, brute force on tiny
inputs, and the exact MISE from the kernel's Fourier coefficients."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import mise
from oracle import triangle as tri

L0 = 4 * math.pi


def _quad(f, a, b, points):
    pts = sorted(p for p in points if a < p < b)
    val, err = integrate.quad(f, a, b, points=pts or None, limit=400, epsabs=1e-14, epsrel=1e-13)
    return val


@pytest.mark.parametrize("h", [0.01, 0.7, 3.0, 0.5 * L0])
def test_kernel_integrates_to_one(h):
    f = lambda t: float(tri.kernel(t, h, L0))
    assert abs(_quad(f, 0.0, L0, [h, L0 - h]) - 1.0) < 1e-12


@pytest.mark.parametrize("h,d", [(0.3, 0.0), (0.3, 0.17), (0.3, 0.45), (1.1, 2.0), (2.9, 5.9),
                                 (0.45 * L0, 0.2), (0.45 * L0, 0.5 * L0), (0.5 * L0, 1.0)])
def test_conv2_equals_quadrature(h, d):
    """Tbar(d) = int_0^L T(t - d) T(t) dt, integrated numerically with the
    kinks of both triangles (and their periodic images) as breakpoints;
    h near L/2 exercises the image term."""
    f = lambda t: float(tri.kernel(t - d, h, L0) * tri.kernel(t, h, L0))
    kinks = []
    for c in (0.0, d):
        for off in (-h, 0.0, h):
            kinks.append((c + off) % L0)
    val = _quad(f, 0.0, L0, kinks)
    assert abs(float(tri.conv2(d, h, L0)) - val) < 1e-11 * max(1.0, 1.0 / h)


@pytest.mark.parametrize("h", [0.05, 1.0, 0.5 * L0])
def test_conv2_at_zero_and_mass(h):
    assert abs(float(tri.conv2_at_zero(h, L0)) - 2.0 / (3.0 * h)) < 1e-15 / h
    assert float(tri.conv2(0.0, h, L0)) == float(tri.conv2_at_zero(h, L0))
    f = lambda t: float(tri.conv2(t, h, L0))
    assert abs(_quad(f, 0.0, L0, [h, 2 * h, L0 - h, L0 - 2 * h]) - 1.0) < 1e-12


def test_conv2_is_symmetric_and_periodic():
    h = 0.8
    d = np.linspace(-3 * L0, 3 * L0, 101)
    np.testing.assert_allclose(tri.conv2(d, h, L0), tri.conv2(-d, h, L0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(tri.conv2(d, h, L0), tri.conv2(d + L0, h, L0), rtol=0, atol=1e-14)


def test_rejects_widths_beyond_half_period():
    with pytest.raises(ValueError):
        tri.kernel(0.1, 0.51 * L0, L0)
    with pytest.raises(ValueError):
        tri.conv2(0.1, 0.0, L0)


def test_two_particles_closed_form():
    x = np.array([0.3, 1.0])
    h = 0.5
    r = 0.7  # beyond the triangle, inside the convolution's support
    cvv, S1, S2 = tri.cv_curve(x, L0, [h])
    assert S2[0] == 0.0
    u = r / h
    assert abs(S1[0] - (2.0 - u) ** 3 / 6.0 / h) < 1e-15
    assert abs(cvv[0] - (2 * (2 / (3 * h)) + 2 * S1[0]) / 4.0) < 1e-15


def test_pair_sums_match_plain_loops():
    rng = np.random.default_rng([5, 9])
    x = rng.uniform(0, L0, 23)
    hs = [0.2, 0.9, 2.5, 0.5 * L0]
    S1, S2 = tri.pair_sums(x, L0, hs, block=7)
    for b, h in enumerate(hs):
        s1 = s2 = 0.0
        for i in range(len(x)):
            for j in range(i + 1, len(x)):
                r = abs(x[i] - x[j])
                r = min(r, L0 - r)
                s2 += max(0.0, 1.0 - r / h) / h
                for img in (r, L0 - r):
                    u = img / h
                    if u <= 1:
                        s1 += (2 / 3 - u * u + u ** 3 / 2) / h
                    elif u < 2:
                        s1 += (2 - u) ** 3 / 6 / h
        assert abs(S1[b] - s1) < 1e-12 * max(1.0, abs(s1))
        assert abs(S2[b] - s2) < 1e-12 * max(1.0, abs(s2))


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_deposit_is_a_partition_of_unity_at_integer_widths(p):
    """Hats of half-width p dx (p integer) sampled at spacing dx sum to p, so
    the deposit carries unit mass: sum_g rho_g dx = 1 to rounding."""
    M = 64
    dx = L0 / M
    x = np.random.default_rng([5, 11, p]).uniform(0, L0, 500)
    rho = tri.deposit(x, L0, M, h=p * dx)
    assert abs(np.sum(rho) * dx - 1.0) < 1e-13


def test_width_dx_is_linear_weighting():
    """h = dx is standard PIC's first-order (cloud-in-cell) weighting: a
    particle at (g0 + t) dx puts (1 - t) on node g0 and t on node g0 + 1."""
    M = 32
    dx = L0 / M
    for g0, t in ((3, 0.25), (31, 0.6), (0, 0.0)):
        x = np.array([(g0 + t) * dx])
        rho = tri.deposit(x, L0, M, h=dx) * dx
        expect = np.zeros(M)
        expect[g0] += 1 - t
        expect[(g0 + 1) % M] += t
        np.testing.assert_allclose(rho, expect, atol=1e-14)


def test_gather_is_the_adjoint_of_deposit():
    M = 48
    rng = np.random.default_rng([5, 13])
    x = rng.uniform(0, L0, 300)
    hi = rng.uniform(0.05, 2.0, 300)
    F = rng.normal(size=M)
    rho = tri.deposit(x, L0, M, h_i=hi)
    G = tri.gather(x, L0, F, h_i=hi)
    dx = L0 / M
    assert abs(np.sum(G) - len(x) * dx * np.dot(F, rho)) < 1e-11 * np.sum(np.abs(G))


def test_fourier_coefficients_by_quadrature():
    h = 0.9
    for m in (1, 2, 7):
        f = lambda t: float(tri.kernel(t, h, L0)) * math.cos(2 * math.pi * m * t / L0)
        val = _quad(f, 0.0, L0, [h, L0 - h])
        assert abs(val - float(tri.fourier_coeffs(m, h, L0))) < 1e-12


@pytest.mark.parametrize("h", [0.35, 1.2])
def test_cv_is_unbiased_for_mise_minus_int_f2(h):
    """Sec. II.B: E[CV] = MISE - int f^2 for any kernel; the seed-mean of the
    direct triangle CV must agree with the exact value from the triangle's
    Fourier coefficients (independent of the B-spline form of Tbar)."""
    L = 2 * math.pi
    n, R = 150, 1200
    coeffs = mise.cosine_coeffs(0.6)
    vals = np.empty(R)
    for r in range(R):
        x = W.cosine_positions(np.random.default_rng([78, r]), n, L, 0.6, 1.0)
        c, _, _ = tri.cv_curve(x, L, [h])
        vals[r] = c[0]
    rho = tri.fourier_coeffs(np.arange(1, 400001), h, L)
    expect = mise.mise_from_coeffs(rho, n, L, coeffs) - mise.int_f_squared(L, coeffs)
    se = vals.std(ddof=1) / math.sqrt(R)
    assert abs(vals.mean() - expect) < 4 * se
