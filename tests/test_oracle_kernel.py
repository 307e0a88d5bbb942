"""Pins of the oracle's kernel, convolution, deposit and gather against facts
fixed outside the oracle: 50-digit Bessel values, Bessel identities,
quadrature, SciPy's von Mises law and the closed-form grid sum."""
import math

import mpmath
import numpy as np
import pytest
from scipy import special, stats

from oracle import vonmises as vm, density

mpmath.mp.dps = 50


# ---------------------------------------------------------------- Bessel (P-1)

@pytest.mark.parametrize("x", list(np.logspace(-6, math.log10(2e4), 41)))
def test_i0e_matches_50_digit_bessel(x):
    ref = mpmath.besseli(0, mpmath.mpf(float(x))) * mpmath.exp(-mpmath.mpf(float(x)))
    assert abs(vm.i0e(x) - float(ref)) <= 2e-15 * float(ref)


@pytest.mark.parametrize("m,k", [(1, 0.3), (2, 5.0), (7, 40.0), (64, 900.0), (128, 1e4), (3, 1e-4)])
def test_bessel_ratio_matches_50_digit(m, k):
    ref = mpmath.besseli(m, mpmath.mpf(k)) / mpmath.besseli(0, mpmath.mpf(k))
    assert abs(vm.bessel_ratio(m, k) - float(ref)) <= 1e-14 * float(ref) + 1e-300


@pytest.mark.parametrize("k", [0.01, 1.0, 37.0, 900.0, 1e4])
def test_neumann_identity(k):
    # sum_{m in Z} I_m(k)^2 = I_0(2k), both sides scaled by exp(-2k)
    m = np.arange(1, int(10 * math.sqrt(k) + 60))
    lhs = special.ive(0, k) ** 2 + 2.0 * np.sum(special.ive(m, k) ** 2)
    assert abs(lhs - special.ive(0, 2 * k)) <= 1e-14 * special.ive(0, 2 * k)


@pytest.mark.parametrize("k", [0.5, 20.0, 3000.0])
def test_bessel_recurrence(k):
    m = np.arange(1, 30)
    lhs = special.ive(m - 1, k) - special.ive(m + 1, k)
    rhs = (2.0 * m / k) * special.ive(m, k)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-300)


# ------------------------------------------------------- kernel density (P-2)

@pytest.mark.parametrize("k", [0.0, 1e-3, 1.0, 37.0, 1000.0, 2e4])
@pytest.mark.parametrize("L", [2 * math.pi, 4 * math.pi, 1.0])
def test_kernel_integrates_to_one(k, L):
    Q = int(10 * math.sqrt(k) + 32) * 2
    xq = np.arange(Q) * (L / Q)
    # the exponent -2 kappa s^2 carries a relative rounding error of a few ulp,
    # so the kernel's own conditioning grows like sqrt(kappa)
    assert abs(np.sum(vm.kernel(xq, k, L)) * (L / Q) - 1.0) <= 2e-14 + 5e-16 * math.sqrt(k)


@pytest.mark.parametrize("k", [0.3, 4.0, 55.0, 500.0])
def test_kernel_is_scipy_von_mises_law(k):
    L = 4 * math.pi
    d = np.linspace(-L, 2 * L, 301)
    th = np.mod(2 * math.pi * d / L + math.pi, 2 * math.pi) - math.pi
    ref = (2 * math.pi / L) * stats.vonmises.pdf(th, k)
    np.testing.assert_allclose(vm.kernel(d, k, L), ref, rtol=1e-12, atol=1e-300)


def test_kernel_symmetric_and_periodic():
    L = 3.0
    d = np.linspace(0, L, 97)
    np.testing.assert_allclose(vm.kernel(d, 12.0, L), vm.kernel(-d, 12.0, L), rtol=1e-14)
    np.testing.assert_allclose(vm.kernel(d + L, 12.0, L), vm.kernel(d, 12.0, L), rtol=1e-12)


# ------------------------------------------------ two-fold convolution (P-3)

@pytest.mark.parametrize("k", [0.0, 0.5, 5.0, 37.0, 400.0, 3000.0])
@pytest.mark.parametrize("frac", [0.0, 1e-7, 0.013, 0.25, 0.4999, 0.5, 0.77])
def test_conv2_equals_quadrature(k, frac):
    L = 4 * math.pi
    a, b = 1.1, 1.1 + frac * L
    Q = int(40 * math.sqrt(k) + 256)
    t = np.arange(Q) * (L / Q)
    quad = np.sum(vm.kernel(t - a, k, L) * vm.kernel(t - b, k, L)) * (L / Q)
    val = vm.conv2(a - b, k, L)
    assert abs(val - quad) <= 1e-13 * quad + 1e-300


def test_conv2_at_zero_and_antipode():
    L = 2 * math.pi
    for k in (0.7, 9.0, 120.0):
        # I0(2k)/(L I0(k)^2) and 1/(L I0(k)^2), unscaled SciPy i0 (moderate k)
        assert abs(vm.conv2_at_zero(k, L) - special.i0(2 * k) / (L * special.i0(k) ** 2)) \
            <= 1e-13 * vm.conv2_at_zero(k, L)
        assert abs(vm.conv2(L / 2, k, L) - 1.0 / (L * special.i0(k) ** 2)) \
            <= 1e-13 / (L * special.i0(k) ** 2)


def test_width_kappa_round_trip():
    L = 4 * math.pi
    M = 64
    dx = L / M
    # the standard-PIC reference width 2*dx maps to (M/(4 pi))^2
    assert abs(vm.kappa_from_width(2 * dx, L) - (M / (4 * math.pi)) ** 2) < 1e-12
    assert abs(vm.width_from_kappa(vm.kappa_from_width(0.37, L), L) - 0.37) < 1e-15


def test_wrap():
    L = 4 * math.pi
    x = np.array([-1e-18, -L, 0.0, L, 2.5 * L, -0.5 * L, L - 1e-15])
    w = vm.wrap(x, L)
    assert np.all(w >= 0) and np.all(w < L)
    np.testing.assert_allclose(w[[1, 2, 3]], 0.0)
    np.testing.assert_allclose(w[4], 0.5 * L)
    np.testing.assert_allclose(w[5], 0.5 * L)


# --------------------------------------- deposit/gather grid identity (P-4, P-5)

def grid_sum_closed_form(x, L, M, k):
    """dx sum_g K(x_g - x) = 1 + 2 sum_{q>=1} rho_{qM} cos(q M theta)."""
    th = 2 * math.pi * np.asarray(x) / L
    q = np.arange(1, 40)
    rho = special.ive(q * M, k) / special.ive(0, k)
    return 1.0 + 2.0 * np.sum(rho[None, :] * np.cos(np.outer(th, q * M)), axis=1)


@pytest.mark.parametrize("M,k", [(64, 900.0), (64, 1000.0), (256, 1e4), (128, 3.0), (2, 0.5), (7, 30.0)])
def test_gather_of_ones_is_grid_sum_identity(M, k):
    L = 4 * math.pi
    rng = np.random.default_rng(5)
    x = L * rng.random(300)
    G = density.gather(x, L, np.ones(M), kappa=k)
    np.testing.assert_allclose(G, grid_sum_closed_form(x, L, M, k), rtol=1e-13, atol=1e-15)


def test_deposit_mass_is_mean_grid_sum():
    L, M, k = 2 * math.pi, 64, 700.0
    rng = np.random.default_rng(6)
    x = L * rng.random(500)
    rho = density.deposit(x, L, M, kappa=k)
    mass = rho.sum() * L / M
    assert abs(mass - grid_sum_closed_form(x, L, M, k).mean()) <= 1e-13
    # the aliasing term is large for a narrow kernel: particles on a node
    # carry mass 1 + 2 sum_q rho_{qM} > 1, not 1
    on_node = density.deposit(np.zeros(5), L, M, kappa=k).sum() * L / M
    assert abs(on_node - grid_sum_closed_form(np.zeros(1), L, M, k)[0]) <= 1e-13
    assert on_node - 1.0 > 0.05


def test_deposit_matches_scipy_von_mises_mixture():
    L, M = 4 * math.pi, 32
    rng = np.random.default_rng(7)
    x = L * rng.random(40)
    kap = 10.0 ** rng.uniform(-1, 3, 40)
    rho = density.deposit(x, L, M, kappa_i=kap)
    th_g = 2 * math.pi * np.arange(M) / M
    ref = np.zeros(M)
    for xi, ki in zip(x, kap):
        ref += (2 * math.pi / L) * stats.vonmises.pdf(th_g, ki, loc=2 * math.pi * xi / L)
    np.testing.assert_allclose(rho, ref / 40, rtol=1e-12)


@pytest.mark.parametrize("M", [5, 64, 256])
def test_gather_is_adjoint_of_deposit(M):
    L = 4 * math.pi
    rng = np.random.default_rng(M)
    x = L * rng.random(700)
    kap = 10.0 ** rng.uniform(0, 4, 700)
    F = rng.standard_normal(M)
    rho = density.deposit(x, L, M, kappa_i=kap)
    G = density.gather(x, L, F, kappa_i=kap)
    assert abs((L / M) * np.dot(F, rho) - G.mean()) <= 1e-13 * (np.abs(F).max())
