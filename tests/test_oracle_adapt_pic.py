"""Pins of the oracle's adaptive widths, PIC step, Anderson-Darling test and
width-update rule."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W
from oracle import adtest, density, pic, update, vonmises as vm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------ adaptive widths (P-12)

def test_pilot_interpolation_is_exact_on_linear_pieces_and_wraps():
    L, M = 4.0, 8
    pilot = np.arange(M, dtype=float) + 1.0           # 1..8
    dx = L / M
    x = np.array([0.0, 0.25 * dx, 3.5 * dx, L - 0.25 * dx])
    f = density.pilot_at_particles(x, L, pilot)
    np.testing.assert_allclose(f, [1.0, 1.25, 4.5, 0.25 * 8.0 + 0.75 * 1.0], rtol=1e-15)


def test_adapt_invariants():
    L, M = 4 * math.pi, 256
    x = W.cosine_positions(np.random.default_rng(12), 5000, L, 0.5, 0.5)
    pilot = density.deposit(x[:2000], L, M, kappa=30.0)
    k_i, log_g, nf = density.adapt_widths(x, L, pilot, 30.0, 0.5)
    assert nf == 0
    assert abs(np.mean(np.log(k_i / 30.0))) < 1e-13
    # denser regions get narrower kernels
    f = density.pilot_at_particles(x, L, pilot)
    order = np.argsort(f)
    assert np.all(np.diff(k_i[order]) >= -1e-12 * k_i.max())
    # alpha = 0 and a uniform pilot both leave every width at kappa*
    k0, _, _ = density.adapt_widths(x, L, pilot, 30.0, 0.0)
    np.testing.assert_allclose(k0, 30.0, rtol=1e-15)
    ku, lg, _ = density.adapt_widths(x, L, np.full(M, 1.0 / L), 30.0, 0.5)
    np.testing.assert_allclose(ku, 30.0, rtol=1e-14)
    assert abs(lg - math.log(1.0 / L)) < 1e-14
    # alpha = 0.5 makes kappa_i proportional to the pilot
    np.testing.assert_allclose(k_i / f, (k_i / f)[0], rtol=1e-12)


def test_constant_widths_reproduce_global_deposit():
    L, M = 4 * math.pi, 64
    x = W.cosine_positions(np.random.default_rng(13), 900, L, 0.5, 0.5)
    a = density.deposit(x, L, M, kappa=17.0)
    b = density.deposit(x, L, M, kappa_i=np.full(900, 17.0))
    np.testing.assert_allclose(a, b, rtol=1e-15)


def test_floor_counts_nonpositive_pilot():
    L, M = 1.0, 4
    pilot = np.array([0.0, 0.0, 1.0, 1.0])
    x = np.array([0.1, 0.6, 0.8])
    k_i, log_g, nf = density.adapt_widths(x, L, pilot, 5.0, 0.5)
    assert nf == 1 and np.all(np.isfinite(k_i)) and np.isfinite(log_g)


def test_paper_constants():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert update.THRESHOLD == c["p_threshold"]
    assert update.ADJUST_RATE == c["adjust_rate"]
    import inspect
    assert inspect.signature(density.adapt_widths).parameters["alpha"].default == c["silverman_alpha"]


# --------------------------------------------------------- Poisson, E (P-13)

@pytest.mark.parametrize("M", [8, 64, 128, 512])
def test_poisson_solves_the_difference_equation(M):
    L = 4 * math.pi
    dx = L / M
    rng = np.random.default_rng(M)
    rq = rng.standard_normal(M)
    phi = pic.poisson_fd(rq, dx)
    lap = (np.roll(phi, 1) - 2 * phi + np.roll(phi, -1)) / dx ** 2
    np.testing.assert_allclose(lap, -(rq - rq.mean()), atol=1e-12 * np.abs(rq).max())
    assert abs(phi.mean()) < 1e-12


def test_poisson_single_mode_closed_form():
    M, m0, L = 128, 3, 4 * math.pi
    dx = L / M
    g = np.arange(M)
    rq = np.cos(2 * math.pi * m0 * g / M)
    phi = pic.poisson_fd(rq, dx)
    expect = dx * dx / (2 - 2 * math.cos(2 * math.pi * m0 / M)) * rq
    np.testing.assert_allclose(phi, expect, atol=1e-13)
    E = pic.efield_centered(phi, dx)
    expect_E = dx * dx / (2 - 2 * math.cos(2 * math.pi * m0 / M)) * \
        (np.cos(2 * math.pi * m0 * (g - 1) / M) - np.cos(2 * math.pi * m0 * (g + 1) / M)) / (2 * dx)
    np.testing.assert_allclose(E, expect_E, atol=1e-13)


def test_push_is_literal_leapfrog_and_wraps():
    L = 2.0
    x = np.array([0.1, 1.95, 0.5])
    v = np.array([1.0, 1.0, -3.0])
    E = np.array([0.5, -1.0, 0.0])
    xn, vn = pic.push(x, v, E, 0.1, L)
    np.testing.assert_allclose(vn, [0.95, 1.1, -3.0])
    np.testing.assert_allclose(xn, [0.195, (1.95 + 0.11) - 2.0, 0.2])


def test_cold_plasma_oscillates_at_plasma_frequency():
    """A cold, slightly displaced electron population oscillates at the plasma
    frequency 1 in these units (Sec. III.A): the field energy vanishes at
    t = pi/2 and 3 pi/2 when the displacement has turned into velocity."""
    L, M, n, dt = 2 * math.pi, 64, 4096, 0.05
    x0 = np.arange(n) * (L / n)
    x = vm.wrap(x0 + 0.002 * np.sin(x0), L)
    v = np.zeros(n)
    kap = np.full(n, 400.0)
    energies = []
    for _ in range(int(round(2 * math.pi / dt))):
        x, v, rho, E = pic.field_step(x, v, kap, L, M, dt)
        energies.append(float(np.sum(E * E)))
    e = np.array(energies)
    mins = [i for i in range(1, len(e) - 1) if e[i] < e[i - 1] and e[i] <= e[i + 1]]
    assert len(mins) == 2
    # energy recorded before the push of step i+1, i.e. at t = i*dt
    assert abs(mins[0] * dt - math.pi / 2) < 3 * dt
    assert abs(mins[1] * dt - 3 * math.pi / 2) < 3 * dt


# --------------------------------------------------- Anderson-Darling (P-14)

def test_ad_statistic_matches_scipy():
    rng = np.random.default_rng(21)
    for n in (5, 100, 3000):
        u = rng.random(n)
        res = stats.goodness_of_fit(stats.uniform, u, known_params={"loc": 0.0, "scale": 1.0},
                                    statistic="ad", n_mc_samples=1, rng=0)
        assert abs(adtest.ad_statistic(u * 3.0, 3.0) - res.statistic) <= 1e-10 * max(1.0, res.statistic)


def test_ad_published_upper_tail_points():
    g = json.load(open(os.path.join(GOLDEN, "ad_critical_points.json")))
    for p in g["points"]:
        assert abs(adtest.ad_pvalue(p["a2"]) - p["upper_tail"]) <= p["abs_tol"]


def ad_upper_tail_charfn(x, T=6000.0, h=0.01):
    """Upper tail of the limiting law of A^2 by Gil-Pelaez inversion of its
    characteristic function, a route independent of the Anderson-Darling
    series the oracle sums. The limit law is that of sum_j Y_j^2 / (j(j+1))
    with Y_j standard normal, so
        phi(t) = prod_j (1 - 2 i t / (j (j+1)))^(-1/2)
               = sqrt(-2 pi i t / cos((pi/2) sqrt(1 + 8 i t)))
    (the roots of j^2 + j - 2 i t and Gamma(1/2 - z) Gamma(1/2 + z) =
    pi / cos(pi z)); the branch is the continuous one from phi(0) = 1.
    F(x) = 1/2 - (1/pi) int_0^inf Im(exp(-i t x) phi(t)) / t dt, by
    Simpson's rule (the integrand is analytic and |phi| ~ exp(-pi sqrt(t)/2),
    below 1e-50 at T)."""
    t = np.arange(1, int(round(T / h)) + 1) * h
    s = np.sqrt(1.0 + 8j * t)
    lr = np.log(-2j * math.pi * t) - np.log(np.cos(0.5 * math.pi * s))
    logphi = 0.5 * (lr.real + 1j * np.unwrap(lr.imag))
    f = np.imag(np.exp(-1j * t * x + logphi)) / t
    y = np.concatenate([[1.0 - x], f])  # t -> 0 limit: E[A^2] - x = 1 - x
    if (y.shape[0] - 1) % 2:
        y = y[:-1]
    integral = h / 3.0 * (y[0] + y[-1] + 4.0 * y[1:-1:2].sum() + 2.0 * y[2:-1:2].sum())
    return 0.5 + integral / math.pi


@pytest.mark.parametrize("a2", [0.5, 1.933, 2.492, 3.070, 3.857, 3.8781, 5.0, 7.0])
def test_ad_tail_matches_characteristic_function(a2):
    """The oracle's p-value against the characteristic-function inversion,
    through the tail where the width-update rule acts (p <= 0.02)."""
    assert abs(adtest.ad_pvalue(a2) - ad_upper_tail_charfn(a2)) <= 1e-12


def test_ad_limit_law_moments():
    """The limiting law is that of sum_j Y_j^2 / (j(j+1)), Y_j standard normal:
    mean 1 and variance 2 (pi^2/3 - 3)."""
    zs = np.linspace(0.02, 14.0, 1400)
    cdf = np.array([adtest.ad_cdf(z) for z in zs])
    # E[X] = int (1 - F), E[X^2] = int 2 z (1 - F)
    m1 = integrate.trapezoid(1 - cdf, zs) + 0.02 * 1.0
    m2 = integrate.trapezoid(2 * zs * (1 - cdf), zs) + 0.02 ** 2
    assert abs(m1 - 1.0) < 2e-3
    assert abs((m2 - m1 ** 2) - 2 * (math.pi ** 2 / 3 - 3)) < 5e-3


def test_ad_pvalues_of_uniform_samples_are_uniform():
    rng = np.random.default_rng(22)
    ps = [adtest.ad_pvalue(adtest.ad_statistic(rng.random(400), 1.0)) for _ in range(300)]
    assert stats.kstest(ps, "uniform").pvalue > 1e-3


# ----------------------------------------------------------- update rule (P-15)

def test_update_rule_scripted_sequence():
    g = json.load(open(os.path.join(GOLDEN, "update_rule_sequence.json")))
    widths = iter(g["solve_widths"])
    s = update.initial_state(g["h0"], g["threshold"])
    assert s.p_th == 2 * g["threshold"]
    for st in g["steps"]:
        s, fired = update.step(s, st["p"], lambda: next(widths), g["threshold"], g["rate"])
        assert fired == st["fired"]
        assert abs(s.p_th - st["p_th"]) < 1e-15
        assert abs(s.h_target - st["h_target"]) < 1e-15
        assert abs(s.h_opt - st["h_opt"]) < 1e-13
