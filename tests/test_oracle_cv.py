"""Pins of the oracle's CV objective: closed forms for tiny n, quadrature of
the squared estimate, the Fourier-moment identity, invariances, the
unbiasedness of Sec. II.B against the exact MISE, the behaviour argued in
Appendix A, and the location of the minimiser."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cv, density, mise, vonmises as vm


def test_two_particles_closed_form():
    L = 4 * math.pi
    for k in (0.2, 3.0, 80.0, 2500.0):
        for d in (1e-6, 0.3, L / 2, 0.9 * L):
            x = np.array([0.7, vm.wrap(0.7 + d, L)])
            c, S1, S2 = cv.cv_curve(x, L, [k])
            expect = 0.5 * (vm.conv2_at_zero(k, L) + vm.conv2(d, k, L)) - 2.0 * vm.kernel(d, k, L)
            assert abs(c[0] - expect) <= 1e-13 * abs(expect) + 1e-300


def test_antipodal_pair_uses_unscaled_bessel():
    L = 2 * math.pi
    from scipy import special
    for k in (0.5, 7.0, 60.0):
        x = np.array([0.0, math.pi])
        c, _, _ = cv.cv_curve(x, L, [k])
        i0k = special.i0(k)
        kbar0 = special.i0(2 * k) / (L * i0k ** 2)
        kbar_pi = 1.0 / (L * i0k ** 2)
        k_pi = math.exp(-k) / (L * i0k)
        expect = 0.5 * (kbar0 + kbar_pi) - 2.0 * k_pi
        assert abs(c[0] - expect) <= 1e-12 * abs(expect)


@pytest.mark.parametrize("n,k", [(7, 2.0), (60, 30.0), (250, 400.0)])
def test_first_term_is_integral_of_squared_estimate(n, k):
    L = 4 * math.pi
    rng = np.random.default_rng(n)
    x = W.cosine_positions(rng, n, L, 0.3, 0.5)
    S1, S2 = cv.pair_sums(x, L, [k])
    first = (n * vm.conv2_at_zero(k, L) + 2 * S1[0]) / n ** 2
    Q = int(40 * math.sqrt(k) + 512)
    f = density.deposit(x, L, Q, kappa=k)          # estimate on a fine periodic grid
    quad = np.sum(f * f) * (L / Q)
    assert abs(first - quad) <= 1e-12 * quad


@pytest.mark.parametrize("n,k", [(9, 1.0), (120, 50.0), (300, 3000.0)])
def test_second_term_is_leave_one_out_mean(n, k):
    L = 4 * math.pi
    rng = np.random.default_rng(100 + n)
    x = W.cosine_positions(rng, n, L, 0.3, 0.5)
    S1, S2 = cv.pair_sums(x, L, [k])
    # 2/n sum_i fhat_{-i}(X_i), with fhat_{-i} = (n fhat(X_i) - K(0)) / (n - 1)
    full = np.array([vm.kernel(xi - x, k, L).mean() for xi in x])
    loo = (n * full - vm.kernel(0.0, k, L)) / (n - 1)
    second = 2.0 * loo.mean()
    assert abs(4 * S2[0] / (n * (n - 1)) - second) <= 1e-12 * second


@pytest.mark.parametrize("n", [2, 3, 50, 300, 1000])
def test_fourier_identity_matches_direct_sums(n):
    L = 4 * math.pi
    rng = np.random.default_rng(1000 + n)
    x = W.cosine_positions(rng, n, L, 0.5, 0.5)
    kap = np.logspace(-3, 4, 15)
    S1, S2 = cv.pair_sums(x, L, kap)
    F1, F2 = cv.pair_sums_fourier(x, L, kap)
    np.testing.assert_allclose(F1, S1, rtol=1e-12, atol=1e-14 * n)
    np.testing.assert_allclose(F2, S2, rtol=1e-12, atol=1e-14 * n)


def test_uniform_kernel_limit():
    L = 4 * math.pi
    x = W.cosine_positions(np.random.default_rng(3), 77, L, 0.2, 0.5)
    c, _, _ = cv.cv_curve(x, L, [0.0])
    assert abs(c[0] + 1.0 / L) <= 1e-14


def test_invariances():
    L = 4 * math.pi
    rng = np.random.default_rng(11)
    x = W.cosine_positions(rng, 200, L, 0.5, 0.5)
    kap = [0.5, 7.0, 300.0, 9000.0]
    c0, _, _ = cv.cv_curve(x, L, kap)
    for y in (vm.wrap(x + 2.345, L), vm.wrap(L - x, L), rng.permutation(x)):
        c1, _, _ = cv.cv_curve(y, L, kap)
        np.testing.assert_allclose(c1, c0, rtol=1e-12)


@pytest.mark.parametrize("truth", ["vonmises", "cosine"])
def test_cv_is_unbiased_for_mise_minus_int_f2(truth):
    """Sec. II.B: E[CV] + int f^2 = MISE; the seed-mean of CV over many
    independent draws must agree with the exact MISE - int f^2."""
    L = 2 * math.pi
    n, k, R = 200, 5.0, 1500
    if truth == "vonmises":
        coeffs = mise.vonmises_coeffs(3.0)
    else:
        coeffs = mise.cosine_coeffs(0.6)
    vals = np.empty(R)
    for r in range(R):
        rng = np.random.default_rng([77, r])
        if truth == "vonmises":
            x = W.vonmises_positions(rng, n, L, 0.0, 3.0)
        else:
            x = W.cosine_positions(rng, n, L, 0.6, 1.0)
        c, _, _ = cv.cv_curve_fourier(x, L, [k])
        vals[r] = c[0]
    expect = mise.expected_cv(k, n, L, coeffs)
    se = vals.std(ddof=1) / math.sqrt(R)
    assert abs(vals.mean() - expect) < 4 * se


def test_cv_fourier_route_is_exact_for_unbiasedness_check():
    # the check above uses the Fourier route for speed; it equals the direct one
    L = 2 * math.pi
    x = W.vonmises_positions(np.random.default_rng(0), 200, L, 0.0, 3.0)
    a, _, _ = cv.cv_curve(x, L, [5.0])
    b, _, _ = cv.cv_curve_fourier(x, L, [5.0])
    assert abs(a[0] - b[0]) <= 1e-13


def test_mise_closed_form_small_n_by_monte_carlo():
    """The closed form itself: average integrated squared error of the
    estimate over draws, computed by quadrature of (fhat - f)^2."""
    L, n, k, R = 2 * math.pi, 50, 4.0, 600
    alpha = 0.6
    Q = 256
    xq = np.arange(Q) * (L / Q)
    f = (1 + alpha * np.cos(xq)) / L
    ise = np.empty(R)
    for r in range(R):
        x = W.cosine_positions(np.random.default_rng([78, r]), n, L, alpha, 1.0)
        fh = density.deposit(x, L, Q, kappa=k)
        ise[r] = np.sum((fh - f) ** 2) * (L / Q)
    expect = mise.mise(k, n, L, mise.cosine_coeffs(alpha))
    assert abs(ise.mean() - expect) < 4 * ise.std(ddof=1) / math.sqrt(R)


def test_appendix_a_behaviour():
    """Without leave-one-out the objective keeps falling as the kernel narrows
    (its diagonal (Kbar(0) - 2K(0))/n tends to minus infinity); with it, the
    objective grows like Kbar(0)/n for distinct points."""
    L = 4 * math.pi
    x = W.cosine_positions(np.random.default_rng(9), 40, L, 0.3, 0.5)
    kap = np.array([1e4, 1e6, 1e8])
    bad = cv.cv_without_leave_one_out(x, L, kap)
    good, _, _ = cv.cv_curve(x, L, kap)
    assert bad[0] > bad[1] > bad[2]
    assert good[0] < good[1] < good[2]
    n = len(x)
    np.testing.assert_allclose(good[2], vm.conv2_at_zero(1e8, L) / n, rtol=1e-6)
    np.testing.assert_allclose(bad[2], (vm.conv2_at_zero(1e8, L) - 2 * vm.kernel(0.0, 1e8, L)) / n,
                               rtol=1e-6)


def test_minimiser_lands_near_mise_optimum():
    """Median over 64 seeds of the CV minimiser (fine kappa grid) lies within
    a factor 2 of the exact-MISE optimum; the optimum grows with n."""
    L, alpha, n = 4 * math.pi, 0.5, 4096
    coeffs = mise.cosine_coeffs(alpha)
    kopt = mise.kappa_opt(n, L, coeffs)
    grid = np.logspace(-1, 3, 161)
    picks = []
    for s in range(64):
        x = W.cosine_positions(np.random.default_rng([79, s]), n, L, alpha, 0.5)
        c, _, _ = cv.cv_curve_fourier(x, L, grid)
        picks.append(grid[cv.cv_argmin(c)])
    med = float(np.median(np.log(picks)))
    assert abs(med - math.log(kopt)) < math.log(2.0)
    assert mise.kappa_opt(4 * n, L, coeffs) > kopt > mise.kappa_opt(n // 4, L, coeffs)


def test_argmin_takes_first_of_ties():
    assert cv.cv_argmin(np.array([3.0, 1.0, 2.0, 1.0])) == 1


def test_needs_two_particles():
    with pytest.raises(ValueError):
        cv.cv_curve(np.array([1.0]), 1.0, [1.0])


def test_bench_reference_small_case_is_the_oracles():
    """The plain-small entries of tests/golden/bench_reference.json (read by
    bench.py's precision form) are what the oracle computes now."""
    import json
    import os
    from oracle import density as od
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bench_reference.json")
    ref = json.load(open(path))["precision_small"]["f32_positions"]
    p = W.plain_small()
    x = p.x.astype(np.float32).astype(np.float64)
    c, S1, S2 = cv.cv_curve(x, p.L, p.kappas)
    assert np.array_equal(c, ref["cv"]) and np.array_equal(S1, ref["S1"]) and cv.cv_argmin(c) == ref["argmin"]
    for k, g in zip(p.kappas, ref["grids"]):
        assert np.array_equal(od.deposit(x, p.L, p.M, kappa=float(k)), g)
