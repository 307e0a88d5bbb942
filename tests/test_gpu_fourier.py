"""GPU parity of the Fourier-moment route: kde_cv_scan_fourier,
kde_cv_refine and kde_adapt_widths_exact against the oracle.

Tolerances (FP64 arithmetic in both position precisions):
* CV values: 1e-12 relative (the objective is formed as 2A/N^2 - 4C/(N(N-1))
  - 1 over sums of positive terms, plus the leave-one-out difference).
* Pair sums: 1e-12 relative plus 1e-13 of the double sum they come from
  (sum_{i,j} Kbar resp. K, diagonal included): S1 and S2 are that sum minus
  its diagonal, so where the diagonal dominates they carry a few rounding
  units of it.
* Refinement: the objective at the minimiser to 1e-12 relative; the
  minimiser in u = log(kappa) to 1e-9 (the slope of the objective is formed
  to about 1e-12 of its terms, and the curvature turns that into the
  distance between the roots); where the minimum sits at an end of the
  bracket, the same end.
* Exact pilot widths: 1e-12 relative in double plus 2 alpha 64 u K(0)/f_i
  (the series carries a few rounding units of the kernel's peak
  K(0) = (1/L)(1 + 2 sum rho_m)); 1e-6 relative in float.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cv as ocv
from oracle import refine as oref
from oracle.vonmises import conv2_at_zero, i0e, kernel, wrap
from tests.gpu_util import announce, host, rel_err, to_gpu

pytestmark = pytest.mark.gpu


def npx(x, dtype):
    return np.asarray(x, dtype=np.float64 if dtype == "f64" else np.float32)


def check_scan(cv, sums, am, x64, L, kappas, ref=None):
    if ref is None:
        ref = ocv.cv_curve(x64, L, kappas)
    ref_cv, S1, S2 = ref
    n = len(x64)
    B = len(kappas)
    assert rel_err(cv, ref_cv).max() <= 1e-12, rel_err(cv, ref_cv)
    tot1 = n * conv2_at_zero(kappas, L) + 2 * S1
    tot2 = n * kernel(0.0, kappas, L) + 2 * S2
    assert np.all(np.abs(sums[:B] - S1) <= 1e-12 * np.abs(S1) + 1e-13 * tot1)
    assert np.all(np.abs(sums[B:] - S2) <= 1e-12 * np.abs(S2) + 1e-13 * tot2)
    am_ref = ocv.cv_argmin(ref_cv)
    if am != am_ref:
        assert abs(ref_cv[am] - ref_cv[am_ref]) <= 2e-12 * np.abs(ref_cv).max()


def run_scan(kde, x, L, kappas):
    cv, sums, am = kde.cv_scan_fourier(to_gpu(x), L, kappas)
    return host(cv), host(sums), int(host(am)[0])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scan_plain_small(gpu, dtype):
    p = W.plain_small()
    x = npx(p.x, dtype)
    announce("fourier scan plain-small", dtype)
    cv, sums, am = run_scan(gpu, x, p.L, p.kappas)
    check_scan(cv, sums, am, x.astype(np.float64), p.L, p.kappas)


@pytest.mark.parametrize("n", [2, 3, 7, 255, 1025, 3000])
def test_scan_sizes_and_kappa_range(gpu, n):
    L = 4 * math.pi
    rng = np.random.default_rng([31, n])
    x = W.cosine_positions(rng, n, L, 0.4, 0.5)
    kap = np.array([0.0, 1e-3, 0.7, 5.0, 40.0, 300.0, 2500.0, 2e4, 1e5])
    announce("fourier scan sizes", n)
    cv, sums, am = run_scan(gpu, x, L, kap)
    check_scan(cv, sums, am, x, L, kap)


def test_scan_wrapped_positions_and_64_kappas(gpu):
    L = 2.75
    rng = np.random.default_rng(33)
    x = L * rng.random(1500) + L * rng.integers(-3, 3, 1500)
    kap = W.log_kappas(0.05, 3e4, 64)
    announce("fourier scan B=64")
    cv, sums, am = run_scan(gpu, x, L, kap)
    check_scan(cv, sums, am, wrap(x, L), L, kap)


def test_scan_paper_scale_against_oracle_fourier_and_pairs(gpu):
    """65,536 paper-scale positions, 32 kappas in [1, 1e4]: against the
    oracle's Fourier route (SciPy Bessel ratios, pinned to the direct sums)
    and against the GPU pair kernel."""
    p = W.plain_paper_scale(n=1 << 16)
    x = p.x[:p.n_cv]
    announce("fourier scan paper-scale", len(x))
    cv, sums, am = run_scan(gpu, x, p.L, p.kappas)
    check_scan(cv, sums, am, x, p.L, p.kappas, ref=ocv.cv_curve_fourier(x, p.L, p.kappas))
    cvp, _, amp = gpu.cv_scan(to_gpu(x), p.L, p.kappas)
    assert rel_err(cv, host(cvp)).max() <= 2e-12 and am == int(host(amp)[0])


def test_scan_deterministic(gpu):
    p = W.plain_small()
    a = run_scan(gpu, p.x, p.L, p.kappas)
    b = run_scan(gpu, p.x, p.L, p.kappas)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def run_refine(kde, x, L, kappas):
    res, cv, am = kde.cv_refine(to_gpu(x), L, kappas)
    return host(res), host(cv), int(host(am)[0])


def check_refine(res, x64, L, kappas):
    k_o, v_o, b_o, (lo, hi) = oref.cv_minimise(x64, L, kappas)
    assert int(res[4]) == b_o
    assert abs(res[1] - v_o) <= 1e-12 * abs(v_o)
    if k_o in (lo, hi):
        assert res[0] == k_o
    else:
        assert abs(math.log(res[0]) - math.log(k_o)) <= 1e-9, (res[0], k_o)
    return k_o


@pytest.mark.parametrize("seed,n,alpha", [(1, 300, 0.5), (2, 1000, 0.3), (3, 2500, 0.1), (4, 700, 0.5)])
def test_refine_matches_oracle_minimiser(gpu, seed, n, alpha):
    L = 4 * math.pi
    rng = np.random.default_rng([35, seed])
    x = W.cosine_positions(rng, n, L, alpha, 0.5)
    kap = W.log_kappas(1.0, 1e4, 16)
    announce("fourier refine", seed, n)
    res, cv, am = run_refine(gpu, x, L, kap)
    check_refine(res, x, L, kap)
    assert am == int(res[4])
    assert res[1] <= cv.min() * (1 - 1e-15) or res[1] <= cv.min()


def test_refine_plain_small_both_precisions(gpu):
    p = W.plain_small()
    announce("fourier refine plain-small")
    res, _, _ = run_refine(gpu, p.x, p.L, p.kappas)
    k_o = check_refine(res, p.x, p.L, p.kappas)
    res32, _, _ = run_refine(gpu, p.x.astype(np.float32), p.L, p.kappas)
    check_refine(res32, p.x.astype(np.float32).astype(np.float64), p.L, p.kappas)
    assert abs(res32[0] / k_o - 1) < 1e-3


def test_refine_edges(gpu):
    L = 2 * math.pi
    # two particles far apart: the objective rises from the first kappa
    kap = W.log_kappas(0.1, 1e3, 13)
    announce("fourier refine edge")
    res, _, _ = run_refine(gpu, np.array([0.5, 2.2]), L, kap)
    assert int(res[4]) == 0 and res[0] == kap[0]
    # one kappa: no bracket, the scan's value
    res1, cv1, _ = run_refine(gpu, np.array([0.5, 0.8, 2.0]), L, [3.0])
    assert res1[0] == 3.0 and res1[1] == cv1[0]


def run_adapt(kde, x, L, kstar, alpha):
    k, lg, nf = kde.adapt_widths_exact(to_gpu(x), L, kstar, alpha)
    return host(k), float(host(lg)[0]), int(host(nf)[0])


@pytest.mark.parametrize("n", [1, 5, 300, 4097])
@pytest.mark.parametrize("kstar", [0.5, 30.0, 2000.0])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adapt_exact(gpu, n, kstar, dtype):
    L = 4 * math.pi
    rng = np.random.default_rng([37, n])
    x = npx(W.cosine_positions(rng, n, L, 0.5, 0.5), dtype)
    alpha = 0.5
    announce("fourier adapt exact", n, kstar, dtype)
    k, lg, nf = run_adapt(gpu, x, L, kstar, alpha)
    x64 = x.astype(np.float64)
    ref, lg_ref, nf_ref = oref.adapt_widths_exact(x64, L, kstar, alpha)
    assert nf == nf_ref == 0
    if dtype == "f64":
        f = oref.pilot_exact(x64, L, kstar)
        k0 = 1.0 / (L * i0e(kstar))
        bound = 1e-12 + 2 * alpha * 64 * 2.0 ** -53 * k0 / f
        assert np.all(np.abs(k - ref) <= bound * ref)
        assert abs(lg - lg_ref) <= 1e-12 * max(1.0, abs(lg_ref)) + 64 * 2.0 ** -53 * k0 / f.min()
    else:
        assert rel_err(k, ref).max() <= 1e-6


def test_adapt_exact_against_grid_pilot_on_fine_grid(gpu):
    """With a pilot grid fine enough for linear interpolation to be exact to
    ~1e-7, the grid and exact pilots give the same widths to that level."""
    p = W.plain_small()
    x = to_gpu(p.x)
    kstar = 30.0
    k_exact, _, _ = gpu.adapt_widths_exact(x, p.L, kstar, 0.5)
    pilot = gpu.deposit(x, p.L, 4096, kappa=kstar)
    k_grid, _, _ = gpu.adapt_widths(x, p.L, pilot, kstar, 0.5)
    assert rel_err(host(k_grid), host(k_exact)).max() < 1e-5


def test_bad_arguments(gpu):
    import torch
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.KdeError):
        gpu.cv_scan_fourier(x, 1.0, [1.0, 2e6])            # beyond the Fourier limit
    with pytest.raises(gpu.KdeError):
        gpu.cv_scan_fourier(x, 1.0, [3.0, 1.0])            # not ascending
    with pytest.raises(gpu.KdeError):
        gpu.cv_refine(x[:1], 1.0, [1.0])                   # N < 2
    with pytest.raises(gpu.KdeError):
        gpu.adapt_widths_exact(x, 1.0, 0.0, 0.5)           # kappa* must be > 0


def test_refine_paper_scale_against_oracle_fourier_minimiser(gpu):
    """kde_cv_refine on the paper-scale CV subsample (65,536 particles, 32
    kappas in [1, 1e4]) against the oracle's Fourier-route objective (SciPy
    Bessel ratios, pinned to the direct sums) minimised by a bounded search
    in the same bracket: the objective at the minimiser to 1e-12 relative,
    the minimiser to the search's own resolution in log(kappa) (the minimum
    is flat: an objective known to 1e-16 pins it to about 1e-6)."""
    from scipy import optimize
    p = W.plain_paper_scale(n=1 << 16)
    x = p.x[:p.n_cv]
    announce("fourier refine paper-scale", len(x))
    res, cv, am = run_refine(gpu, x, p.L, p.kappas)
    lo, hi = oref.bracket(p.kappas, am)
    f = lambda u: float(ocv.cv_curve_fourier(x, p.L, [math.exp(u)])[0][0])
    r = optimize.minimize_scalar(f, bounds=(math.log(lo), math.log(hi)), method="bounded", options={"xatol": 1e-10})
    assert abs(res[1] - r.fun) <= 1e-12 * abs(r.fun)
    assert res[1] <= r.fun + 1e-14 * abs(r.fun)
    assert abs(math.log(res[0]) - r.x) <= 2e-5


def test_adapt_exact_full_size_sampled(gpu):
    """kde_adapt_widths_exact on all 1,048,576 paper-scale particles: the
    width ratios of sampled particles, kappa_i / kappa_0 = (f_i / f_0)^(2
    alpha), against the oracle's direct-sum pilot at those particles (the
    ratios do not involve the geometric mean over all N)."""
    p = W.plain_paper_scale()
    x = p.x
    kstar, alpha = 30.0, 0.5
    announce("fourier adapt exact full size", len(x))
    k, lg, nf = run_adapt(gpu, x, p.L, kstar, alpha)
    rng = np.random.default_rng(51)
    idx = np.concatenate([[0], rng.choice(len(x), 40, replace=False)])
    f = np.array([float(np.mean(kernel(x[i] - x, kstar, p.L))) for i in idx])
    ref = (f / f[0]) ** (2 * alpha)
    got = k[idx] / k[0]
    k0 = 1.0 / (p.L * i0e(kstar))
    bound = 1e-12 + 2 * alpha * 64 * 2.0 ** -53 * k0 * (1 / f + 1 / f[0])
    assert np.all(np.abs(got - ref) <= bound * ref)
    assert nf == 0
