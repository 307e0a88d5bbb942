"""GPU parity of kde_cv_scan against the oracle (element by element).

Tolerances: FP64 path 1e-12 relative per CV value and per pair sum; FP32
form 1e-6 relative (positions rounded to float32 first, the oracle run in
float64 on the same rounded positions). The argmin must equal the oracle's,
or lie within the tie band where two CV values differ by less than twice
the error bound."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cv as ocv
from oracle.vonmises import conv2_at_zero
from tests.gpu_util import announce, host, rel_err, to_gpu

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6}


def run_gpu_cv(kde, x, L, kappas, dtype):
    import torch
    xt = to_gpu(x, torch.float64 if dtype == "f64" else torch.float32)
    cv, sums, am = kde.cv_scan(xt, L, kappas)
    return host(cv), host(sums), int(host(am)[0])


def assert_argmin_ok(am_gpu, cv_ref, tol):
    am_ref = ocv.cv_argmin(cv_ref)
    if am_gpu == am_ref:
        return
    band = 2 * tol * np.abs(cv_ref).max()
    assert abs(cv_ref[am_gpu] - cv_ref[am_ref]) <= band, (am_gpu, am_ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_plain_small_config(gpu, dtype):
    p = W.plain_small() if dtype == "f64" else W.precision_small()
    x64 = np.asarray(p.x, dtype=np.float64)
    announce("cv plain-small", dtype, len(x64), len(p.kappas))
    cv, sums, am = run_gpu_cv(gpu, p.x, p.L, p.kappas, dtype)
    ref_cv, S1, S2 = ocv.cv_curve(x64, p.L, p.kappas)
    tol = TOL[dtype]
    assert rel_err(cv, ref_cv).max() <= tol, rel_err(cv, ref_cv)
    assert rel_err(sums[:len(S1)], S1).max() <= tol
    assert rel_err(sums[len(S1):], S2).max() <= tol
    assert_argmin_ok(am, ref_cv, tol)


@pytest.mark.parametrize("n", [2, 3, 7, 63, 64, 65, 255, 256, 257, 511, 600, 1025])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_small_and_ragged_sizes(gpu, n, dtype):
    L = 4 * math.pi
    rng = np.random.default_rng([7, n])
    x = W.cosine_positions(rng, n, L, 0.4, 0.5)
    if dtype == "f32":
        x = x.astype(np.float32)
    kap = np.array([0.0, 1e-3, 0.7, 5.0, 19.0, 40.0, 90.0, 300.0, 2500.0, 2e4])
    announce("cv ragged", n, dtype)
    cv, sums, am = run_gpu_cv(gpu, x, L, kap, dtype)
    ref_cv, S1, S2 = ocv.cv_curve(np.asarray(x, np.float64), L, kap)
    tol = TOL[dtype]
    if dtype == "f64":
        assert rel_err(cv, ref_cv).max() <= tol
    else:
        # the float form's error is relative to the larger of the objective's
        # two terms: where CV crosses zero (here at the largest kappa) the
        # difference of two O(1/L) terms is smaller than either
        first = (n * conv2_at_zero(kap, L) + 2 * S1) / n ** 2
        assert np.all(np.abs(cv - ref_cv) <= tol * np.maximum(np.abs(ref_cv), first))
    B = len(kap)
    # pair sums: the kernel skips terms below exp(-70) times the largest
    # possible term (1/(L I0e(k)^2) for Kbar, 1/(L I0e(k)) for K)
    from oracle.vonmises import i0e
    if dtype == "f64":
        skipped = math.exp(-70.0) * n * n / 2
        for got, ref, w in ((sums[:B], S1, 1 / (L * i0e(kap) ** 2)), (sums[B:], S2, 1 / (L * i0e(kap)))):
            assert np.all(np.abs(got - ref) <= tol * np.abs(ref) + skipped * w)
    else:
        # a float exponent carries |exponent| ulps, so a sum made of a few
        # far-tail terms has no 1e-6 relative accuracy; each sum is held to
        # 1e-6 of the objective it enters instead
        first = (n * conv2_at_zero(kap, L) + 2 * S1) / n ** 2
        scale = np.maximum(np.abs(ref_cv), first)
        assert np.all(2 * np.abs(sums[:B] - S1) / n ** 2 <= tol * scale)
        assert np.all(4 * np.abs(sums[B:] - S2) / (n * (n - 1)) <= tol * scale)
    assert_argmin_ok(am, ref_cv, tol)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_many_kappas_and_odd_domain(gpu, dtype):
    # B = 64 (four chunks), unsorted-looking input, L not a multiple of pi
    L = 2.75
    rng = np.random.default_rng(99)
    x = L * rng.random(1500) + L * rng.integers(-3, 3, 1500)   # positions off [0, L): wrapped on device
    kap = W.log_kappas(0.05, 3e4, 64)
    xin = x.astype(np.float32) if dtype == "f32" else x
    announce("cv B=64", dtype)
    cv, sums, am = run_gpu_cv(gpu, xin, L, kap, dtype)
    from oracle.vonmises import wrap
    ref_cv, S1, S2 = ocv.cv_curve(wrap(np.asarray(xin, np.float64), L), L, kap)
    assert rel_err(cv, ref_cv).max() <= TOL[dtype]
    assert_argmin_ok(am, ref_cv, TOL[dtype])


def test_power_sums_on_far_tile_pairs(gpu):
    """Four clusters a quarter period apart, 1024 particles each (4096: 16
    tiles): on tile pairs of clusters half a period apart every pair has c
    near 0, so concentrations up to about 40 take the double kernel's
    power-sum route there, on neighbouring clusters up to about 11, and on
    near tile pairs only those below 8.08; the K-bar and K sums and the
    objective against the oracle's direct sums."""
    L = 2 * math.pi
    rng = np.random.default_rng([11174, 4, 4])
    x = np.concatenate([rng.normal(c * L / 4, 0.02, 1024) for c in range(4)])
    kap = np.array([1.0, 6.0, 8.05, 9.0, 11.0, 15.0, 25.0, 34.0, 39.0, 41.0, 60.0, 300.0])
    announce("cv power sums on far tile pairs", len(x))
    cv, sums, am = run_gpu_cv(gpu, x, L, kap, "f64")
    from oracle.vonmises import wrap
    ref_cv, S1, S2 = ocv.cv_curve(wrap(x, L), L, kap)
    assert rel_err(cv, ref_cv).max() <= TOL["f64"]
    B = len(kap)
    assert rel_err(sums[:B], S1).max() <= TOL["f64"]
    assert rel_err(sums[B:], S2).max() <= TOL["f64"]
    assert_argmin_ok(am, ref_cv, TOL["f64"])


def test_coincident_and_antipodal_points(gpu):
    # pairs at distance 0 (c = 1) and L/2 (c = 0) exercise both I0e regimes
    L = 2 * math.pi
    x = np.array([0.0, 0.0, math.pi, math.pi, 1.0, 1.0 + 1e-9, 4.0])
    kap = np.array([0.0, 0.5, 8.0, 60.0, 5000.0])
    announce("cv coincident")
    cv, sums, am = run_gpu_cv(gpu, x, L, kap, "f64")
    ref_cv, S1, S2 = ocv.cv_curve(x, L, kap)
    assert rel_err(cv, ref_cv).max() <= 1e-12


def test_paper_scale_against_fourier_identity(gpu):
    """N = 65,536, 32 kappas in [1, 1e4] (the CV scan of the paper-scale
    workload), checked against the oracle's Fourier-moment route (pinned to
    the direct sums on the CPU)."""
    p = W.plain_paper_scale(n=1 << 16)
    x = p.x[:p.n_cv]
    announce("cv paper-scale f64", len(x))
    cv, sums, am = run_gpu_cv(gpu, x, p.L, p.kappas, "f64")
    ref_cv, S1, S2 = ocv.cv_curve_fourier(x, p.L, p.kappas)
    assert rel_err(cv, ref_cv).max() <= 1e-12
    assert rel_err(sums[:32], S1).max() <= 1e-12
    assert rel_err(sums[32:], S2).max() <= 1e-12
    assert_argmin_ok(am, ref_cv, 1e-12)
    announce("cv paper-scale f32", len(x))
    cv32, _, am32 = run_gpu_cv(gpu, x.astype(np.float32), p.L, p.kappas, "f32")
    ref32, _, _ = ocv.cv_curve_fourier(x.astype(np.float32).astype(np.float64), p.L, p.kappas)
    assert rel_err(cv32, ref32).max() <= 1e-6
    assert_argmin_ok(am32, ref32, 1e-6)


def test_deterministic(gpu):
    p = W.plain_small()
    a = run_gpu_cv(gpu, p.x, p.L, p.kappas, "f64")
    b = run_gpu_cv(gpu, p.x, p.L, p.kappas, "f64")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    a = run_gpu_cv(gpu, p.x.astype(np.float32), p.L, p.kappas, "f32")
    b = run_gpu_cv(gpu, p.x.astype(np.float32), p.L, p.kappas, "f32")
    assert np.array_equal(a[0], b[0])


def test_permutation_changes_nothing_beyond_rounding(gpu):
    p = W.plain_small()
    rng = np.random.default_rng(5)
    a, _, _ = run_gpu_cv(gpu, p.x, p.L, p.kappas, "f64")
    b, _, _ = run_gpu_cv(gpu, rng.permutation(p.x), p.L, p.kappas, "f64")
    assert rel_err(a, b).max() <= 1e-13


def test_bad_arguments_raise(gpu):
    import torch
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.KdeError):
        gpu.cv_scan(x, 1.0, [3.0, 1.0])
    with pytest.raises(gpu.KdeError):
        gpu.cv_scan(x[:1], 1.0, [1.0])
    with pytest.raises(ValueError):
        gpu.cv_scan(x.to(torch.int32), 1.0, [1.0])


def test_extreme_concentrations(gpu):
    """Concentrations up to the scan's limit (1e12) on clustered positions
    (groups of three within 1e-7 L), so that waves stay live where other
    lanes' exponents reach about -2e12: the exponential's reduction must
    hold over that whole range. FP64, against the oracle."""
    L = 4 * math.pi
    rng = np.random.default_rng(73)
    base = L * rng.random(100)
    x = np.concatenate([base, base + 1e-7 * L * rng.random(100), base + 2e-7 * L * rng.random(100)]) % L
    kap = np.array([1.0, 1e3, 1e6, 1e9, 1e12])
    announce("cv extreme kappas")
    cv, sums, am = run_gpu_cv(gpu, x, L, kap, "f64")
    ref_cv, S1, S2 = ocv.cv_curve(x, L, kap)
    n, B = len(x), len(kap)
    assert rel_err(cv, ref_cv).max() <= TOL["f64"], rel_err(cv, ref_cv)
    from oracle.vonmises import i0e
    skipped = math.exp(-70.0) * n * n / 2
    for got, ref, w in ((sums[:B], S1, 1 / (L * i0e(kap) ** 2)), (sums[B:], S2, 1 / (L * i0e(kap)))):
        assert np.all(np.abs(got - ref) <= TOL["f64"] * np.abs(ref) + skipped * w)
    assert_argmin_ok(am, ref_cv, TOL["f64"])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_small_argument_range_boundary(gpu, dtype):
    """Concentrations with 2 kappa below the Bessel fits' switch point
    (16 in double, 8 in float) take their own loop; values on both sides of
    and at that point, against the oracle, on a ragged size with a diagonal
    tile pair."""
    L = 4 * math.pi
    rng = np.random.default_rng(71)
    x = W.cosine_positions(rng, 700, L, 0.4, 0.5)
    if dtype == "f32":
        x = x.astype(np.float32)
    kap = np.array([0.5, 3.99, 4.0, 4.01, 7.99, 8.0, 8.01, 20.0, 60.0])
    announce("cv small-argument boundary", dtype)
    cv, sums, am = run_gpu_cv(gpu, x, L, kap, dtype)
    ref_cv, S1, S2 = ocv.cv_curve(np.asarray(x, dtype=np.float64), L, kap)
    tol = TOL[dtype]
    n, B = len(x), len(kap)
    if dtype == "f64":
        from oracle.vonmises import i0e
        assert rel_err(cv, ref_cv).max() <= tol, rel_err(cv, ref_cv)
        skipped = math.exp(-70.0) * n * n / 2
        for got, ref, w in ((sums[:B], S1, 1 / (L * i0e(kap) ** 2)), (sums[B:], S2, 1 / (L * i0e(kap)))):
            assert np.all(np.abs(got - ref) <= tol * np.abs(ref) + skipped * w)
    else:
        first = (n * conv2_at_zero(kap, L) + 2 * S1) / n ** 2
        scale = np.maximum(np.abs(ref_cv), first)
        assert np.all(np.abs(cv - ref_cv) <= tol * scale)
        assert np.all(2 * np.abs(sums[:B] - S1) / n ** 2 <= tol * scale)
        assert np.all(4 * np.abs(sums[B:] - S2) / (n * (n - 1)) <= tol * scale)
    assert_argmin_ok(am, ref_cv, tol)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pass_size_changes_nothing(gpu, dtype):
    """The tuned pass size (concentrations per pass) and the split of a
    tile pair over workgroups by concentration range must not change any
    bit (20 and 32 concentrations, so the last group is ragged and the
    small-argument concentrations are split over groups)."""
    import torch
    p = W.plain_small()
    prec = gpu.KDE_F64 if dtype == "f64" else gpu.KDE_F32
    x = p.x if dtype == "f64" else p.x.astype(np.float32)
    shapes = [(4, 0), (8, 0), (16, 0), (4, 4), (4, 8), (8, 8), (16, 16), (8, 24)]
    if dtype == "f32":  # float passes are 4 or 8
        shapes = [(c, g) for c, g in shapes if c != 16]
    # 20 concentrations: 3 below the float Bessel split (2 kappa < 8) and 5
    # below the double one (2 kappa < 16); 32: 5 and 7, so groups of 4
    # split the small-argument concentrations of both forms over units
    for count in (20, 32):
        kap = W.log_kappas(1.0, 1e4, count)
        outs = []
        try:
            for c, g in shapes:
                gpu.kde_tune_set(prec, [1 << 62], [c], [g])
                outs.append(run_gpu_cv(gpu, x, p.L, kap, dtype))
        finally:
            if __import__("os").path.exists(gpu.TUNE_FILE):
                gpu.load_tuning(gpu.TUNE_FILE)
            else:
                gpu.kde_tune_set(prec, [1 << 62], [8])
        for o in outs[1:]:
            assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_slots_holding_several_tile_pairs(gpu, dtype):
    """N = 70,001: 274 tiles (the last one ragged) and 37,675 tile pairs
    dealt to 32,768 slots, so 4,907 slots sum two tile pairs from different
    bands of separation; against the oracle's Fourier-moment route (pinned
    to the direct sums on the CPU)."""
    L = 4 * math.pi
    x = W.cosine_positions(np.random.default_rng([7, 70001]), 70001, L, 0.3, 0.5)
    kap = W.log_kappas(1.0, 3e3, 12)
    if dtype == "f32":
        x = x.astype(np.float32)
    announce("cv several tile pairs per slot", dtype, len(x))
    cv, sums, am = run_gpu_cv(gpu, x, L, kap, dtype)
    ref_cv, S1, S2 = ocv.cv_curve_fourier(np.asarray(x, dtype=np.float64), L, kap)
    tol = TOL[dtype]
    assert rel_err(cv, ref_cv).max() <= tol, rel_err(cv, ref_cv)
    if dtype == "f64":
        assert rel_err(sums[:12], S1).max() <= tol
        assert rel_err(sums[12:], S2).max() <= tol
    assert_argmin_ok(am, ref_cv, tol)


def test_pass_size_changes_nothing_with_several_tile_pairs_per_slot(gpu):
    """The bitwise invariance of the pass size and concentration split at
    N = 80,000 (49,141 tile pairs over 32,768 slots), float form."""
    L = 4 * math.pi
    x = W.cosine_positions(np.random.default_rng([7, 80000]), 80000, L, 0.3, 0.5).astype(np.float32)
    kap = W.log_kappas(1.0, 1e4, 20)
    outs = []
    announce("cv pass size, several tile pairs per slot")
    try:
        for c, g in ((4, 0), (4, 8), (8, 0)):
            gpu.kde_tune_set(gpu.KDE_F32, [1 << 62], [c], [g])
            outs.append(run_gpu_cv(gpu, x, L, kap, "f32"))
    finally:
        if __import__("os").path.exists(gpu.TUNE_FILE):
            gpu.load_tuning(gpu.TUNE_FILE)
        else:
            gpu.kde_tune_set(gpu.KDE_F32, [1 << 62], [8])
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
