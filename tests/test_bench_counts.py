"""The benchmark's exact term counts behind its roofline figures, against
brute force on small inputs: count_evaluated_terms (the (pair, kappa)
terms of the von Mises CV sums whose K-bar exponent -2 kappa (1 - cos(pi d
/ L)) is at least -70, d the periodic distance) and count_tri_terms (the
(pair, width) terms of the triangle CV sums inside the support, d < 2 h,
or every pair once 2 h reaches L/2)."""
import importlib.util
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _distances(x, L):
    xs = np.asarray(x, dtype=np.float64) % L
    d = np.abs(xs[:, None] - xs[None, :])
    d = np.minimum(d, L - d)
    iu = np.triu_indices(len(xs), 1)
    return d[iu]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_evaluated_terms_match_brute_force(bench, seed):
    rng = np.random.default_rng([11174, 99, seed])
    L = 4 * math.pi
    x = np.concatenate([rng.uniform(-L, 2 * L, 250), rng.normal(3.0, 0.05, 60)])  # a cluster and wrapped values
    kappas = [1e-3, 1.0, 34.9, 35.0, 36.0, 200.0, 1e4, 1e7]
    d = _distances(x, L)
    brute = sum(int(np.count_nonzero(-2.0 * k * (1.0 - np.cos(math.pi * d / L)) >= -bench.SKIP_EXPONENT))
                for k in kappas)
    assert bench.count_evaluated_terms(x, L, kappas) == brute


@pytest.mark.parametrize("seed", [0, 1])
def test_triangle_terms_match_brute_force(bench, seed):
    rng = np.random.default_rng([11174, 98, seed])
    L = 2 * math.pi
    x = rng.uniform(0.0, L, 400)
    widths = [0.01, 0.1, 0.5, 1.2, L / 4 + 1e-9, L / 2]
    d = _distances(x, L)
    n = len(x)
    brute = 0
    for h in widths:
        brute += n * (n - 1) // 2 if 2 * h >= L / 2 else int(np.count_nonzero(d < 2 * h))
    assert bench.count_tri_terms(x, L, widths) == brute


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_pair_kernel_ops_prices_each_branch(bench, prec):
    # small-argument concentrations (2 kappa below the Bessel split, 1.01
    # times it in double: 8.05 is one there, 8.1 is not) have
    # every pair's term at their own price plus the per-pair power sums; the
    # rest are priced per evaluated term; counts by brute force
    rng = np.random.default_rng([11174, 97, 0 if prec == "f64" else 1])
    L = 4 * math.pi
    x = rng.uniform(0.0, L, 300)
    kappas = [0.5, 3.0, 7.9, 8.05, 8.1, 50.0, 3e3]
    d = _distances(x, L)
    pairs = len(d)
    x0 = {"f64": 16.0 * 1.01, "f32": 8.0}[prec]  # the small-argument fits' reach
    pure_k = [k for k in kappas if 2.0 * k < x0]
    rest = sum(int(np.count_nonzero(-2.0 * k * (1.0 - np.cos(math.pi * d / L)) >= -bench.SKIP_EXPONENT))
               for k in kappas if 2.0 * k >= x0)
    per_term = {"f64": 46, "f32": 20}[prec]
    pure_term = {"f64": 15 + 1, "f32": 5 + 12 + 2}[prec]
    per_pair = {"f64": 20 + 21, "f32": 0}[prec]
    want = rest * per_term + len(pure_k) * pairs * pure_term + pairs * per_pair
    ops, evaluated, pure = bench.pair_kernel_ops(x, L, kappas, prec)
    assert pure == len(pure_k) * pairs
    assert evaluated == rest + pure
    assert ops == want


def test_power_sum_route_is_safe_and_counted(bench):
    # four tight clusters a quarter period apart: tiles of far clusters take
    # concentrations above X0/2 on the power-sum route; every pair on the
    # route must have 2 kappa |cos(pi d / L)| below 1.01 X0 (the fit's reach),
    # and the route's evaluated terms are counted by brute force
    rng = np.random.default_rng([11174, 96])
    L = 2 * math.pi
    x = np.concatenate([rng.normal(c * L / 4, 0.01, 512) for c in range(4)])
    kappas = [1.0, 4.0, 9.0, 12.0, 20.0, 36.0, 500.0]
    detail = []
    terms, evaluated, wpairs = bench.power_sum_route(x, L, kappas, detail)
    xs = np.asarray(x) % L
    n = len(x)
    npure = sum(1 for k in kappas if 2 * k < 1.01 * 16.0)
    assert terms > npure * n * (n - 1) // 2  # the route reaches past the small concentrations
    want_terms = want_eval = want_pairs = 0
    for ti, tj, pe in detail:
        d = np.abs(xs[ti][:, None] - xs[tj][None, :])
        d = np.minimum(d, L - d)
        same = ti[0] == tj[0]
        live = np.triu(np.ones_like(d, dtype=bool), 1) if same else np.ones_like(d, dtype=bool)
        c = np.abs(np.cos(math.pi * d / L))
        for b in range(pe):
            k = kappas[b]
            if 2 * k >= 1.01 * 16.0:
                assert np.all(2 * k * c[live] < 1.01 * 16.0)
            want_eval += int(np.count_nonzero(live & (-2 * k * (1 - c) >= -bench.SKIP_EXPONENT)))
        want_terms += pe * int(np.count_nonzero(live))
        want_pairs += int(np.count_nonzero(live))
    assert (terms, evaluated, wpairs) == (want_terms, want_eval, want_pairs)


def test_basis_constants_follow_the_kernel_sources(bench):
    # the route and skip rules bench.py replays are the kernel's own: the
    # double small-argument reach, the Bessel split points and the skip bound
    import re
    csrc = os.path.join(ROOT, "paper_1804_11174_amd", "csrc")
    dev_cv = open(os.path.join(csrc, "dev_cv.hpp")).read()
    internal = open(os.path.join(csrc, "kde_internal.hpp")).read()
    coeffs = open(os.path.join(csrc, "bessel_coeffs.inc")).read()
    reach = re.search(r"struct PureReach<double> \{\s*static constexpr double value = ([0-9.]+);", dev_cv)
    assert reach and float(reach.group(1)) == bench.PURE_REACH["f64"]
    assert bench.PURE_REACH["f32"] == 1.0
    skip = re.search(r"constexpr double kSkipExponent = ([0-9.]+);", internal)
    assert skip and float(skip.group(1)) == bench.SKIP_EXPONENT
    for prec, macro in (("f64", "KDE_I0E_F64_X0"), ("f32", "KDE_I0E_F32_X0")):
        x0 = re.search(r"#define %s ([0-9.]+)f?" % macro, coeffs)
        assert x0 and float(x0.group(1)) == bench.BESSEL_X0[prec]
    tile = re.search(r"constexpr int kCvTile = (\d+);", internal)
    assert tile and int(tile.group(1)) == bench.CV_TILE
    # the cell count of the sort that orders the tiles: n / 32, clamped to [1, 8192]
    layout = open(os.path.join(csrc, "layout.hip")).read()
    assert "int64_t cells = n / 32;" in layout and "if (cells > 8192) cells = 8192;" in layout
