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
