"""The device's Bessel coefficient tables (csrc/bessel_coeffs.inc) against
mpmath, on the CPU: the small-argument fits I0(x) = Q((x/X0)^2) evaluated by
Horner's rule in the target precision on [0, reach X0] (the double pair
kernel uses its fit up to 1.01 X0 for concentrations whose every pair takes
that branch; float keeps X0), and the large-argument fits sqrt(x) I0e(x) =
P(X0/x) on [X0, 1e6]."""
import math
import os
import re

import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_1804_11174_amd", "csrc", "bessel_coeffs.inc")

# (X0 macro, small table, large table, dtype, relative bound, reach)
FORMS = {
    "f64": ("KDE_I0E_F64_X0", "KDE_I0E_F64_SMALL", "KDE_I0E_F64_FIT", np.float64, 2e-15, 1.01),
    "f32": ("KDE_I0E_F32_X0", "KDE_I0E_F32_SMALL", "KDE_I0E_F32_FIT", np.float32, 5e-7, 1.0),
}


def _table(text, name):
    body = re.search(r"#define %s \{([^}]*)\}" % name, text).group(1)
    return [float(v.strip().rstrip("f")) for v in body.split(",")]


def _macro(text, name):
    return float(re.search(r"#define %s ([0-9.eE+-]+)f?" % name, text).group(1))


def _horner(coef, t, dt):
    r = dt(coef[-1])
    for c in reversed(coef[:-1]):
        r = dt(r * t + dt(c))
    return float(r)


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_small_argument_fit_holds_to_its_reach(form):
    x0n, small, _, dt, bound, reach = FORMS[form]
    text = open(INC).read()
    x0 = _macro(text, x0n)
    coef = _table(text, small)
    worst = 0.0
    for k in range(401):
        x = reach * x0 * k / 400.0
        u = dt(x / x0)
        t = dt(u * u)
        ref = float(mpmath.besseli(0, x))
        worst = max(worst, abs(_horner(coef, t, dt) / ref - 1.0))
    assert worst < bound, worst


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_large_argument_fit(form):
    x0n, _, fit, dt, bound, _ = FORMS[form]
    text = open(INC).read()
    x0 = _macro(text, x0n)
    coef = _table(text, fit)
    worst = 0.0
    for x in np.geomspace(x0, 1e6, 300):
        v = dt(x0 / x)
        ref = float(mpmath.sqrt(x) * mpmath.besseli(0, x) * mpmath.exp(-x))
        worst = max(worst, abs(_horner(coef, v, dt) / ref - 1.0))
    assert worst < bound, worst
