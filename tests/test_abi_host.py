"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/kde.h declares, sizes workspaces, and rejects bad
arguments before enqueuing anything."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1804_11174_amd as kde

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(kde_[a-z_0-9]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    return kde.require_library()


def test_library_exports_every_declared_function(lib):
    names = declared_functions()
    assert {"kde_cv_scan", "kde_deposit", "kde_gather", "kde_adapt_widths", "kde_workspace_size"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n
    # the binding covers every declared function with the same name
    for n in names:
        assert hasattr(kde, n), n


def test_abi_version_and_status_text(lib):
    import re
    with open(os.path.join(ROOT, "include", "kde.h")) as f:
        declared = int(re.search(r"#define KDE_ABI_VERSION (\d+)", f.read()).group(1))
    assert kde.kde_abi_version() == declared
    assert kde.kde_status_str(0) == "ok"
    assert "argument" in kde.kde_status_str(1)


def dom(L=4 * math.pi, M=64, prec=kde.KDE_F64):
    return kde.kde_domain(L, M, prec)


def test_workspace_sizes_grow_with_n():
    a = kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom(), 4096, 8)
    b = kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom(), 65536, 32)
    assert 0 < a < b
    assert kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, dom(M=256), 1 << 20) > 0
    assert kde.kde_workspace_size(kde.KDE_OP_GATHER, dom(), 1000) == 0
    assert kde.kde_workspace_size(kde.KDE_OP_ADAPT, dom(), 1000) > 0
    # float form needs less room for the packed particles
    assert kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom(prec=kde.KDE_F32), 65536, 32) < b


@pytest.mark.parametrize("bad,msg", [
    (dict(L=-1.0), "L must"), (dict(L=float("nan")), "L must"), (dict(M=1), "M must"),
    (dict(M=5000), "M must"), (dict(prec=7), "prec"),
])
def test_workspace_size_rejects_bad_domain(bad, msg):
    d = dict(L=1.0, M=64, prec=kde.KDE_F64)
    d.update(bad)
    with pytest.raises(kde.KdeError) as e:
        kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, kde.kde_domain(d["L"], d["M"], d["prec"]), 100)
    assert msg in str(e.value) and e.value.status == 1


def _call_cv(lib, N, kappas, ws=None, ws_bytes=0, x=1):
    k = np.asarray(kappas, dtype=np.float64)
    d = dom()
    return lib.kde_cv_scan(ctypes.byref(d), N, x, len(k), k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           1, None, None, ws, ws_bytes, None)


def test_cv_scan_argument_checks(lib):
    # every failing case returns before touching the device (fake pointers)
    assert _call_cv(lib, 1, [1.0]) == 1 and "N must" in kde.kde_last_error()
    assert _call_cv(lib, 10, [2.0, 1.0]) == 1 and "ascending" in kde.kde_last_error()
    assert _call_cv(lib, 10, [-1.0]) == 1 and "kappa" in kde.kde_last_error()
    assert _call_cv(lib, 10, [float("inf")]) == 1
    assert _call_cv(lib, 10, list(range(1, 66))) == 1 and "B must" in kde.kde_last_error()
    # missing or unaligned or short workspace
    assert _call_cv(lib, 10, [1.0]) == 2
    assert _call_cv(lib, 10, [1.0], ws=256 + 8, ws_bytes=1 << 20) == 2 and "aligned" in kde.kde_last_error()
    assert _call_cv(lib, 10, [1.0], ws=4096, ws_bytes=16) == 2 and "too small" in kde.kde_last_error()


def test_deposit_gather_adapt_argument_checks(lib):
    d = dom()
    assert lib.kde_deposit(ctypes.byref(d), 10, None, None, 1.0, 1, None, 0, None) == 1
    assert lib.kde_deposit(ctypes.byref(d), 10, 1, None, -1.0, 1, None, 0, None) == 1
    assert lib.kde_gather(ctypes.byref(d), 0, 1, None, 1.0, 1, 1, None, 0, None) == 1
    assert lib.kde_adapt_widths(ctypes.byref(d), 10, 1, 1, 0.0, 0.5, 1, None, None, None, 0, None) == 1
    assert "kappa_star" in kde.kde_last_error()
    assert lib.kde_adapt_widths(ctypes.byref(d), 10, 1, 1, 3.0, -0.5, 1, None, None, None, 0, None) == 1
    assert lib.kde_workspace_size(99, ctypes.byref(d), 10, 0, ctypes.byref(ctypes.c_size_t())) == 1


def test_probe_argument_checks(lib):
    """The issue-rate probe rejects bad arguments before launching anything."""
    assert lib.kde_probe_peak(0, 8, 64, None, None) == 1            # no output buffer
    assert lib.kde_probe_peak(0, 0, 64, 1, None) == 1               # no workgroups
    assert lib.kde_probe_peak(0, 65537, 64, 1, None) == 1           # too many
    assert lib.kde_probe_peak(0, 8, 6, 1, None) == 1                # not a multiple of 4
    assert lib.kde_probe_peak(0, 8, (1 << 30) + 4, 1, None) == 1    # too many steps
    assert lib.kde_probe_peak(7, 8, 64, 1, None) == 1               # unknown kind
    assert b"kind" in lib.kde_last_error()


def test_shape_argument_checks(lib):
    """The triangle shape takes half-widths in (0, L/2]; an unknown shape and
    adaptive widths with the triangle are refused (fake pointers: every case
    fails before touching the device)."""
    L = 4 * math.pi
    tri = kde.kde_domain(L, 64, kde.KDE_F64, kde.KDE_SHAPE_TRIANGLE, 0)
    bad = kde.kde_domain(L, 64, kde.KDE_F64, 7, 0)
    with pytest.raises(kde.KdeError) as e:
        kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, bad, 100)
    assert "shape" in str(e.value)
    assert kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, tri, 1000, 8) == \
        kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom(), 1000, 8)

    def cv(widths):
        k = np.asarray(widths, dtype=np.float64)
        return lib.kde_cv_scan(ctypes.byref(tri), 10, 1, len(k), k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               1, None, None, None, 0, None)
    assert cv([0.0, 1.0]) == 1 and "half-width" in kde.kde_last_error()
    assert cv([1.0, 0.51 * L]) == 1 and "half-width" in kde.kde_last_error()
    assert cv([1.0, 0.5 * L]) == 2  # valid widths: stops at the missing workspace
    assert lib.kde_deposit(ctypes.byref(tri), 10, 1, None, 0.6 * L, 1, None, 0, None) == 1
    assert "half-width" in kde.kde_last_error()
    assert lib.kde_gather(ctypes.byref(tri), 10, 1, None, -1.0, 1, 1, None, 0, None) == 1
    assert lib.kde_adapt_widths(ctypes.byref(tri), 10, 1, 1, 3.0, 0.5, 1, None, None, None, 0, None) == 1
    assert "von Mises" in kde.kde_last_error()


def test_last_error_is_cleared_by_a_good_call():
    with pytest.raises(kde.KdeError):
        kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, dom(M=1), 100)
    assert kde.kde_last_error() != ""
    kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, dom(), 100)
    assert kde.kde_last_error() == ""


def test_tuning_table_round_trip():
    kde.kde_tune_set(kde.KDE_F64, [1000, 50000, 1 << 40], [4, 8, 16], [4, 0, 32])
    assert kde.kde_tune_get(kde.KDE_F64, 10) == (4, 4)
    assert kde.kde_tune_get(kde.KDE_F64, 1000) == (4, 4)
    assert kde.kde_tune_get(kde.KDE_F64, 1001) == (8, 0)
    assert kde.kde_tune_get(kde.KDE_F64, 10 ** 9) == (16, 32)
    assert kde.kde_tune_get(kde.KDE_F64, 1 << 50) == (16, 32)   # last entry covers everything larger
    kde.kde_tune_set(kde.KDE_F64, [1 << 40], [8])                # no group column: whole list per unit
    assert kde.kde_tune_get(kde.KDE_F64, 10) == (8, 0)
    with pytest.raises(kde.KdeError):
        kde.kde_tune_set(kde.KDE_F64, [10], [5])
    with pytest.raises(kde.KdeError):
        kde.kde_tune_set(kde.KDE_F64, [10, 5], [4, 8])
    with pytest.raises(kde.KdeError):                           # group not a multiple of chunk
        kde.kde_tune_set(kde.KDE_F64, [10], [8], [12])
    with pytest.raises(kde.KdeError):                           # group beyond the kappa limit
        kde.kde_tune_set(kde.KDE_F64, [10], [16], [80])
    with pytest.raises(kde.KdeError):                           # float passes are 4 or 8
        kde.kde_tune_set(kde.KDE_F32, [10], [16])
    # restore the shipped table (or the built-in default)
    if os.path.exists(kde.TUNE_FILE):
        kde.load_tuning(kde.TUNE_FILE)
    else:
        kde.kde_tune_set(kde.KDE_F64, [1 << 62], [16])


@pytest.mark.parametrize("a2", [0.05, 0.3, 1.0, 1.933, 2.492, 3.878, 7.0, 15.0])
def test_ad_pvalue_host_matches_oracle(a2):
    """The library's host p-value (its own trapezoid quadrature of the
    Anderson-Darling series) against the oracle's (SciPy quad of the same
    series, itself pinned to published points and a characteristic-function
    inversion)."""
    from oracle import adtest
    assert abs(kde.kde_ad_pvalue(a2) - adtest.ad_pvalue(a2)) <= 1e-9


def test_ad_pvalue_host_across_the_range():
    """The host p-value at 60 points log-spaced over A^2 in [0.02, 40]
    against the oracle's adaptive quadrature of the same series (1e-12
    absolute), and non-increasing in A^2 on a finer grid up to A^2 = 20
    (p above 1e-10; beyond, 1 - P(A^2 <= z) is below the resolution of
    the series' sum): the trapezoid step follows the width of the
    integrands' analytic strip, so no part of the range may lose accuracy."""
    import numpy as np
    from oracle import adtest
    for a2 in np.geomspace(0.02, 40.0, 60):
        assert abs(kde.kde_ad_pvalue(float(a2)) - adtest.ad_pvalue(float(a2))) <= 1e-12, a2
    p = [kde.kde_ad_pvalue(float(a2)) for a2 in np.geomspace(0.02, 20.0, 2000)]
    assert all(q <= r + 1e-15 for r, q in zip(p, p[1:]))


def test_ad_pvalue_host_published_tail_points():
    """The host p-value at Anderson and Darling's (1954) printed points,
    the 2.5 % and 1 % points included: the tail where the width-update rule
    acts (p <= 0.01 fires it, half of p_th re-fires it)."""
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "ad_critical_points.json")))
    assert len(g["points"]) >= 4
    for p in g["points"]:
        assert abs(kde.kde_ad_pvalue(p["a2"]) - p["upper_tail"]) <= p["abs_tol"], p


def test_ad_pvalue_host_matches_characteristic_function():
    """The host p-value against the Gil-Pelaez inversion of the limit law's
    characteristic function (an independent route), across the tail."""
    from tests.test_oracle_adapt_pic import ad_upper_tail_charfn
    for a2 in (2.492, 3.070, 3.0775, 3.857, 3.8781, 4.5, 6.0):
        assert abs(kde.kde_ad_pvalue(a2) - ad_upper_tail_charfn(a2)) <= 1e-9, a2


def test_cv_workspace_is_bounded_in_n():
    """The CV partial sums take at most 32,768 slot rows whatever N: at
    N = 2^20 and B = 64 the workspace is the packed positions (24 B per
    particle), the sort histogram and 32,768 x 128 doubles of slot sums,
    not 8.4 million tile pairs x 128 doubles."""
    n = 1 << 20
    w = kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom(), n, 64)
    assert w <= 24 * n + 8192 * 128 * 4 + 32768 * 128 * 8 + 256 * 128 * 8 + 64 * 1024
    # the allocation-free scan's array holds the paper-scale scan (N = 65,536, B = 32)
    for prec in (kde.KDE_F64, kde.KDE_F32):
        assert kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom(prec=prec), 65536, 32) <= (24 << 20)
        assert kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom(prec=prec), 16384, 64) <= (24 << 20)


def test_noalloc_scan_refuses_beyond_its_array_on_the_host(lib):
    """kde_cv_scan_noalloc checks its arguments and its size limit before
    anything touches the device (the pointers are never dereferenced)."""
    d = dom()
    k = np.linspace(1.0, 64.0, 64)
    kp = k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(4096)
    st = lib.kde_cv_scan_noalloc(ctypes.byref(d), 1 << 20, fake, 64, kp, fake, None, None, None)
    assert st == 2 and "holds" in kde.kde_last_error()
    st = lib.kde_cv_scan_noalloc(ctypes.byref(d), 1, fake, 64, kp, fake, None, None, None)
    assert st == 1


def test_ad_pvalue_edges():
    assert kde.kde_ad_pvalue(0.0) == 1.0
    assert kde.kde_ad_pvalue(-1.0) == 1.0
    assert kde.kde_ad_pvalue(500.0) == 0.0


def test_damping_rate_host_function_matches_oracle(lib):
    """kde_damping_rate runs on the host: against the oracle's two-peak
    slope on a noisy damped oscillation, and its argument checks."""
    from oracle import landau
    rng = np.random.default_rng(9)
    dt = 0.01
    t = np.arange(1500) * dt
    W = np.exp(-0.13 * t) * (np.cos(1.285 * t) ** 2 + 1e-3) * (1 + 1e-3 * rng.standard_normal(t.shape[0]))
    rate, peaks = kde.kde_damping_rate(W, dt)
    assert peaks == tuple(landau.first_two_peaks(W))
    assert rate == landau.damping_rate(W, dt) or abs(rate - landau.damping_rate(W, dt)) < 1e-15
    r2, p2 = kde.kde_damping_rate(np.exp(-np.arange(10.0)), dt)
    assert math.isnan(r2) and p2 == (-1, -1)
    with pytest.raises(kde.KdeError):
        kde.kde_damping_rate([1.0, 2.0], dt)
    with pytest.raises(kde.KdeError):
        kde.kde_damping_rate([1.0, 0.0, 1.0, 2.0], dt)
