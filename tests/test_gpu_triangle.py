"""GPU parity of the first-order (triangular) shape of adjustable width:
kde_cv_scan, kde_deposit and kde_gather with dom.shape = triangle, against
the oracle's direct sums (oracle/triangle.py).

Tolerances: FP64 path 1e-12 relative per CV value, pair sum and grid value;
float form 1e-6 (CV values relative to the larger of the objective's two
terms, as for the von Mises kernel). Grid values are relative per node
plus a bound from the kernel's conditioning: the triangle's value
t = 1 - r/h has slope 1/h, so
the absolute rounding of the distance r (about u L in double, where
positions of size L enter; about u dx in float, where the offset from the
nearest node is rounded) becomes u S / h of absolute error in t, and the
rounding of r/h itself adds u (r/h <= 1 inside the support). Near the edge
of a support t is small and these absolute errors exceed the relative
tolerance; for narrow widths on fine grids they do so everywhere (the
oracle's own distances carry the same error). Gathered values are compared
normwise (a field crosses zero)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cv as ocv
from oracle import triangle as tri
from tests.gpu_util import announce, host, rel_err, to_gpu

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6}


def tdt(dtype):
    import torch
    return torch.float64 if dtype == "f64" else torch.float32


def npx(x, dtype):
    return np.asarray(x, dtype=np.float64 if dtype == "f64" else np.float32)


def f32_widths(h, L):
    """Half-widths rounded to float32 and kept inside (0, L/2]."""
    h32 = np.asarray(h, dtype=np.float32)
    top = np.float32(0.5 * L)
    if float(top) > 0.5 * L:
        top = np.nextafter(top, np.float32(0))
    return np.minimum(h32, top)


def conditioning_floor(x, L, M, h, dtype):
    """Per node: (1/N) sum over the particles whose support covers the node
    of 8 u (1 + S / h_i) / h_i (see the module docstring)."""
    x = np.asarray(x, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    u, S = (2.0 ** -53, L) if dtype == "f64" else (2.0 ** -24, L / M)
    g = np.arange(M) * (L / M)
    r = tri.periodic_distance(g[:, None] - x[None, :], L)
    cover = r < h[None, :] * (1 + 1e-6)
    return 8 * u * np.sum(cover * ((1 + S / h) / h)[None, :], axis=1) / len(x)


def gather_floor(L, M, h, F, dtype):
    """Per particle: the deposit's per-node bound 8 u (1 + S / h_i) / h_i
    times dx |F|max over the at most 2 h_i / dx + 2 nodes of its support."""
    h = np.asarray(h, dtype=np.float64)
    u, S = (2.0 ** -53, L) if dtype == "f64" else (2.0 ** -24, L / M)
    dx = L / M
    return dx * np.abs(F).max() * (2 * h / dx + 2) * 8 * u * (1 + S / h) / h


def widths_for(L, M, count):
    """Half-widths from a quarter cell to half the period, ascending; the
    widest ones (> L/4) reach their periodic image."""
    return np.geomspace(0.25 * L / M, 0.5 * L, count)


def run_cv(kde, x, L, widths, dtype):
    xt = to_gpu(npx(x, dtype))
    cv, sums, am = kde.cv_scan(xt, L, widths, shape=kde.KDE_SHAPE_TRIANGLE)
    return host(cv), host(sums), int(host(am)[0])


def check_cv(cv, sums, am, x64, L, widths, tol):
    ref_cv, S1, S2 = tri.cv_curve(x64, L, widths)
    n = len(x64)
    B = len(widths)
    first = (n * tri.conv2_at_zero(widths, L) + 2 * S1) / n ** 2
    if tol < TOL["f32"]:
        assert rel_err(cv, ref_cv).max() <= tol, rel_err(cv, ref_cv)
    else:
        # the float form's error is relative to the larger of the objective's
        # two terms: its distances carry a float rounding (the phase
        # difference converted to float, the width's scale), which a CV value
        # that is the difference of two near-equal terms keeps at their size
        err = np.abs(cv - ref_cv) / np.maximum(np.abs(ref_cv), first)
        assert err.max() <= tol, err
    # each pair sum is held to tol of the objective term it enters (a sum of
    # a few edge-of-support terms has no relative accuracy of its own)
    assert np.all(2 * np.abs(sums[:B] - S1) / n ** 2 <= tol * first)
    assert np.all(4 * np.abs(sums[B:] - S2) / (n * (n - 1)) <= tol * first)
    am_ref = ocv.cv_argmin(ref_cv)
    if am != am_ref:
        assert abs(ref_cv[am] - ref_cv[am_ref]) <= 2 * tol * np.abs(ref_cv).max()
    return ref_cv


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cv_plain_small_positions(gpu, dtype):
    p = W.plain_small()
    x = npx(p.x, dtype)
    widths = widths_for(p.L, p.M, 24)
    announce("tri cv plain-small", dtype, len(x))
    cv, sums, am = run_cv(gpu, x, p.L, widths, dtype)
    check_cv(cv, sums, am, x.astype(np.float64), p.L, widths, TOL[dtype])


@pytest.mark.parametrize("n", [2, 3, 7, 63, 64, 65, 255, 256, 257, 511, 600, 1025, 3001])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cv_small_and_ragged_sizes(gpu, n, dtype):
    L = 4 * math.pi
    rng = np.random.default_rng([17, n])
    x = npx(W.cosine_positions(rng, n, L, 0.4, 0.5), dtype)
    widths = np.array([1e-4, 0.01, 0.05, 0.2, 0.7, 2.0, 3.2, 0.26 * L, 0.4 * L, 0.5 * L])
    announce("tri cv ragged", n, dtype)
    cv, sums, am = run_cv(gpu, x, L, widths, dtype)
    check_cv(cv, sums, am, x.astype(np.float64), L, widths, TOL[dtype])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_cv_many_widths_wrapped_input(gpu, dtype):
    # B = 64 (several passes), positions off [0, L) (wrapped on the device)
    L = 2.75
    rng = np.random.default_rng(199)
    x = L * rng.random(2000) + L * rng.integers(-3, 3, 2000)
    x = npx(x, dtype)
    widths = np.geomspace(1e-3, 0.5 * L, 64)
    announce("tri cv B=64", dtype)
    cv, sums, am = run_cv(gpu, x, L, widths, dtype)
    from oracle.vonmises import wrap
    check_cv(cv, sums, am, wrap(x.astype(np.float64), L), L, widths, TOL[dtype])


def test_cv_clustered_positions_skip_far_tiles(gpu):
    """Two tight clusters half a period apart: with narrow widths whole tile
    pairs lie outside every support and are skipped; the sums must still
    equal the direct ones (including pairs that straddle x = 0)."""
    L = 1.0
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0.0, 0.01, 1500), rng.normal(0.5, 0.02, 1300)]) % L
    widths = np.array([1e-4, 1e-3, 4e-3, 0.01, 0.03])
    announce("tri cv clusters")
    cv, sums, am = run_cv(gpu, x, L, widths, "f64")
    check_cv(cv, sums, am, x, L, widths, 1e-12)


def test_cv_coincident_points_and_support_edges(gpu):
    # pairs at distance 0, exactly h, exactly 2h and L/2
    L = 8.0
    x = np.array([0.0, 0.0, 1.0, 2.0, 4.0, 4.0, 6.0, 7.5])
    widths = np.array([0.5, 1.0, 2.0, 4.0])
    announce("tri cv edges")
    cv, sums, am = run_cv(gpu, x, L, widths, "f64")
    check_cv(cv, sums, am, x, L, widths, 1e-12)


def test_cv_larger_n_invariance(gpu):
    """N = 65,536 paper-scale positions, 32 widths: rotation by a quarter
    period and reversal leave every CV value unchanged to rounding, and the
    float form agrees with the FP64 path to the float tolerance."""
    p = W.plain_paper_scale(n=1 << 16)
    x = p.x[:p.n_cv]
    widths = widths_for(p.L, p.M, 32)
    announce("tri cv paper-scale f64", len(x))
    a, _, am = run_cv(gpu, x, p.L, widths, "f64")
    b, _, _ = run_cv(gpu, (x + 0.25 * p.L) % p.L, p.L, widths, "f64")
    c, _, _ = run_cv(gpu, (p.L - x) % p.L, p.L, widths, "f64")
    assert rel_err(b, a).max() <= 1e-12 and rel_err(c, a).max() <= 1e-12
    announce("tri cv paper-scale f32", len(x))
    d, _, _ = run_cv(gpu, x.astype(np.float32), p.L, widths, "f32")
    ref32 = run_cv(gpu, x.astype(np.float32).astype(np.float64), p.L, widths, "f64")[0]
    assert rel_err(d, ref32).max() <= 1e-6


def test_cv_deterministic(gpu):
    p = W.plain_small()
    widths = widths_for(p.L, p.M, 16)
    a = run_cv(gpu, p.x, p.L, widths, "f64")
    b = run_cv(gpu, p.x, p.L, widths, "f64")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_bad_widths_raise(gpu):
    import torch
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    tri_shape = gpu.KDE_SHAPE_TRIANGLE
    with pytest.raises(gpu.KdeError):
        gpu.cv_scan(x, 1.0, [0.0, 0.1], shape=tri_shape)     # h = 0
    with pytest.raises(gpu.KdeError):
        gpu.cv_scan(x, 1.0, [0.1, 0.6], shape=tri_shape)     # h > L/2
    with pytest.raises(gpu.KdeError):
        gpu.deposit(x, 1.0, 16, kappa=0.0, shape=tri_shape)
    with pytest.raises(gpu.KdeError):
        gpu.adapt_widths(x, 1.0, torch.ones(16, dtype=torch.float64, device="cuda"), 0.1, 0.5,
                         shape=tri_shape)


@pytest.mark.parametrize("M", [2, 7, 64, 100, 256, 257, 512, 1000, 4096])
@pytest.mark.parametrize("n", [1, 5, 300, 4097])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deposit_sizes_per_particle_widths(gpu, M, n, dtype):
    L = 4 * math.pi
    rng = np.random.default_rng([21, M, n])
    x = npx(W.cosine_positions(rng, n, L, 0.3, 0.5), dtype)
    h = np.minimum(0.5 * L, (L / M) * 10.0 ** rng.uniform(-0.5, 1.5, n))
    h = f32_widths(h, L) if dtype == "f32" else h
    announce("tri deposit sizes", M, n, dtype)
    rho = host(gpu.deposit(to_gpu(x), L, M, kappa_i=to_gpu(h), shape=gpu.KDE_SHAPE_TRIANGLE))
    x64, h64 = x.astype(np.float64), h.astype(np.float64)
    ref = tri.deposit(x64, L, M, h_i=h64)
    floor = conditioning_floor(x64, L, M, h64, dtype)
    assert np.all(np.abs(rho - ref) <= TOL[dtype] * np.abs(ref) + floor)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deposit_global_width_is_cic_at_one_cell(gpu, dtype):
    """h = dx is standard PIC's linear weighting: every particle's weights
    on its two nodes sum to one, so the grid mass is exactly 1 / dx."""
    p = W.plain_small()
    x = npx(p.x, dtype)
    dx = p.L / p.M
    for h in (dx, 2.5 * dx, 0.5 * p.L):
        announce("tri deposit global", dtype, h)
        rho = host(gpu.deposit(to_gpu(x), p.L, p.M, kappa=float(h), shape=gpu.KDE_SHAPE_TRIANGLE))
        ref = tri.deposit(x.astype(np.float64), p.L, p.M, h=h)
        floor = conditioning_floor(x, p.L, p.M, np.full(len(x), h), dtype)
        assert np.all(np.abs(rho - ref) <= TOL[dtype] * np.abs(ref) + floor)
    rho = host(gpu.deposit(to_gpu(x), p.L, p.M, kappa=dx, shape=gpu.KDE_SHAPE_TRIANGLE))
    assert abs(rho.sum() * dx - 1.0) <= 4 * TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gather_and_adjointness(gpu, dtype):
    L, M, n = 4 * math.pi, 128, 3000
    rng = np.random.default_rng(22)
    x = npx(W.cosine_positions(rng, n, L, 0.5, 0.5), dtype)
    h = (L / M) * 10.0 ** rng.uniform(-0.3, 1.2, n)
    h = f32_widths(h, L) if dtype == "f32" else h
    F = np.sin(2 * math.pi * np.arange(M) / M * 3) + 0.3
    shape = gpu.KDE_SHAPE_TRIANGLE
    announce("tri gather", dtype)
    G = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa_i=to_gpu(h), shape=shape))
    ref = tri.gather(x.astype(np.float64), L, F, h_i=h.astype(np.float64))
    assert np.abs(G - ref).max() <= TOL[dtype] * np.abs(ref).max()
    rho = host(gpu.deposit(to_gpu(x), L, M, kappa_i=to_gpu(h), shape=shape))
    lhs = (L / M) * np.dot(F, rho)
    assert abs(lhs - G.astype(np.float64).mean()) <= 4 * TOL[dtype] * np.abs(F).max()
    Gg = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa=0.3, shape=shape))
    refg = tri.gather(x.astype(np.float64), L, F, h=0.3)
    assert np.abs(Gg - refg).max() <= TOL[dtype] * np.abs(refg).max()


@pytest.mark.parametrize("M", [2, 7, 64, 257, 1000])
@pytest.mark.parametrize("n", [1, 300, 4097])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gather_sizes_and_support_edges(gpu, M, n, dtype):
    """Triangle gather over ragged sizes with widths from 0.01 cells to L/2
    (short supports visit only the nodes near the particle, long ones the
    whole circle), whole-cell widths whose support ends on a node, and
    particles on nodes, at half cells and next to the wrap point; then
    h = dx on a constant field, where the two linear weights sum to one."""
    L = 3.0
    dx = L / M
    rng = np.random.default_rng([23, M, n])
    x = L * rng.random(n)
    x[: n // 4] = dx * rng.integers(0, M, n // 4)
    x[n // 4: n // 3] = dx * (rng.integers(0, M, n // 3 - n // 4) + 0.5)
    x[n // 3: n // 3 + 4] = [0.0, L * (1 - 1e-12), 1e-12, L - 0.5 * dx][: min(4, n - n // 3)]
    cells = 10.0 ** rng.uniform(-2, math.log10(max(M / 2, 1.01)), n)
    cells[::5] = rng.integers(1, max(2, M // 2) + 1, cells[::5].shape)
    h = np.minimum(0.5 * L, dx * cells)
    x = npx(x, dtype)
    h = f32_widths(h, L) if dtype == "f32" else h
    F = np.cos(2 * math.pi * np.arange(M) / M) + 0.5 * np.sin(10 * math.pi * np.arange(M) / M) + 1.1
    shape = gpu.KDE_SHAPE_TRIANGLE
    announce("tri gather sizes", M, n, dtype)
    G = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa_i=to_gpu(npx(h, dtype)), shape=shape))
    h64 = npx(h, dtype).astype(np.float64)
    ref = tri.gather(x.astype(np.float64), L, F, h_i=h64)
    assert np.all(np.abs(G - ref) <= TOL[dtype] * np.abs(ref).max() + gather_floor(L, M, h64, F, dtype))
    G1 = host(gpu.gather(to_gpu(x), L, to_gpu(np.ones(M)), kappa=dx, shape=shape))
    assert np.abs(G1 - 1.0).max() <= 8 * TOL[dtype]
