"""GPU parity of kde_deposit, kde_gather and kde_adapt_widths against the
oracle, and of the paper-scale pipeline (CV scan -> pilot deposit -> adapt
-> adaptive deposit -> gather) at its full size on sampled outputs.

Tolerances: FP64 1e-12 relative per grid value and per concentration;
FP32 form 1e-6. Gathered values are compared normwise (max |diff| / max
|ref|) because a field crosses zero."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cv as ocv, density as od
from tests.gpu_util import announce, host, rel_err, to_gpu

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6}


def tdtype(dtype):
    import torch
    return torch.float64 if dtype == "f64" else torch.float32


def npx(x, dtype):
    return np.asarray(x, dtype=np.float64 if dtype == "f64" else np.float32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deposit_plain_small_all_kappas(gpu, dtype):
    p = W.plain_small()
    x = npx(p.x, dtype)
    xt = to_gpu(x)
    for k in p.kappas:
        announce("deposit plain-small", dtype, k)
        rho = host(gpu.deposit(xt, p.L, p.M, kappa=float(k)))
        ref = od.deposit(x.astype(np.float64), p.L, p.M, kappa=k)
        assert rel_err(rho, ref).max() <= TOL[dtype], (k, rel_err(rho, ref).max())


@pytest.mark.parametrize("M", [2, 7, 64, 100, 256, 257, 512, 1000, 4096])
@pytest.mark.parametrize("n", [1, 5, 300, 4097])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deposit_grid_and_particle_counts(gpu, M, n, dtype):
    L = 4 * math.pi
    rng = np.random.default_rng([11, M, n])
    x = npx(W.cosine_positions(rng, n, L, 0.3, 0.5), dtype)
    kap = npx(10.0 ** rng.uniform(-1, 3, n), dtype)
    announce("deposit sizes", M, n, dtype)
    rho = host(gpu.deposit(to_gpu(x), L, M, kappa_i=to_gpu(kap)))
    ref = od.deposit(x.astype(np.float64), L, M, kappa_i=kap.astype(np.float64))
    # relative per node, plus an absolute floor in units of the peak density
    # mean_i K_i(0): a kernel-tail term with exponent e carries about |e|
    # rounding units and |e| exp(e) <= 1/e, and float exponentials underflow
    from oracle.vonmises import i0e
    peak = np.mean(1.0 / (L * i0e(kap.astype(np.float64))))
    floor = (4 * 2.0 ** -24 if dtype == "f32" else 1e-15) * peak
    assert np.all(np.abs(rho - ref) <= TOL[dtype] * np.abs(ref) + floor)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_extreme_concentrations(gpu, dtype):
    """Per-particle concentrations from moderate to far beyond any use (up
    to 1e300 in double, where the exponent is clamped before the
    exponential; 1e30 in float) in one deposit and one gather, against the
    oracle. The floor is the moderate particles' peak density: the narrow
    kernels vanish at every node a particle does not sit on. In float a
    term with natural exponent e carries about (1 + |e|) rounding units and
    exp2 underflows near e = -104, so a value dominated by one narrow kernel
    is held to 128 units (7.6e-6) instead of 1e-6; in double |e| <= 1000
    after the clamp keeps every term within 1e-12."""
    L, M, n = 4 * math.pi, 256, 600
    rng = np.random.default_rng(74)
    x = npx(L * rng.random(n), dtype)
    big = [1e6, 1e12, 1e15, 1e300] if dtype == "f64" else [1e6, 1e12, 1e20, 1e30]
    kap = npx(rng.choice([5.0, 50.0] + big, n), dtype)
    announce("extreme kappas", dtype)
    rho = host(gpu.deposit(to_gpu(x), L, M, kappa_i=to_gpu(kap)))
    x64, k64 = x.astype(np.float64), kap.astype(np.float64)
    ref = od.deposit(x64, L, M, kappa_i=k64)
    from oracle.vonmises import i0e
    moderate = k64 <= 50.0
    peak = np.mean(1.0 / (L * i0e(k64[moderate]))) * moderate.mean()
    floor = (4 * 2.0 ** -24 if dtype == "f32" else 1e-15) * peak
    rel = TOL[dtype] if dtype == "f64" else 128 * 2.0 ** -24
    assert np.all(np.isfinite(rho))
    assert np.all(np.abs(rho - ref) <= rel * np.abs(ref) + floor)
    F = np.cos(2 * math.pi * np.arange(M) / M) + 1.5
    G = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa_i=to_gpu(kap)))
    ref_G = od.gather(x64, L, F, kappa_i=k64)
    assert np.all(np.isfinite(G))
    scale = np.abs(ref_G[moderate]).max()
    assert np.all(np.abs(G - ref_G) <= rel * np.abs(ref_G) + 4 * TOL[dtype] * scale)


def test_sharp_kernels_near_nodes(gpu):
    """FP64 deposit and gather with sharp kernels (kappa 1e4 .. 1e12) at
    1e-9 .. 1e-5 L from interior nodes, beside moderate ones: the exponent
    -2 kappa s^2 needs s with full relative accuracy there, which the
    half-angle tables alone do not give. Interior nodes only: the oracle's
    sin(pi (x_g - x) / L) itself loses that accuracy for d near +-L."""
    L, M = 4 * math.pi, 64
    dx = L / M
    rng = np.random.default_rng(75)
    nodes = rng.choice(np.arange(2, M - 2), 12, replace=False)
    offs = np.array([1e-9, -1e-9, 1e-7, -1e-7, 1e-5, -1e-5]) * L
    xs, ks = [], []
    for k, g in enumerate(nodes):
        for j, o in enumerate(offs):
            xs.append(g * dx + o)
            ks.append([1e4, 1e8, 1e12][(k + j) % 3])
    xm = L * rng.random(200)
    x = np.concatenate([np.array(xs), xm])
    kap = np.concatenate([np.array(ks), np.full(200, 5.0)])
    announce("sharp kernels near nodes")
    rho = host(gpu.deposit(to_gpu(x), L, M, kappa_i=to_gpu(kap)))
    ref = od.deposit(x, L, M, kappa_i=kap)
    from oracle.vonmises import i0e
    floor = 1e-15 * 200 / len(x) / (L * i0e(5.0))
    assert np.all(np.abs(rho - ref) <= TOL["f64"] * np.abs(ref) + floor), rel_err(rho, ref).max()
    F = np.cos(2 * math.pi * np.arange(M) / M) + 1.5
    G = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa_i=to_gpu(kap)))
    ref_G = od.gather(x, L, F, kappa_i=kap)
    bound = TOL["f64"] * np.abs(ref_G) + 1e-15 * np.abs(ref_G).max()
    bad = np.flatnonzero(~(np.abs(G - ref_G) <= bound))
    assert bad.size == 0, [(int(i), x[i], kap[i], G[i], ref_G[i]) for i in bad[:5]]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gather_and_adjointness(gpu, dtype):
    L, M, n = 4 * math.pi, 128, 3000
    rng = np.random.default_rng(12)
    x = npx(W.cosine_positions(rng, n, L, 0.5, 0.5), dtype)
    kap = npx(10.0 ** rng.uniform(0, 3.5, n), dtype)
    F = np.sin(2 * math.pi * np.arange(M) / M * 3) + 0.3
    announce("gather", dtype)
    G = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa_i=to_gpu(kap)))
    ref = od.gather(x.astype(np.float64), L, F, kappa_i=kap.astype(np.float64))
    assert np.abs(G - ref).max() <= TOL[dtype] * np.abs(ref).max()
    rho = host(gpu.deposit(to_gpu(x), L, M, kappa_i=to_gpu(kap)))
    lhs = (L / M) * np.dot(F, rho)
    assert abs(lhs - G.astype(np.float64).mean()) <= 4 * TOL[dtype] * np.abs(F).max()
    # global kappa path
    Gg = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa=40.0))
    refg = od.gather(x.astype(np.float64), L, F, kappa=40.0)
    assert np.abs(Gg - refg).max() <= TOL[dtype] * np.abs(refg).max()


@pytest.mark.parametrize("M", [7, 64, 100, 128, 257, 1000])
@pytest.mark.parametrize("n", [1, 5, 300, 4097, 40000])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gather_grid_and_particle_counts(gpu, M, n, dtype):
    """Gather at ragged particle counts and grid sizes that give every node
    split the kernel uses (1, 2, 4 or 8 lanes per particle, lane j over the
    nodes j, j + S, ...), against the oracle, per-particle widths."""
    L = 2.0
    rng = np.random.default_rng([21, M, n])
    x = npx(L * rng.random(n), dtype)
    kap = npx(10.0 ** rng.uniform(0, 4, n), dtype)
    F = np.cos(2 * math.pi * np.arange(M) / M) + 0.25 * np.sin(6 * math.pi * np.arange(M) / M) + 1.2
    announce("gather sizes", M, n, dtype)
    G = host(gpu.gather(to_gpu(x), L, to_gpu(F), kappa_i=to_gpu(kap)))
    ref = od.gather(x.astype(np.float64), L, F, kappa_i=kap.astype(np.float64))
    assert np.all(np.abs(G - ref) <= TOL[dtype] * np.abs(ref).max())


def test_gather_of_ones_matches_grid_sum_identity(gpu):
    from scipy import special
    L, M, k = 2 * math.pi, 64, 900.0
    x = L * np.random.default_rng(13).random(777)
    G = host(gpu.gather(to_gpu(x), L, to_gpu(np.ones(M)), kappa=k))
    th = 2 * math.pi * x / L
    q = np.arange(1, 30)
    expect = 1 + 2 * np.sum((special.ive(q * M, k) / special.ive(0, k))[None, :] * np.cos(np.outer(th, q * M)), 1)
    assert np.abs(G - expect).max() <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("alpha", [0.5, 0.0, 1.3])
def test_adapt_widths(gpu, dtype, alpha):
    L, M, n = 4 * math.pi, 256, 20000
    rng = np.random.default_rng(14)
    x = npx(W.cosine_positions(rng, n, L, 0.5, 0.5), dtype)
    pilot = od.deposit(x[:3000].astype(np.float64), L, M, kappa=30.0)
    announce("adapt", dtype, alpha)
    k_i, lg, nf = gpu.adapt_widths(to_gpu(x), L, to_gpu(pilot), 30.0, alpha)
    k_i, lg, nf = host(k_i), host(lg)[0], int(host(nf)[0])
    ref_k, ref_lg, ref_nf = od.adapt_widths(x.astype(np.float64), L, pilot, 30.0, alpha)
    assert rel_err(k_i, ref_k).max() <= TOL[dtype]
    assert abs(lg - ref_lg) <= TOL[dtype] * abs(ref_lg)
    assert nf == ref_nf == 0


def test_adapt_floors_zero_pilot(gpu):
    L, M = 1.0, 8
    pilot = np.array([0.0, 0.0, 0.0, 1.0, 2.0, 1.0, 0.5, 0.0])
    x = np.array([0.05, 0.3, 0.45, 0.6, 0.9, 0.99])
    k_i, lg, nf = gpu.adapt_widths(to_gpu(x), L, to_gpu(pilot), 5.0, 0.5)
    ref_k, ref_lg, ref_nf = od.adapt_widths(x, L, pilot, 5.0, 0.5)
    assert int(host(nf)[0]) == ref_nf >= 1
    assert rel_err(host(k_i), ref_k).max() <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_paper_scale_pipeline_sampled(gpu, dtype):
    """The full paper-scale pipeline at its real size: CV on the first 65,536
    of 1,048,576 particles (32 kappas), pilot deposit at kappa*, adaptive
    widths, adaptive deposit and gather of the adaptive density. Grid values
    are checked at 16 sampled nodes over all particles, widths everywhere,
    gathered values at 2048 sampled particles."""
    import torch
    p = W.plain_paper_scale()
    x = npx(p.x, dtype)
    xt = to_gpu(x)
    announce("pipeline paper-scale", dtype)
    cv, sums, am = gpu.cv_scan(xt[:p.n_cv], p.L, p.kappas)
    b = int(host(am)[0])
    kstar = float(p.kappas[b])
    ref_cv, _, _ = ocv.cv_curve_fourier(x[:p.n_cv].astype(np.float64), p.L, p.kappas)
    assert rel_err(host(cv), ref_cv).max() <= TOL[dtype]
    assert b == ocv.cv_argmin(ref_cv)
    pilot = gpu.deposit(xt, p.L, p.M, kappa=kstar)
    k_i, lg, nf = gpu.adapt_widths(xt, p.L, pilot, kstar, 0.5)
    rho = gpu.deposit(xt, p.L, p.M, kappa_i=k_i)
    G = gpu.gather(xt, p.L, rho, kappa_i=k_i)
    torch.cuda.synchronize()
    x64 = x.astype(np.float64)
    rng = np.random.default_rng(2)
    nodes = np.sort(rng.choice(p.M, 16, replace=False))
    xg = nodes * (p.L / p.M)
    # sampled pilot nodes, from all particles
    from oracle.vonmises import kernel
    pil = host(pilot)
    ref_pil = np.array([kernel(g - x64, kstar, p.L).mean() for g in xg])
    assert rel_err(pil[nodes], ref_pil).max() <= TOL[dtype]
    # widths from the GPU pilot (checked above): everything
    ref_k, ref_lg, _ = od.adapt_widths(x64, p.L, pil, kstar, 0.5)
    assert rel_err(host(k_i), ref_k).max() <= TOL[dtype]
    # adaptive density at sampled nodes from the oracle widths
    ki = host(k_i).astype(np.float64)
    r = host(rho)
    ref_r = np.array([kernel(g - x64, ki, p.L).mean() for g in xg])
    assert rel_err(r[nodes], ref_r).max() <= TOL[dtype]
    # gather of the GPU density at sampled particles
    idx = np.sort(rng.choice(len(x64), 2048, replace=False))
    ref_G = od.gather(x64[idx], p.L, r, kappa_i=ki[idx])
    Gs = host(G)[idx]
    assert np.abs(Gs - ref_G).max() <= TOL[dtype] * np.abs(ref_G).max()
