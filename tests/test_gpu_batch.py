"""GPU checks of the batching form: every set's outputs from one graph
launch are bitwise identical to the one-set calls on that set, repeated
graph launches give identical results, and sampled sets match the oracle."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import cv as ocv, density as od
from tests.gpu_util import announce, host, rel_err, to_gpu

pytestmark = pytest.mark.gpu


def small_sets(count, n_hi=6000, seed=0):
    """Sets shaped like the batching workload (N log-uniform, alpha, k, M
    drawn per set) at sizes the oracle can check."""
    out = []
    rng = np.random.default_rng([4242, seed])
    for s in range(count):
        n = int(round(math.exp(rng.uniform(math.log(300), math.log(n_hi)))))
        alpha = float(rng.uniform(0.01, 0.5))
        k = float(rng.choice([0.5, 1.0, 2.0]))
        M = int(rng.choice([64, 128, 256]))
        L = 2 * math.pi / k
        out.append((W.cosine_positions(rng, n, L, alpha, k), L, M))
    # edge shapes: the smallest set, ragged tiles, a grid above 256 nodes
    out.append((W.cosine_positions(rng, 2, 3.0, 0.1, 1.0), 3.0, 2))
    out.append((W.cosine_positions(rng, 257, 5.0, 0.3, 1.0), 5.0, 300))
    return out


def plain(gpu, x, L, M, kappas, alpha=0.5):
    cv, sums, am = gpu.cv_scan(x, L, kappas)
    b = int(host(am)[0])
    kstar = float(kappas[b])
    pilot = gpu.deposit(x, L, M, kappa=kstar)
    k_i, _, _ = gpu.adapt_widths(x, L, pilot, kstar, alpha)
    rho = gpu.deposit(x, L, M, kappa_i=k_i)
    return host(cv), kstar, host(pilot), host(k_i), host(rho)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_equals_one_set_calls_bitwise(gpu, dtype):
    import torch
    sets = small_sets(14, seed=1 if dtype == "f64" else 2)
    td = torch.float64 if dtype == "f64" else torch.float32
    kappas = W.log_kappas(1.0, 1e4, 16)
    xs = [to_gpu(x, td) for x, _, _ in sets]
    announce("batch", dtype, len(sets))
    bt = gpu.Batch(xs, [L for _, L, _ in sets], [M for _, _, M in sets], kappas)
    try:
        bt.run()
        torch.cuda.synchronize()
        ks = host(bt.kappa_star)
        for s, (x, L, M) in enumerate(sets):
            cv, kstar, pilot, k_i, rho = plain(gpu, xs[s], L, M, kappas)
            assert np.array_equal(host(bt.cv[s]), cv), s
            assert ks[s] == kstar, s
            assert np.array_equal(host(bt.pilot[s]), pilot), s
            assert np.array_equal(host(bt.kappa_i[s]), k_i), s
            assert np.array_equal(host(bt.rho[s]), rho), s
    finally:
        bt.close()


def test_batch_graph_replays_are_identical_and_match_oracle(gpu):
    import torch
    sets = small_sets(6, n_hi=2500, seed=3)
    kappas = W.log_kappas(1.0, 1e4, 16)
    xs = [to_gpu(x) for x, _, _ in sets]
    bt = gpu.Batch(xs, [L for _, L, _ in sets], [M for _, _, M in sets], kappas)
    try:
        first = None
        for rep in range(3):
            bt.run()
            # eager work on the same stream between replays
            gpu.cv_scan(xs[0], sets[0][1], kappas)
            torch.cuda.synchronize()
            now = [host(r).copy() for r in bt.rho] + [host(bt.kappa_star).copy()]
            if first is None:
                first = now
            else:
                for a, b in zip(first, now):
                    assert np.array_equal(a, b)
        # oracle on two sets: CV curve, argmin, adaptive density
        for s in (0, len(sets) - 1):
            x, L, M = sets[s]
            ref_cv, _, _ = ocv.cv_curve(x, L, kappas)
            assert rel_err(host(bt.cv[s]), ref_cv).max() <= 1e-12
            b = ocv.cv_argmin(ref_cv)
            assert host(bt.kappa_star)[s] == kappas[b]
            pil = od.deposit(x, L, M, kappa=kappas[b])
            k_i, _, _ = od.adapt_widths(x, L, pil, kappas[b], 0.5)
            ref_rho = od.deposit(x, L, M, kappa_i=k_i)
            assert rel_err(host(bt.rho[s]), ref_rho).max() <= 1e-11
    finally:
        bt.close()


def test_batch_rejects_bad_sets(gpu):
    import torch
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu.KdeError):
        gpu.Batch([x[:1]], [1.0], [8], [1.0, 2.0])
    with pytest.raises(gpu.KdeError):
        gpu.Batch([x], [1.0], [1], [1.0, 2.0])
    with pytest.raises(gpu.KdeError):
        gpu.Batch([x], [1.0], [8], [2.0, 1.0])


def test_batching_workload_full_size(gpu):
    """The batching workload at its real size (512 sets, N log-uniform in
    [1e3, 1e5], float form, 16 kappas): four sets spread over the cost order
    are compared bitwise with the one-set calls and with the oracle (CV by
    the Fourier-moment route, adaptive density at sampled nodes)."""
    import torch
    sets = W.batch_sets(512)
    kappas = sets[0].problem.kappas
    xs = [to_gpu(s.problem.x.astype(np.float32)) for s in sets]
    announce("batching workload 512 sets f32")
    bt = gpu.Batch(xs, [s.problem.L for s in sets], [s.problem.M for s in sets], kappas)
    try:
        bt.run()
        torch.cuda.synchronize()
        ks = host(bt.kappa_star)
        for si in (0, 128, 256, 384):
            p = sets[si].problem
            x32 = p.x.astype(np.float32)
            cv, kstar, pilot, k_i, rho = plain(gpu, xs[si], p.L, p.M, kappas)
            assert np.array_equal(host(bt.cv[si]), cv) and ks[si] == kstar
            assert np.array_equal(host(bt.rho[si]), rho)
            ref_cv, S1, S2 = ocv.cv_curve_fourier(x32.astype(np.float64), p.L, kappas)
            n = len(x32)
            from oracle.vonmises import conv2_at_zero
            first = (n * conv2_at_zero(kappas, p.L) + 2 * S1) / n ** 2
            assert np.all(np.abs(cv - ref_cv) <= 1e-6 * np.maximum(np.abs(ref_cv), first))
            b = ocv.cv_argmin(ref_cv)
            if kappas[b] != kstar:   # tie band of the float form
                assert abs(ref_cv[list(kappas).index(kstar)] - ref_cv[b]) <= 2e-6 * np.abs(ref_cv).max()
            from oracle.vonmises import kernel
            ki = k_i.astype(np.float64)
            x64 = x32.astype(np.float64)
            nodes = np.arange(0, p.M, max(1, p.M // 8))
            ref_r = np.array([kernel(g * p.L / p.M - x64, ki, p.L).mean() for g in nodes])
            assert rel_err(rho[nodes], ref_r).max() <= 1e-6
    finally:
        bt.close()
