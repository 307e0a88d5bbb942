"""The issue-rate probe (kde_probe_peak): every kind runs a short launch and
writes one finite value per thread; the library's timing counts it under
its own id. The rates themselves are measurements, not checked here."""
import numpy as np
import pytest

from tests.gpu_util import announce, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_probe_runs_and_writes_every_thread(gpu, kind):
    import torch
    blocks = 4
    out = torch.full((blocks * 256,), float("nan"), dtype=torch.float64, device="cuda")
    announce("probe", kind)
    gpu.kde_timing_reset()
    gpu.kde_timing_enable(True)
    try:
        gpu.kde_probe_peak(kind, blocks, 64, out)
        torch.cuda.synchronize()
    finally:
        gpu.kde_timing_enable(False)
    v = host(out)
    assert np.all(np.isfinite(v))
    ms, n = gpu.kde_timing_read(gpu.KDE_KERNEL_PROBE)
    assert n == 1 and ms > 0.0
    with pytest.raises(ValueError):
        gpu.kde_probe_peak(kind, blocks * 2, 64, out)   # buffer too small for the launch


def test_timing_records_each_region_once(gpu):
    """Kernel timing with events the launches record themselves: one entry
    per timed region (the pair kernel; the deposit; the three kernels of the
    widths as one region), each positive and the pair kernel's no longer
    than the call; then a session whose steps replay a captured graph
    leaves no event that fails to read."""
    import math
    import time
    import torch
    import workloads as W
    from tests.gpu_util import to_gpu
    L, M = 4 * math.pi, 64
    x = to_gpu(W.cosine_positions(np.random.default_rng(5), 20000, L, 0.3, 0.5))
    kap = W.log_kappas(1.0, 1e3, 8)
    gpu.cv_scan(x, L, kap)
    torch.cuda.synchronize()
    announce("timing regions")
    gpu.kde_timing_reset()
    gpu.kde_timing_enable(True)
    try:
        t0 = time.perf_counter()
        gpu.cv_scan(x, L, kap)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        pilot = gpu.deposit(x, L, M, kappa=5.0)
        gpu.adapt_widths(x, L, pilot, 5.0, 0.5)
        torch.cuda.synchronize()
        counts = {k: gpu.kde_timing_read(k) for k in (gpu.KDE_KERNEL_CV_PAIRS, gpu.KDE_KERNEL_DEPOSIT,
                                                       gpu.KDE_KERNEL_ADAPT)}
        rng = W.rng_for(5, 96)
        s = gpu.Session(to_gpu(W.cosine_positions(rng, 4096, L, 0.01, 0.5)), to_gpu(W.maxwellian(rng, 4096, 1.0)),
                        L, M, 0.1, kap, 2048)
        s.step(3)  # the fixed part of a step is captured into a graph at the first step
        torch.cuda.synchronize()
        s.close()
    finally:
        gpu.kde_timing_enable(False)
    for k, (ms, n) in counts.items():
        assert n == 1 and ms > 0.0, (k, ms, n)
    assert counts[gpu.KDE_KERNEL_CV_PAIRS][0] <= wall_ms
    for k in (gpu.KDE_KERNEL_CV_PAIRS, gpu.KDE_KERNEL_DEPOSIT, gpu.KDE_KERNEL_GATHER, gpu.KDE_KERNEL_ADAPT):
        ms, n = gpu.kde_timing_read(k)  # raises if a recorded pair cannot be read
        if k in counts:
            assert n >= counts[k][1] and ms >= counts[k][0]
