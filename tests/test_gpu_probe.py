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
