"""The allocation-free CV scan (kde_cv_scan_noalloc) against kde_cv_scan,
through the C ABI: two calls in a row, the second smaller, each compared
with the workspace entry point on the same input (same kernels, so the
same bits; the bar of the scan itself is 1e-12 relative in FP64 and 1e-6
in float, both far looser)."""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import announce, host, to_gpu

pytestmark = pytest.mark.gpu


def scan_both(kde, x, L, kappas, prec):
    import torch
    dom = kde.kde_domain(L, 2, prec)
    B, n = len(kappas), x.shape[0]
    outs = []
    for which in ("workspace", "noalloc"):
        cv = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
        sums = torch.full((2 * B,), float("nan"), dtype=torch.float64, device="cuda")
        am = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        if which == "workspace":
            ws = kde.Workspace("cuda")
            ptr, cap = ws.get(kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom, n, B))
            kde.kde_cv_scan(dom, n, x, kappas, cv, sums, am, ptr, cap)
        else:
            kde.kde_cv_scan_noalloc(dom, n, x, kappas, cv, sums, am)
        outs.append((host(cv), host(sums), int(host(am)[0])))
    return outs


def test_noalloc_scan_matches_workspace_scan_twice(gpu):
    import torch
    p = W.plain_paper_scale(n=1 << 16)
    x = to_gpu(p.x[:p.n_cv], torch.float64)
    announce("noalloc scan 1: N = 65,536, B = 32, f64")
    (a_cv, a_s, a_am), (b_cv, b_s, b_am) = scan_both(gpu, x, p.L, p.kappas, gpu.KDE_F64)
    assert np.isfinite(b_cv).all() and np.isfinite(b_s).all()
    assert np.array_equal(a_cv, b_cv) and np.array_equal(a_s, b_s) and a_am == b_am
    # a second, smaller call: whatever the first left in the array must not leak in
    L = 4 * math.pi
    y = to_gpu(W.cosine_positions(np.random.default_rng(91), 3001, L, 0.2, 0.5).astype(np.float32))
    kap = W.log_kappas(1.0, 1e3, 8)
    announce("noalloc scan 2: N = 3,001, B = 8, f32")
    (a_cv, a_s, a_am), (b_cv, b_s, b_am) = scan_both(gpu, y, L, kap, gpu.KDE_F32)
    assert np.isfinite(b_cv).all()
    assert np.array_equal(a_cv, b_cv) and np.array_equal(a_s, b_s) and a_am == b_am


def test_noalloc_refuses_scans_beyond_its_array(gpu):
    import torch
    x = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    cv = torch.empty(64, dtype=torch.float64, device="cuda")
    dom = gpu.kde_domain(1.0, 2, gpu.KDE_F64)
    with pytest.raises(gpu.KdeError) as e:  # N = 65,536 at B = 64 needs 34 MiB
        gpu.kde_cv_scan_noalloc(dom, 1 << 16, x, np.linspace(1, 64, 64), cv, None, None)
    assert e.value.status == 2  # KDE_E_WORKSPACE
