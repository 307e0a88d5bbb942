"""GPU checks of the boundary's status and ordering rules: the numeric
status word (a non-finite position or width is reported as KDE_E_NUMERIC by
the waiting calls and by kde_numeric_check, and faults nothing), sessions
stepped by the request server (kde_server_attach), withdrawal of queued
requests, and the ordering of session creation and request submission after
the caller's stream."""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import announce, host, to_gpu

pytestmark = pytest.mark.gpu


def test_plain_calls_report_non_finite_inputs(gpu):
    import torch
    L, M = 4 * math.pi, 64
    x = W.cosine_positions(np.random.default_rng(3), 3000, L, 0.2, 0.5)
    gpu.kde_numeric_check()  # start from a clear word
    xt = to_gpu(x)
    gpu.cv_scan(xt, L, [1.0, 10.0, 100.0])
    gpu.deposit(xt, L, M, kappa=5.0)
    assert gpu.kde_numeric_check() == 0
    bad = x.copy()
    bad[1234] = np.nan
    announce("non-finite position in plain calls")
    cv, _, _ = gpu.cv_scan(to_gpu(bad), L, [1.0, 10.0, 100.0])
    assert np.isnan(host(cv)).all()
    assert gpu.kde_numeric_check() == gpu.KDE_NUMERIC_POSITION
    assert gpu.kde_numeric_check() == 0  # the check clears the word
    k = torch.full((3000,), 7.0, dtype=torch.float64, device="cuda")
    k[17] = float("inf")
    rho = gpu.deposit(xt, L, M, kappa_i=k)
    assert gpu.kde_numeric_check() == gpu.KDE_NUMERIC_CONCENTRATION
    k[17] = -1.0
    gpu.gather(xt, L, rho, kappa_i=k)
    assert gpu.kde_numeric_check() == gpu.KDE_NUMERIC_CONCENTRATION
    pilot = gpu.deposit(xt, L, M, kappa=5.0)
    gpu.adapt_widths(to_gpu(bad), L, pilot, 5.0)
    assert gpu.kde_numeric_check() == gpu.KDE_NUMERIC_POSITION
    # the float form reports the same
    gpu.cv_scan(to_gpu(bad, torch.float32), L, [1.0, 10.0])
    assert gpu.kde_numeric_check() == gpu.KDE_NUMERIC_POSITION


def test_session_reports_non_finite_state(gpu):
    L, M, n = 4 * math.pi, 64, 4096
    rng = W.rng_for(5, 91)
    x0 = W.cosine_positions(rng, n, L, 0.05, 0.5)
    v0 = W.maxwellian(rng, n, 1.0)
    kap = W.log_kappas(1.0, 1e3, 8)
    bad_x = x0.copy()
    bad_x[5] = np.nan
    with pytest.raises(gpu.KdeError) as e:
        gpu.Session(to_gpu(bad_x), to_gpu(v0), L, M, 0.1, kap, 2048)
    assert e.value.status == gpu.KDE_E_NUMERIC
    bad_v = v0.copy()
    bad_v[7] = np.inf  # finite positions now; the push makes one non-finite
    s = gpu.Session(to_gpu(x0), to_gpu(bad_v), L, M, 0.1, kap, 2048)
    try:
        announce("session stepping into a non-finite position")
        with pytest.raises(gpu.KdeError) as e:
            s.step(2)
        assert e.value.status == gpu.KDE_E_NUMERIC
        st = s.state()
        assert st["step"] == 1 and st["numeric"] != 0
    finally:
        s.close()


def test_batch_status_names_the_set(gpu):
    import torch
    L = 4 * math.pi
    xs, Ls, Ms = [], [], []
    for k in range(5):
        x = W.cosine_positions(np.random.default_rng([9, k]), 2000 + 300 * k, L, 0.2, 0.5)
        if k == 3:
            x[11] = np.nan
        xs.append(to_gpu(x, torch.float32))
        Ls.append(L)
        Ms.append(64)
    b = gpu.Batch(xs, Ls, Ms, W.log_kappas(1.0, 1e3, 8))
    try:
        b.run()
        flags = gpu.kde_batch_status(b.handle, 5)
        # set 3's position makes its pilot, and so its widths, non-finite too
        assert flags[3] & gpu.KDE_NUMERIC_POSITION and flags[:3] + flags[4:] == [0, 0, 0, 0], flags
    finally:
        b.close()


def _outs(x, M, B):
    import torch
    return (torch.empty(B, dtype=torch.float64, device="cuda"), torch.empty(M, dtype=torch.float64, device="cuda"),
            torch.empty(M, dtype=torch.float64, device="cuda"), torch.empty(x.shape[0], dtype=x.dtype, device="cuda"),
            torch.empty(1, dtype=torch.float64, device="cuda"))


def test_server_attached_sessions_match_direct_stepping(gpu):
    """Two sessions stepped by the server beside a stream of requests (one
    of them with a non-finite position) end bitwise where twins stepped
    directly end; the request with the bad position completes with
    KDE_E_NUMERIC and the others are unaffected."""
    import torch
    L, M, n = 4 * math.pi, 128, 16384
    kap = W.log_kappas(1.0, 1e4, 16)
    twins = []
    for k in range(2):
        rng = W.rng_for(5, 80 + k)
        x0 = to_gpu(W.cosine_positions(rng, n, L, 0.01, 0.5), torch.float32)
        v0 = to_gpu(W.maxwellian(rng, n, 1.0), torch.float32)
        twins.append((gpu.Session(x0, v0, L, M, 0.1, kap, 4096), gpu.Session(x0, v0, L, M, 0.1, kap, 4096)))
    reqs = []
    for r in range(12):
        x = W.cosine_positions(np.random.default_rng([12, r]), 3000 + 500 * r, L, 0.3, 0.5).astype(np.float32)
        if r == 5:
            x[100] = np.nan
        reqs.append((to_gpu(x), M))
    srv = gpu.Server(kap, prec=gpu.KDE_F32, budget_bytes=256 << 20, nslots=4, max_batch=8, n_cv=8192)
    try:
        announce("server with attached sessions")
        st_tickets = [srv.attach(a, 9) for a, _ in twins]
        outs = [_outs(x, Mr, 16) for x, Mr in reqs]
        tickets = [srv.submit(gpu.Server.request(x, L, Mr, o)) for (x, Mr), o in zip(reqs, outs)]
        srv.drain()
        for t in st_tickets:
            res = srv.poll(t)
            assert res["status"] == 0 and res["steps"] == 9
        for k, t in enumerate(tickets):
            res = srv.poll(t)
            assert res["status"] == (gpu.KDE_E_NUMERIC if k == 5 else 0), (k, res)
        st = srv.stats()
        assert st["session_steps"] == 18 and st["session_p50_s"] > 0 and st["failed"] == 1
        for a, b in twins:
            b.step(9)
            for f in (gpu.KDE_SESSION_X, gpu.KDE_SESSION_V, gpu.KDE_SESSION_KAPPA, gpu.KDE_SESSION_RHO):
                assert torch.equal(a.read(f), b.read(f)), f
            assert a.state() == b.state()
    finally:
        srv.close()
        for a, b in twins:
            a.close()
            b.close()


def test_server_budget_counts_attached_sessions_and_cancel(gpu):
    import torch
    L, M, n = 4 * math.pi, 64, 8192
    kap = W.log_kappas(1.0, 1e3, 8)
    rng = W.rng_for(5, 95)
    s = gpu.Session(to_gpu(W.cosine_positions(rng, n, L, 0.01, 0.5)), to_gpu(W.maxwellian(rng, n, 1.0)), L, M, 0.1,
                    kap, 2048)
    nbytes = gpu.kde_session_bytes(s.params)
    small = gpu.Server(kap, prec=gpu.KDE_F64, budget_bytes=nbytes // 2, nslots=1, max_batch=1)
    try:
        with pytest.raises(gpu.KdeError) as e:
            small.attach(s, 1)
        assert e.value.status == gpu.KDE_E_BUDGET
    finally:
        small.close()
    srv = gpu.Server(kap, prec=gpu.KDE_F64, budget_bytes=64 << 20, nslots=1, max_batch=1)
    try:
        xs = [to_gpu(W.cosine_positions(np.random.default_rng([13, r]), 20000, L, 0.3, 0.5)) for r in range(6)]
        outs = [_outs(x, M, 8) for x in xs]
        tickets = [srv.submit(gpu.Server.request(x, L, M, o)) for x, o in zip(xs, outs)]
        withdrawn = srv.cancel(tickets[-1])  # one slot: the last one is still queued
        srv.drain()
        assert withdrawn
        assert srv.poll(tickets[-1])["status"] == gpu.KDE_E_CANCELLED
        assert all(srv.poll(t)["status"] == 0 for t in tickets[:-1])
        assert srv.stats()["cancelled"] == 1
    finally:
        srv.close()
        s.close()


def test_create_and_submit_follow_the_callers_stream(gpu):
    """Inputs written by the caller's stream right before the call (behind a
    long spin on that stream): the session's copies and the request's work
    wait for them, so the results equal those from inputs that were ready."""
    import torch
    L, M, n = 4 * math.pi, 64, 8192
    kap = W.log_kappas(1.0, 1e3, 8)
    rng = W.rng_for(5, 96)
    x_ready = to_gpu(W.cosine_positions(rng, n, L, 0.05, 0.5))
    v_ready = to_gpu(W.maxwellian(rng, n, 1.0))
    ref = gpu.Session(x_ready, v_ready, L, M, 0.1, kap, 2048)
    x_late = torch.zeros_like(x_ready)
    v_late = torch.zeros_like(v_ready)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        torch.cuda._sleep(200_000_000)  # tens of milliseconds of spinning before the copies
        x_late.copy_(x_ready)
        v_late.copy_(v_ready)
        late = gpu.Session(x_late, v_late, L, M, 0.1, kap, 2048)
    try:
        for f in (gpu.KDE_SESSION_X, gpu.KDE_SESSION_V, gpu.KDE_SESSION_KAPPA):
            assert torch.equal(late.read(f), ref.read(f)), f
    finally:
        ref.close()
        late.close()
    srv = gpu.Server(kap, prec=gpu.KDE_F64, budget_bytes=64 << 20, nslots=2, max_batch=4)
    try:
        o_ready, o_late = _outs(x_ready, M, 8), _outs(x_ready, M, 8)
        t0 = srv.submit(gpu.Server.request(x_ready, L, M, o_ready))
        x2 = torch.zeros_like(x_ready)
        with torch.cuda.stream(stream):
            torch.cuda._sleep(200_000_000)
            x2.copy_(x_ready)
            t1 = srv.submit(gpu.Server.request(x2, L, M, o_late), stream)
        srv.drain()
        assert srv.poll(t0)["status"] == 0 and srv.poll(t1)["status"] == 0
        for a, b in zip(o_ready, o_late):
            assert torch.equal(a, b)
    finally:
        srv.close()


def test_server_detaches_a_cancelled_session_and_wait_blocks(gpu):
    """A session attached for unbounded steps detaches when cancelled: its
    ticket (kde_server_wait) ends with KDE_E_CANCELLED and the steps it took,
    after which it is where a twin stepped that many times directly is; the
    request submitted beside it completes through kde_server_wait."""
    import time
    import torch
    L, M, n = 4 * math.pi, 64, 8192
    kap = W.log_kappas(1.0, 1e3, 8)
    rng = W.rng_for(5, 97)
    x0 = to_gpu(W.cosine_positions(rng, n, L, 0.01, 0.5), torch.float32)
    v0 = to_gpu(W.maxwellian(rng, n, 1.0), torch.float32)
    a, b = gpu.Session(x0, v0, L, M, 0.1, kap, 2048), gpu.Session(x0, v0, L, M, 0.1, kap, 2048)
    srv = gpu.Server(kap, prec=gpu.KDE_F32, budget_bytes=64 << 20, nslots=2, max_batch=4)
    try:
        announce("attached session detached by cancel")
        st = srv.attach(a, 1 << 40)
        x = to_gpu(W.cosine_positions(np.random.default_rng([14, 1]), 5000, L, 0.3, 0.5).astype(np.float32))
        out = _outs(x, M, 8)
        res = srv.wait(srv.submit(gpu.Server.request(x, L, M, out)))
        assert res["status"] == 0
        t0 = time.monotonic()
        while srv.stats()["session_steps"] < 3 and time.monotonic() - t0 < 30:
            time.sleep(0.01)
        assert srv.cancel(st)
        res = srv.wait(st)
        assert res["status"] == gpu.KDE_E_CANCELLED and 3 <= res["steps"] < (1 << 40)
        assert srv.stats()["failed"] == 0
        b.step(int(res["steps"]))
        for f in (gpu.KDE_SESSION_X, gpu.KDE_SESSION_V, gpu.KDE_SESSION_KAPPA):
            assert torch.equal(a.read(f), b.read(f)), f
        assert a.state() == b.state()
        a.step(1)  # the caller owns it again
    finally:
        srv.close()
        a.close()
        b.close()
