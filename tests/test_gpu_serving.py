"""GPU checks of the serving form: resident PIC sessions against the
oracle's KDE-PIC step and width-update rule, checkpoint/restore, and the
request server (results identical alone and in a mix, budget admission)."""
import math
import threading

import numpy as np
import pytest

import workloads as W
from oracle import adtest, cv as ocv, density as od, pic, update, vonmises as vm
from tests.gpu_util import announce, host, rel_err, to_gpu

pytestmark = pytest.mark.gpu


def oracle_session(x0, v0, L, M, dt, kappas, n_cv, steps, alpha=0.5, thr=0.01, rate=0.05):
    def solve(x):
        c, _, _ = ocv.cv_curve(x[:n_cv], L, kappas)
        return kappas[ocv.cv_argmin(c)]
    k0 = solve(x0)
    st = update.initial_state(vm.width_from_kappa(k0, L), thr)
    pil = od.deposit(x0, L, M, kappa=k0)
    k_i, _, _ = od.adapt_widths(x0, L, pil, k0, alpha)
    x, v = x0.copy(), v0.copy()
    hist = []
    for _ in range(steps):
        x, v, rho, E = pic.field_step(x, v, k_i, L, M, dt)
        a2 = adtest.ad_statistic(x, L)
        p = adtest.ad_pvalue(a2)
        st, fired = update.step(st, p, lambda: vm.width_from_kappa(solve(x), L), thr, rate)
        kstar = float(vm.kappa_from_width(st.h_opt, L))
        pil = od.deposit(x, L, M, kappa=kstar)
        k_i, _, _ = od.adapt_widths(x, L, pil, kstar, alpha)
        hist.append(dict(a2=a2, p=p, fired=fired, kstar=kstar, rho=rho, E=E))
    return x, v, k_i, st, hist

def test_ad_statistic_with_tied_sort_keys(gpu):
    """Positions in clusters of four 1e-12 L apart, in descending order
    within each cluster: the double sort keys (L 2^-32 resolution) tie, so
    the runs of equal keys must be put in order by value. After one step of
    negligible motion (dt = 1e-15, cold start) the session's A^2 equals the
    oracle's on the positions it holds."""
    L, M, n = 4 * math.pi, 64, 4096
    rng = np.random.default_rng(77)
    base = L * (0.001 + 0.998 * rng.random(n // 4))
    x0 = np.concatenate([base + k * 1e-12 * L for k in (3, 2, 1, 0)])
    v0 = np.zeros(n)
    announce("AD statistic with tied keys")
    s = gpu.Session(to_gpu(x0), to_gpu(v0), L, M, 1e-15, W.log_kappas(1.0, 1e3, 8), 1024)
    try:
        s.step(1)
        a2 = s.state()["last_a2"]
        ref = adtest.ad_statistic(host(s.read(gpu.KDE_SESSION_X)), L)
        assert abs(a2 - ref) <= 1e-10 * abs(ref), (a2, ref)
    finally:
        s.close()


@pytest.mark.parametrize("alpha_density", [0.1, 0.01])
def test_session_steps_match_oracle(gpu, alpha_density):
    L, M, n, dt = 4 * math.pi, 64, 2048, 0.1
    rng = W.rng_for(5, 77)
    x0 = W.cosine_positions(rng, n, L, alpha_density, 0.5)
    v0 = W.maxwellian(rng, n, 1.0)
    kappas = W.log_kappas(1.0, 1e4, 16)
    n_cv, steps = 1024, 3
    announce("session vs oracle", alpha_density)
    s = gpu.Session(to_gpu(x0), to_gpu(v0), L, M, dt, kappas, n_cv)
    try:
        ox, ov, ok, ost, hist = oracle_session(x0, v0, L, M, dt, kappas, n_cv, steps)
        fired = 0
        for k in range(steps):
            s.step(1)
            info = s.state()
            h = hist[k]
            assert abs(info["last_a2"] - h["a2"]) <= 1e-10 * abs(h["a2"])
            assert abs(info["last_p"] - h["p"]) <= 1e-9
            fired += int(h["fired"])
            assert info["fired"] == fired
            assert abs(info["kappa_star"] - h["kstar"]) <= 1e-12 * h["kstar"]
        rho = host(s.read(gpu.KDE_SESSION_RHO))
        E = host(s.read(gpu.KDE_SESSION_E))
        assert rel_err(rho, hist[-1]["rho"]).max() <= 1e-11
        assert np.abs(E - hist[-1]["E"]).max() <= 1e-11 * np.abs(hist[-1]["E"]).max()
        x = host(s.read(gpu.KDE_SESSION_X))
        v = host(s.read(gpu.KDE_SESSION_V))
        dx = np.abs(x - ox)
        dx = np.minimum(dx, L - dx)
        assert dx.max() <= 1e-11
        assert np.abs(v - ov).max() <= 1e-11
        assert rel_err(host(s.read(gpu.KDE_SESSION_KAPPA)), ok).max() <= 1e-10
        assert abs(info["h_opt"] - ost.h_opt) <= 1e-12 * ost.h_opt
        assert abs(info["p_th"] - ost.p_th) <= 1e-9
    finally:
        s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_session_checkpoint_restore_is_bitwise(gpu, dtype):
    import torch
    L, M, n, dt = 4 * math.pi, 128, 8192, 0.1
    rng = W.rng_for(5, 78)
    td = torch.float64 if dtype == "f64" else torch.float32
    x0 = to_gpu(W.cosine_positions(rng, n, L, 0.05, 0.5), td)
    v0 = to_gpu(W.maxwellian(rng, n, 1.0), td)
    kappas = W.log_kappas(1.0, 1e4, 16)
    a = gpu.Session(x0, v0, L, M, dt, kappas, 4096)
    b = gpu.Session(x0, v0, L, M, dt, kappas, 4096)
    try:
        a.step(3)
        blob = a.save()
        a.step(4)
        b.restore(blob)
        b.step(4)
        for f in (gpu.KDE_SESSION_X, gpu.KDE_SESSION_V, gpu.KDE_SESSION_KAPPA, gpu.KDE_SESSION_RHO,
                  gpu.KDE_SESSION_E):
            assert torch.equal(a.read(f), b.read(f)), f
        assert a.state() == b.state()
    finally:
        a.close()
        b.close()


def plain_outputs(gpu, x, L, M, kappas, n_cv):
    cv, _, am = gpu.cv_scan(x[:n_cv], L, kappas)
    b = int(host(am)[0])
    kstar = float(kappas[b])
    pilot = gpu.deposit(x, L, M, kappa=kstar)
    k_i, _, _ = gpu.adapt_widths(x, L, pilot, kstar, 0.5)
    rho = gpu.deposit(x, L, M, kappa_i=k_i)
    return host(cv), kstar, host(pilot), host(k_i), host(rho)


def make_requests(count, seed, n_lo=500, n_hi=40000, dtype=None):
    import torch
    td = dtype or torch.float32
    rng = np.random.default_rng([5, 1000, seed])
    reqs = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        M = int(rng.choice([64, 128, 256, 512]))
        alpha = float(rng.uniform(0.01, 0.5))
        L = 4 * math.pi
        x = to_gpu(W.cosine_positions(rng, n, L, alpha, 0.5).astype(np.float32), td)
        reqs.append((x, L, M))
    return reqs


def test_server_results_same_alone_and_in_mix(gpu):
    """Requests served with several slots and batching, while a PIC session
    steps on its own stream, give the same bits as each request alone."""
    import torch
    kappas = W.log_kappas(1.0, 1e4, 16)
    n_cv = 8192
    reqs = make_requests(40, seed=1)
    srv = gpu.Server(kappas, prec=gpu.KDE_F32, budget_bytes=64 << 20, nslots=4, max_batch=8, n_cv=n_cv)
    outs = []
    for x, L, M in reqs:
        outs.append((torch.empty(len(kappas), dtype=torch.float64, device="cuda"),
                     torch.empty(M, dtype=torch.float64, device="cuda"),
                     torch.empty(M, dtype=torch.float64, device="cuda"),
                     torch.empty(x.shape[0], dtype=x.dtype, device="cuda"),
                     torch.empty(1, dtype=torch.float64, device="cuda")))
    rng = W.rng_for(5, 79)
    sx = to_gpu(W.cosine_positions(rng, 16384, 4 * math.pi, 0.01, 0.5).astype(np.float32))
    sv = to_gpu(W.maxwellian(rng, 16384, 1.0).astype(np.float32))
    sess = gpu.Session(sx, sv, 4 * math.pi, 128, 0.1, kappas, 4096)
    stop = threading.Event()

    def stepper():
        while not stop.is_set():
            sess.step(1)

    th = threading.Thread(target=stepper)
    th.start()
    try:
        announce("server mix", len(reqs))
        tickets = [srv.submit(gpu.Server.request(x, L, M, o)) for (x, L, M), o in zip(reqs, outs)]
        srv.drain()
    finally:
        stop.set()
        th.join()
    try:
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["rejected"] == 0
        assert st["p50_s"] <= st["p99_s"] <= st["max_s"]
        batch_sizes = [srv.poll(t)["batch_size"] for t in tickets]
        assert max(batch_sizes) > 1          # some requests were admitted together
        for (x, L, M), o in zip(reqs, outs):
            cv, kstar, pilot, k_i, rho = plain_outputs(gpu, x, L, M, kappas, min(n_cv, x.shape[0]))
            assert np.array_equal(host(o[0]), cv)
            assert host(o[4])[0] == kstar
            assert np.array_equal(host(o[1]), pilot)
            assert np.array_equal(host(o[3]), k_i)
            assert np.array_equal(host(o[2]), rho)
        assert sess.state()["step"] > 0
    finally:
        srv.close()
        sess.close()


def test_server_budget_admission(gpu):
    import torch
    kappas = W.log_kappas(1.0, 1e4, 16)
    reqs = make_requests(6, seed=2, n_lo=20000, n_hi=30000)
    outs = [(torch.empty(16, dtype=torch.float64, device="cuda"), torch.empty(M, dtype=torch.float64, device="cuda"),
             torch.empty(M, dtype=torch.float64, device="cuda"), torch.empty(x.shape[0], dtype=x.dtype, device="cuda"),
             torch.empty(1, dtype=torch.float64, device="cuda")) for x, L, M in reqs]
    # a budget that holds one request at a time: admission must serialise them
    probe = gpu.Server(kappas, budget_bytes=1 << 30, nslots=1, max_batch=1)
    one = max(gpu.kde_server_request_bytes(probe.handle, gpu.Server.request(x, L, M, o)) for (x, L, M), o in zip(reqs, outs))
    probe.close()
    srv = gpu.Server(kappas, budget_bytes=one + 4096, nslots=4, max_batch=8)
    try:
        for (x, L, M), o in zip(reqs, outs):
            srv.submit(gpu.Server.request(x, L, M, o))
        srv.drain()
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["mean_batch"] == 1.0
        # a request larger than the whole budget is refused at submission
        big = to_gpu(np.linspace(0, 10, 200000).astype(np.float32))
        bo = (torch.empty(16, dtype=torch.float64, device="cuda"), torch.empty(64, dtype=torch.float64, device="cuda"),
              torch.empty(64, dtype=torch.float64, device="cuda"), torch.empty(200000, dtype=torch.float32, device="cuda"),
              torch.empty(1, dtype=torch.float64, device="cuda"))
        with pytest.raises(gpu.KdeError) as e:
            srv.submit(gpu.Server.request(big, 4 * math.pi, 64, bo, n_cv=200000))
        assert e.value.status == gpu.KDE_E_BUDGET
    finally:
        srv.close()


def test_server_large_requests_run_alone_in_order(gpu):
    """With every request classed large (threshold of one term), requests
    run one at a time in arrival order, each in a batch of its own, even
    with several free slots; small ones (default threshold) still batch."""
    import time
    import torch
    kappas = W.log_kappas(1.0, 1e4, 16)
    reqs = make_requests(6, seed=3, n_lo=3000, n_hi=9000)
    outs = [(torch.empty(16, dtype=torch.float64, device="cuda"), torch.empty(M, dtype=torch.float64, device="cuda"),
             torch.empty(M, dtype=torch.float64, device="cuda"), torch.empty(x.shape[0], dtype=x.dtype, device="cuda"),
             torch.empty(1, dtype=torch.float64, device="cuda")) for x, L, M in reqs]
    srv = gpu.Server(kappas, budget_bytes=1 << 30, nslots=4, max_batch=8, large_slots=1, large_terms=1.0)
    try:
        sub, tickets = [], []
        for (x, L, M), o in zip(reqs, outs):
            sub.append(time.perf_counter())
            tickets.append(srv.submit(gpu.Server.request(x, L, M, o)))
        srv.drain()
        res = [srv.poll(t) for t in tickets]
    finally:
        srv.close()
    assert all(r is not None and r["status"] == 0 and r["batch_size"] == 1 for r in res)
    start = [s + r["queue_s"] for s, r in zip(sub, res)]
    end = [s + r["latency_s"] for s, r in zip(sub, res)]
    assert start == sorted(start), "large requests must start in arrival order"
    for k in range(len(res) - 1):
        assert end[k] <= start[k + 1] + 5e-4, f"large requests {k} and {k + 1} overlapped"


def _session_tolerances(dtype, rho_ref, L, kappa_peak):
    """Bounds of one session step in the given form, from its arithmetic.

    Deposit: each grid value to ``r`` relative (1e-12 in double; 1e-6 in the
    float form, plus 4u of the peak kernel value for the exponent rounding of
    far terms). The charge 1 - L rho cancels most of rho, so its error is
    L |d rho| absolute; the Poisson solve with the mean removed and the
    centred difference map a charge error q to a field error of at most
    2 L max|q| (the half-node fields are running sums of dx (q - mean) with
    zero sum). The gather weights of a particle sum to about 1, so the
    gathered field carries that field error plus its own relative rounding;
    the push then adds dt times that to v, and one rounding of v and of x
    (and the storage rounding of x after the wrap) in the form's precision."""
    u = 2.0 ** -24 if dtype == "f32" else 2.0 ** -53
    r = 1e-6 if dtype == "f32" else 1e-12
    drho = r * np.asarray(rho_ref) + 4 * u * kappa_peak
    dE = 2.0 * L * L * drho.max()
    return dict(u=u, r=r, drho=drho, dE=dE)


@pytest.mark.parametrize("dtype,steps", [("f32", 3), ("f64", 2)])
def test_session_at_serving_shape_matches_oracle_stepwise(gpu, dtype, steps):
    """A session of the serving form at its own shape (262,144 particles,
    M = 128, L = 4 pi, dt = 0.1, 16 concentrations in [1, 1e4], CV on the
    first 65,536, alpha = 0.5, threshold 0.01, rate 0.05), held to the
    oracle step by step from the session's own state: before each step x,
    v and kappa_i are read back, the oracle runs one KDE-PIC step (Sec.
    III.A) and the update rule (Sec. II.D) from them, and the session's
    deposit, field, positions, velocities, A^2, p-value, rule decision,
    kappa* and next widths are compared. Step 1 fires the rule here (A^2
    of the 1 % perturbation is about 4.7), so the in-step CV scan on the
    pushed positions is held too (argmin equal, or within the float form's
    tie band). The oracle's CV goes through its Fourier-moment route, which
    is pinned to the direct pair sums on the CPU."""
    import torch
    from oracle import vonmises as vmo
    s0 = W.pic_session(0)
    L, M, dt, kappas, n_cv = s0.L, s0.M, s0.dt, s0.kappas, s0.n_cv
    td = torch.float32 if dtype == "f32" else torch.float64
    announce("serving-shape session", dtype, len(s0.x))
    sess = gpu.Session(to_gpu(s0.x, td), to_gpu(s0.v, td), L, M, dt, kappas, n_cv)
    band = lambda c: 2 * (1e-6 if dtype == "f32" else 1e-12) * np.abs(c).max()
    try:
        info = sess.state()
        x = host(sess.read(gpu.KDE_SESSION_X)).astype(np.float64)
        # creation: CV scan at t = 0, pilot at its optimum, widths
        c0, _, _ = ocv.cv_curve_fourier(x[:n_cv], L, kappas)
        b_or = ocv.cv_argmin(c0)
        b_gpu = int(np.argmin(np.abs(kappas - info["kappa_star"])))
        assert kappas[b_gpu] == info["kappa_star"]
        assert b_gpu == b_or or abs(c0[b_gpu] - c0[b_or]) <= band(c0), (b_gpu, b_or)
        k_gpu = host(sess.read(gpu.KDE_SESSION_KAPPA)).astype(np.float64)
        pil = od.deposit(x, L, M, kappa=info["kappa_star"])
        k_ref, _, _ = od.adapt_widths(x, L, pil, info["kappa_star"], 0.5)
        tol_k = 3e-6 if dtype == "f32" else 1e-11
        assert rel_err(k_gpu, k_ref).max() <= tol_k, rel_err(k_gpu, k_ref).max()
        fired_total = 0
        for k in range(steps):
            before = sess.state()
            x = host(sess.read(gpu.KDE_SESSION_X)).astype(np.float64)
            v = host(sess.read(gpu.KDE_SESSION_V)).astype(np.float64)
            ki = host(sess.read(gpu.KDE_SESSION_KAPPA)).astype(np.float64)
            announce("serving-shape session step", dtype, k + 1)
            sess.step(1)
            info = sess.state()
            rho = od.deposit(x, L, M, kappa_i=ki)
            E = pic.efield_centered(pic.poisson_fd(pic.charge_from_density(rho, L), L / M), L / M)
            Ei = od.gather(x, L, E, kappa_i=ki)
            xr, vr = pic.push(x, v, Ei, dt, L)
            peak = float(np.mean(1.0 / (L * vmo.i0e(ki))))
            t = _session_tolerances(dtype, rho, L, peak)
            g_rho = host(sess.read(gpu.KDE_SESSION_RHO))
            g_E = host(sess.read(gpu.KDE_SESSION_E))
            g_x = host(sess.read(gpu.KDE_SESSION_X)).astype(np.float64)
            g_v = host(sess.read(gpu.KDE_SESSION_V)).astype(np.float64)
            e_rho = np.abs(g_rho - rho)
            e_E = np.abs(g_E - E).max()
            dEi = 1.05 * t["dE"] + 2 * t["r"] * np.abs(E).max()
            dv = dt * dEi + 2 * t["u"] * (np.abs(v) + np.abs(Ei) * dt)
            ex = np.abs(g_x - xr)
            ex = np.minimum(ex, L - ex)
            dx = dt * dv + 3 * t["u"] * L
            print(f"[{dtype} step {k + 1}] rho rel {np.max(e_rho / rho):.2e}  E {e_E:.2e} "
                  f"(bound {t['dE']:.2e}, |E| {np.abs(E).max():.2e})  v {np.max(np.abs(g_v - vr)):.2e}  "
                  f"x {ex.max():.2e}", flush=True)
            assert np.all(e_rho <= t["drho"]), np.max(e_rho / t["drho"])
            assert e_E <= t["dE"], (e_E, t["dE"])
            assert np.all(np.abs(g_v - vr) <= dv), np.max(np.abs(g_v - vr) / dv)
            assert np.all(ex <= dx), np.max(ex / dx)
            # Anderson-Darling on the session's own pushed positions
            a2 = adtest.ad_statistic(g_x, L)
            assert abs(info["last_a2"] - a2) <= 1e-10 * abs(a2), (info["last_a2"], a2)
            p = adtest.ad_pvalue(a2)
            assert abs(info["last_p"] - p) <= 1e-9
            # the rule from the session's state before the step
            st = update.UpdateState(before["p_th"], before["h_opt"], before["h_target"])
            solved = {}

            def solve():
                c, _, _ = ocv.cv_curve_fourier(g_x[:n_cv], L, kappas)
                solved["c"] = c
                return vmo.width_from_kappa(kappas[ocv.cv_argmin(c)], L)

            st_ref, fired = update.step(st, p, solve, 0.01, 0.05)
            fired_total += int(fired)
            assert info["fired"] == fired_total, (info["fired"], fired_total)
            if fired:
                c = solved["c"]
                b_gpu = int(np.argmin(np.abs(vmo.width_from_kappa(kappas, L) - info["h_target"])))
                assert abs(info["h_target"] - vmo.width_from_kappa(kappas[b_gpu], L)) <= 1e-15 * info["h_target"]
                b_or = ocv.cv_argmin(c)
                assert b_gpu == b_or or abs(c[b_gpu] - c[b_or]) <= band(c), (b_gpu, b_or)
                st_ref = update.UpdateState(st_ref.p_th, 0.05 * info["h_target"] + 0.95 * before["h_opt"],
                                            info["h_target"])
            assert abs(info["p_th"] - st_ref.p_th) <= 1e-9
            assert abs(info["h_target"] - st_ref.h_target) <= 1e-14 * st_ref.h_target
            assert abs(info["h_opt"] - st_ref.h_opt) <= 1e-14 * st_ref.h_opt
            kstar = float(vmo.kappa_from_width(st_ref.h_opt, L))
            assert abs(info["kappa_star"] - kstar) <= 1e-13 * kstar
            # the next step's widths from the pilot at kappa*
            pil = od.deposit(g_x, L, M, kappa=info["kappa_star"])
            k_ref, _, _ = od.adapt_widths(g_x, L, pil, info["kappa_star"], 0.5)
            k_gpu = host(sess.read(gpu.KDE_SESSION_KAPPA)).astype(np.float64)
            assert rel_err(k_gpu, k_ref).max() <= tol_k, rel_err(k_gpu, k_ref).max()
        assert fired_total >= 1
    finally:
        sess.close()
