"""GPU checks of the Landau-damping workload (Sec. III.B): standard-PIC
sessions (linear weighting) and the field-energy history against the
oracle, checkpoints with the history, and a short physics run of both
methods on one seeded ensemble.

Tolerances: positions, velocities and grid fields of the FP64 sessions to
1e-11 relative (normwise for fields that cross zero) after a few steps --
the same bar as the KDE sessions; field energies to 1e-11 relative."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import landau, pic
from tests.gpu_util import announce, host, to_gpu

pytestmark = pytest.mark.gpu


def test_standard_session_matches_oracle(gpu):
    e = W.landau_ensemble(11, n=2048, M=64)
    x0, v0 = e.x, e.v(0.4)
    steps, dt = 4, 0.05
    announce("standard session vs oracle")
    s = gpu.Session(to_gpu(x0), to_gpu(v0), e.L, e.M, dt, method=gpu.KDE_PIC_STANDARD, history=steps)
    try:
        x, v = x0.copy(), v0.copy()
        energies = []
        for _ in range(steps):
            x, v, rho, E = landau.field_step_standard(x, v, e.L, e.M, dt)
            energies.append(landau.field_energy(E, e.L))
            # one replay of the session's captured step, then an eager read
            s.step(1)
            gE = host(s.read(gpu.KDE_SESSION_E))
            assert np.max(np.abs(gE - E)) <= 1e-11 * np.abs(E).max()
        gx, gv = host(s.read(gpu.KDE_SESSION_X)), host(s.read(gpu.KDE_SESSION_V))
        assert np.max(np.abs(gx - x)) <= 1e-11 * e.L
        assert np.max(np.abs(gv - v)) <= 1e-11 * np.abs(v).max()
        gE = host(s.read(gpu.KDE_SESSION_E))
        assert np.max(np.abs(gE - E)) <= 1e-11 * np.abs(E).max()
        grho = host(s.read(gpu.KDE_SESSION_RHO))
        assert np.max(np.abs(grho - rho) / rho) <= 1e-11
        gW = host(s.read(gpu.KDE_SESSION_ENERGY))
        assert gW.shape == (steps,)
        assert np.max(np.abs(gW - energies) / np.asarray(energies)) <= 1e-11
        assert s.state()["step"] == steps
    finally:
        s.close()


@pytest.mark.parametrize("M", [2, 4, 512, 2048])
def test_standard_session_grid_sizes(gpu, M):
    """The session's field solve over the power-of-two grids it accepts,
    from two nodes to 2048 (several cells per thread of the solver's
    workgroup), against the oracle's DFT solve, after two steps; grid values
    normwise, since small grids and sparse cells hold zeros."""
    e = W.landau_ensemble(12, n=3000, M=M)
    x0, v0 = e.x, e.v(0.3)
    steps, dt = 2, 0.05
    announce("standard session grid size", M)
    s = gpu.Session(to_gpu(x0), to_gpu(v0), e.L, e.M, dt, method=gpu.KDE_PIC_STANDARD, history=steps)
    try:
        x, v = x0.copy(), v0.copy()
        for _ in range(steps):
            x, v, rho, E = landau.field_step_standard(x, v, e.L, e.M, dt)
        s.step(steps)
        gE = host(s.read(gpu.KDE_SESSION_E))
        scale = max(np.abs(E).max(), (e.L / M) * np.abs(1.0 - e.L * rho).max())  # M = 2: E is 0
        assert np.max(np.abs(gE - E)) <= 1e-11 * scale
        grho = host(s.read(gpu.KDE_SESSION_RHO))
        assert np.max(np.abs(grho - rho)) <= 1e-11 * np.abs(rho).max()
        gx, gv = host(s.read(gpu.KDE_SESSION_X)), host(s.read(gpu.KDE_SESSION_V))
        d = np.abs(gx - x)
        assert np.max(np.minimum(d, e.L - d)) <= 1e-11 * e.L
        assert np.max(np.abs(gv - v)) <= 1e-11 * np.abs(v).max()
    finally:
        s.close()


def test_kde_session_energy_history_matches_oracle(gpu):
    """The KDE session's recorded energies equal the oracle's field energy of
    the fields its steps compute (history shorter than the run: later steps
    are not recorded)."""
    from tests.test_gpu_serving import oracle_session
    L, M, n, dt = 4 * math.pi, 64, 2048, 0.1
    rng = W.rng_for(5, 78)
    x0 = W.cosine_positions(rng, n, L, 0.1, 0.5)
    v0 = W.maxwellian(rng, n, 1.0)
    kappas = W.log_kappas(1.0, 1e4, 16)
    announce("kde session energy")
    s = gpu.Session(to_gpu(x0), to_gpu(v0), L, M, dt, kappas, 1024, history=2)
    try:
        _, _, _, _, hist = oracle_session(x0, v0, L, M, dt, kappas, 1024, 3)
        s.step(3)
        gW = host(s.read(gpu.KDE_SESSION_ENERGY))
        assert gW.shape == (2,)
        ref = np.array([landau.field_energy(h["E"], L) for h in hist[:2]])
        assert np.max(np.abs(gW - ref) / ref) <= 1e-11
    finally:
        s.close()


@pytest.mark.parametrize("method", ["standard", "kde"])
def test_checkpoint_carries_the_history(gpu, method):
    e = W.landau_ensemble(12, n=4096, M=64)
    kw = dict(method=gpu.KDE_PIC_STANDARD) if method == "standard" else dict(kappas=W.log_kappas(1, 1e4, 8), n_cv=1024)
    announce("landau checkpoint", method)
    a = gpu.Session(to_gpu(e.x), to_gpu(e.v(0.3)), e.L, e.M, 0.05, history=12, **kw)
    b = gpu.Session(to_gpu(e.x), to_gpu(e.v(0.3)), e.L, e.M, 0.05, history=12, **kw)
    try:
        a.step(5)
        b.restore(a.save())
        a.step(4)
        b.step(4)
        assert np.array_equal(host(a.read(gpu.KDE_SESSION_ENERGY)), host(b.read(gpu.KDE_SESSION_ENERGY)))
        assert np.array_equal(host(a.read(gpu.KDE_SESSION_X)), host(b.read(gpu.KDE_SESSION_X)))
    finally:
        a.close()
        b.close()


def test_landau_run_one_ensemble_both_methods(gpu):
    """The paper's setting on one ensemble (2^15 particles, 256 nodes,
    dt = 0.01, 1500 steps, 0.02 cos x, v_th = 0.4). Standard PIC: the
    two-peak energy rate within 40 % of the theory's 2 Im(omega) (one
    ensemble is noisy; the ensemble statistics are the benchmark's). KDE:
    the kernel multiplies the mode's force by rho_1(kappa)^2 at deposit and
    gather (kappa* averaged over the span of the two peaks; the widths vary
    by a few percent around it), which damps the mode faster; with the
    wide kernel CV picks on this nearly uniform plasma the damping is
    strong, and the two-peak slope near t ~ 3-5 still carries the other
    roots of the initial-value response, so the rate is held to the bracket
    [1.4 x the theory with that response, 0.9 x the plain theory]. The
    library's and the oracle's extraction agree on each history."""
    e = W.landau_ensemble(0)
    rates = {}
    chunk = 50
    for name, kw in (("standard", dict(method=gpu.KDE_PIC_STANDARD)),
                     ("kde", dict(kappas=W.log_kappas(1.0, 1e4, 16), n_cv=e.x.shape[0]))):
        announce("landau run", name)
        s = gpu.Session(to_gpu(e.x), to_gpu(e.v(0.4)), e.L, e.M, e.dt, history=e.steps, **kw)
        kstars = []  # kappa* in force during steps [c chunk, (c + 1) chunk)
        try:
            for _ in range(e.steps // chunk):
                kstars.append(s.state()["kappa_star"])
                s.step(chunk)
            Wt = host(s.read(gpu.KDE_SESSION_ENERGY))
        finally:
            s.close()
        rate, peaks = gpu.kde_damping_rate(Wt, e.dt)
        assert peaks == tuple(landau.first_two_peaks(Wt))
        assert abs(rate - landau.damping_rate(Wt, e.dt)) <= 1e-14 * abs(rate)
        kstar = float(np.mean(kstars[peaks[0] // chunk: peaks[1] // chunk + 1]))
        plain = 2 * landau.landau_root(1.0, 0.4).imag
        if name == "standard":
            rates[name] = (rate, plain)
            assert abs(rate / plain - 1) < 0.4, (name, rate, plain)
        else:
            scaled = 2 * landau.landau_root(1.0, 0.4, response=landau.kernel_response(kstar)).imag
            rates[name] = (rate, plain, scaled, kstar)
            assert 1.4 * scaled < rate < 0.9 * plain, (name, rate, plain, scaled, kstar)
    print("rates", rates)
