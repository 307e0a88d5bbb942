"""Pins of the Landau-damping oracle (oracle/landau.py), CPU only.

The dispersion root is checked against the widely tabulated values for a
Maxwellian plasma and against the weak-damping asymptote; the two-peak rate
against a sampled damped oscillation whose answer is exact; the field energy
against a closed form; the standard-PIC step against conservation laws that
hold for any shared deposit/gather shape and against cold-plasma physics."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import landau, triangle


@pytest.mark.parametrize("klam,wr,wi", [(0.3, 1.1598, -0.0126), (0.4, 1.2850, -0.0661),
                                        (0.5, 1.4156, -0.1533), (1.0, 2.0459, -0.8513)])
def test_landau_root_tabulated(klam, wr, wi):
    w = landau.landau_root(1.0, klam)
    assert abs(w.real - wr) < 6e-4 and abs(w.imag - wi) < 6e-4
    assert abs(landau.dispersion(w, 1.0, klam)) < 1e-12
    # the same root in other units: only k v_th matters
    w2 = landau.landau_root(0.5, 2 * klam)
    assert abs(w2 - w) < 1e-12


@pytest.mark.parametrize("s", [0.9, 0.65, 0.4])
def test_scaled_response_root(s):
    """With the susceptibility scaled by s the root solves the scaled
    relation, reduces to the plain one at s = 1, and in the cold limit
    (k v_th -> 0) the frequency tends to sqrt(s): the plasma frequency of
    the weakened force."""
    w = landau.landau_root(1.0, 0.4, response=s)
    assert abs(landau.dispersion(w, 1.0, 0.4, response=s)) < 1e-12
    assert w.imag < landau.landau_root(1.0, 0.4).imag  # a weaker force damps faster here
    cold = landau.landau_root(1.0, 0.05, response=s)
    assert abs(cold.real / math.sqrt(s) - 1) < 0.02 and abs(cold.imag) < 1e-6
    assert landau.landau_root(1.0, 0.4, response=1.0) == landau.landau_root(1.0, 0.4)


def test_kernel_response_limits():
    assert landau.kernel_response(0.0) == 0.0
    assert abs(landau.kernel_response(1e4) - (1 - 0.5 / 1e4) ** 2) < 1e-8


def test_landau_root_weak_damping_asymptote():
    kl = 0.2
    w = landau.landau_root(1.0, kl)
    asym = -math.sqrt(math.pi / 8) / kl ** 3 * math.exp(-1 / (2 * kl * kl) - 1.5)
    assert 0.8 < w.imag / asym < 1.2


@pytest.mark.parametrize("K,phase", [(157, 0.0), (240, 0.4)])
def test_two_peak_rate_of_a_sampled_damped_oscillation(K, phase):
    """W(t) = exp(2 g t) cos^2(w t + phase) with pi / w = K dt: the samples
    repeat every K steps scaled by exp(2 g K dt), so the two-peak slope is
    2 g to rounding."""
    dt, g = 0.01, -0.0661
    w = math.pi / (K * dt)
    t = np.arange(1500) * dt
    Wt = np.exp(2 * g * t) * np.cos(w * t + phase) ** 2
    p = landau.first_two_peaks(Wt)
    assert p[1] - p[0] == K
    assert abs(landau.damping_rate(Wt, dt) - 2 * g) < 1e-12


def test_two_peak_rate_needs_two_peaks():
    assert math.isnan(landau.damping_rate(np.exp(-np.arange(50.0)), 0.1))


def test_field_energy_single_mode():
    L, M, A = 2 * math.pi, 64, 0.3
    E = A * np.sin(2 * math.pi * 3 * np.arange(M) / M)
    assert abs(landau.field_energy(E, L) - A * A * L / 4) < 1e-15


def test_standard_step_conserves_charge_and_momentum():
    """Linear weighting is a partition of unity (grid mass 1 exactly), and
    with the same shape for deposit and gather the centred field exerts no
    net force on the particles (sum_i E_i = N dx sum_g E_g rho_g = 0)."""
    e = W.landau_ensemble(3, n=3000, M=64)
    x, v = e.x, e.v(0.4)
    for _ in range(3):
        x_new, v_new, rho, E = landau.field_step_standard(x, v, e.L, e.M, 0.05)
        assert abs(rho.sum() * e.L / e.M - 1.0) < 1e-13
        assert abs(v_new.sum() - v.sum()) < 1e-12 * len(v)
        x, v = x_new, v_new


def test_standard_cold_plasma_oscillates_undamped():
    """A cold plasma (v = 0) with a small cosine perturbation oscillates at
    the plasma frequency: the field energy peaks every pi / omega_p and
    does not decay."""
    e = W.landau_ensemble(4, n=4096, M=64)
    x, v = e.x, np.zeros_like(e.x)
    dt, Wt = 0.02, []
    for _ in range(400):
        x, v, rho, E = landau.field_step_standard(x, v, e.L, e.M, dt)
        Wt.append(landau.field_energy(E, e.L))
    p = landau.first_two_peaks(Wt)
    assert abs((p[1] - p[0]) * dt - math.pi) < 0.1
    assert abs(landau.damping_rate(Wt, dt)) < 0.02


def test_standard_deposit_is_linear_weighting():
    """At h = dx the triangle is linear ('cloud-in-cell') weighting: each
    particle puts 1 - t and t on its two nodes (t its offset in cells)."""
    L, M = 2 * math.pi, 32
    rng = np.random.default_rng(48)
    x = L * rng.random(50)
    dx = L / M
    j = np.floor(x / dx).astype(int)
    t = x / dx - j
    ref = np.zeros(M)
    np.add.at(ref, j % M, 1 - t)
    np.add.at(ref, (j + 1) % M, t)
    assert np.allclose(triangle.deposit(x, L, M, h=dx), ref / (len(x) * dx), rtol=1e-12, atol=1e-14)
