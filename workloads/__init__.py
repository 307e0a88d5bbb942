"""Seeded synthetic inputs for the KDE noise-reduction hot path.

This module only draws random inputs. It holds none of the method's
arithmetic: no kernel, no Bessel function, no density estimate. Both the
CPU oracle (through the tests) and the GPU path consume the arrays drawn
here, so neither side needs a random generator of its own.

Every draw uses numpy's PCG64 through ``numpy.random.default_rng`` seeded
with the triple ``[11174, cfg, idx]``:

* ``cfg`` names the workload (1..5 below), ``idx`` the set, session or
  request stream within it.
* Positions come from rejection sampling of the cosine-perturbed uniform
  density ``f(x) = (1 + alpha*cos(k*x)) / L`` on ``[0, L)``. This is the
  initial-condition shape of the paper's Langmuir and Landau runs (Sec. III.A
  and III.B: a uniform density plus a small cosine perturbation), with
  ``alpha`` and ``k`` chosen per workload.
* Velocities, where a workload needs them, are Maxwellian:
  ``v_th * standard_normal`` (Sec. III.B).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_ROOT = 11174


def rng_for(cfg: int, idx: int = 0) -> np.random.Generator:
    """The generator for workload ``cfg``, set/session/stream ``idx``."""
    return np.random.default_rng([SEED_ROOT, int(cfg), int(idx)])


def cosine_positions(rng: np.random.Generator, n: int, L: float, alpha: float,
                     k: float) -> np.ndarray:
    """Draw ``n`` positions on [0, L) from ``(1 + alpha*cos(k x)) / L``.

    Rejection sampling, in batches of ``2n`` proposals: a proposal x is kept
    when ``u*(1+alpha) < 1 + alpha*cos(k x)`` with u uniform on [0, 1).
    Accepted values keep their draw order; batches repeat until at least
    ``n`` are accepted, then the array is cut to ``n``.
    """
    if n < 0:
        raise ValueError("n must be >= 0")
    if not (0.0 <= alpha < 1.0):
        raise ValueError("alpha must lie in [0, 1)")
    out: List[np.ndarray] = []
    have = 0
    while have < n:
        x = L * rng.random(2 * n if n > 0 else 1)
        u = rng.random(x.shape[0])
        keep = x[u * (1.0 + alpha) < 1.0 + alpha * np.cos(k * x)]
        out.append(keep)
        have += keep.shape[0]
    if n == 0:
        return np.empty(0, dtype=np.float64)
    return np.concatenate(out)[:n].astype(np.float64, copy=False)


def maxwellian(rng: np.random.Generator, n: int, v_th: float) -> np.ndarray:
    """Velocities ``v_th * N(0, 1)``."""
    return v_th * rng.standard_normal(n)


def log_kappas(lo: float, hi: float, count: int) -> np.ndarray:
    """``count`` concentrations log-spaced over [lo, hi] (both ends kept)."""
    if count == 1:
        return np.array([float(lo)])
    b = np.arange(count, dtype=np.float64)
    return 10.0 ** (math.log10(lo) + b * (math.log10(hi) - math.log10(lo)) / (count - 1))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclass
class KdeProblem:
    """One particle set plus the scan and grid it is processed with."""
    name: str
    x: np.ndarray                 # positions on [0, L), float64 (or float32 form)
    L: float
    M: int
    kappas: np.ndarray            # candidate concentrations, ascending
    alpha_density: float          # perturbation amplitude the set was drawn with
    k_wave: float
    n_cv: int                     # particles the CV scan runs on (a prefix of x)
    adapt_alpha: float = 0.5      # Silverman sensitivity (Sec. II.C)
    v: Optional[np.ndarray] = None


def plain_small(seed_idx: int = 0) -> KdeProblem:
    """4096 particles, L = 4*pi, k = 0.5, alpha = 0.1, M = 64, 8 kappas in [1, 1e3]."""
    L = 4.0 * math.pi
    rng = rng_for(1, seed_idx)
    x = cosine_positions(rng, 4096, L, 0.1, 0.5)
    return KdeProblem("plain-small", x, L, 64, log_kappas(1.0, 1e3, 8), 0.1, 0.5, 4096)


def plain_paper_scale(seed_idx: int = 0, n: int = 1 << 20, n_cv: int = 1 << 16) -> KdeProblem:
    """Landau-shaped set: alpha = 0.5, L = 4*pi, M = 256; CV on the first 65,536
    particles over 32 kappas in [1, 1e4]; adaptation on all 1,048,576."""
    L = 4.0 * math.pi
    rng = rng_for(2, seed_idx)
    x = cosine_positions(rng, n, L, 0.5, 0.5)
    return KdeProblem("plain-paper-scale", x, L, 256, log_kappas(1.0, 1e4, 32), 0.5, 0.5,
                      min(n_cv, n))


def precision_small(seed_idx: int = 0) -> KdeProblem:
    """The 4096-particle set of ``plain_small`` with positions rounded to float32."""
    p = plain_small(seed_idx)
    p.name = "precision-small"
    p.x = p.x.astype(np.float32)
    return p


@dataclass
class BatchSet:
    index: int
    problem: KdeProblem


def batch_sets(count: int = 512, kappa_count: int = 16,
               indices: Optional[List[int]] = None) -> List[BatchSet]:
    """Independent sets: N log-uniform in [1e3, 1e5], alpha ~ U[0.01, 0.5],
    k in {0.5, 1, 2}, L = 2*pi/k, M in {64, 128, 256}; 16 kappas in [1, 1e4].

    Set ``s`` draws, from ``rng_for(4, s)`` and in this order: N, alpha, k, M,
    then its positions.
    """
    out = []
    ids = range(count) if indices is None else indices
    for s in ids:
        rng = rng_for(4, s)
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e5)))))
        alpha = float(rng.uniform(0.01, 0.5))
        k = float(rng.choice([0.5, 1.0, 2.0]))
        M = int(rng.choice([64, 128, 256]))
        L = 2.0 * math.pi / k
        x = cosine_positions(rng, n, L, alpha, k)
        out.append(BatchSet(s, KdeProblem(f"batch-{s}", x, L, M,
                                          log_kappas(1.0, 1e4, kappa_count),
                                          alpha, k, n)))
    return out


@dataclass
class SessionInit:
    index: int
    x: np.ndarray
    v: np.ndarray
    L: float
    M: int
    dt: float
    kappas: np.ndarray
    n_cv: int


def pic_session(index: int, n: int = 262144, M: int = 128, dt: float = 0.1,
                v_th: float = 1.0, alpha: float = 0.01, k: float = 0.5,
                L: float = 4.0 * math.pi, n_cv: int = 65536,
                kappa_count: int = 16) -> SessionInit:
    """A resident PIC session: cosine-perturbed positions (0.01*cos(0.5 x) on
    L = 4*pi), Maxwellian velocities with v_th = 1, M = 128, dt = 0.1.
    Positions are drawn first, velocities after, from ``rng_for(5, index)``."""
    rng = rng_for(5, index)
    x = cosine_positions(rng, n, L, alpha, k)
    v = maxwellian(rng, n, v_th)
    return SessionInit(index, x, v, L, M, dt, log_kappas(1.0, 1e4, kappa_count), min(n_cv, n))


@dataclass
class Request:
    arrival_s: float
    problem: KdeProblem


def request_stream(count: int, rate_per_s: float, n_lo: float = 1e3, n_hi: float = 1e6,
                   Ms=(64, 128, 256, 512), kappa_count: int = 16, n_cv: int = 65536,
                   stream_idx: int = 1000) -> List[Request]:
    """Poisson arrivals of KDE/CV solve requests (float32 form).

    From ``rng_for(5, stream_idx)`` each request draws its inter-arrival gap
    (exponential with the given rate), N (log-uniform in [n_lo, n_hi]), M,
    alpha ~ U[0.01, 0.5], then its positions (k = 0.5, L = 4*pi).
    """
    rng = rng_for(5, stream_idx)
    t = 0.0
    out = []
    L = 4.0 * math.pi
    for r in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        M = int(rng.choice(list(Ms)))
        alpha = float(rng.uniform(0.01, 0.5))
        x = cosine_positions(rng, n, L, alpha, 0.5).astype(np.float32)
        out.append(Request(t, KdeProblem(f"req-{r}", x, L, M, log_kappas(1.0, 1e4, kappa_count),
                                         alpha, 0.5, min(n_cv, n))))
    return out


def vonmises_positions(rng: np.random.Generator, n: int, L: float, mu: float,
                       kappa_f: float) -> np.ndarray:
    """Positions whose angle 2*pi*x/L follows a von Mises law VM(mu, kappa_f)
    (numpy's own sampler), mapped to [0, L)."""
    th = rng.vonmises(mu, kappa_f, n)
    x = (th % (2.0 * math.pi)) * (L / (2.0 * math.pi))
    x[x >= L] = 0.0
    return x


@dataclass
class LandauEnsemble:
    """One ensemble of the Landau-damping workload (Sec. III.B): positions
    from ``(1 + amp cos(k x)) / L`` on ``L = 2 pi / k`` and unit-normal
    velocity draws ``z``; a run at thermal velocity v_th uses ``v_th * z``,
    so every thermal velocity and both methods share the same random
    numbers (common random numbers)."""
    index: int
    x: np.ndarray
    z: np.ndarray
    L: float
    M: int
    dt: float
    steps: int

    def v(self, v_th: float) -> np.ndarray:
        return v_th * self.z


def landau_ensemble(index: int, n: int = 1 << 15, M: int = 256, dt: float = 0.01, steps: int = 1500,
                    amp: float = 0.02, k: float = 1.0) -> LandauEnsemble:
    """Ensemble ``index`` of the Landau workload: 2^15 particles, 256 nodes,
    dt = 0.01, 1500 steps, density perturbation 0.02 cos(1.0 x) (Sec. III.B).
    Positions first, then the velocity draws, from ``rng_for(6, index)``."""
    L = 2.0 * math.pi / k
    rng = rng_for(6, index)
    x = cosine_positions(rng, n, L, amp, k)
    z = rng.standard_normal(n)
    return LandauEnsemble(index, x, z, L, M, dt, steps)
