"""Write bench_reference.json: the oracle's results for the inputs bench.py
times, so that bench.py can state the error of every timed result without
calling the oracle itself.

Runs the FP64 oracle only (oracle/), on the seeded inputs of workloads/:

* precision_small -- the 4096-particle plain-small set (L = 4 pi, M = 64,
  8 concentrations in [1, 1e3]): the CV objective, its pair sums and first
  minimum by direct pair sums (Sec. II.B, Eq. cv_def), and the grid density
  at every concentration (Eq. kde), on the float32-rounded positions (the
  precision form's input) and on the float64 positions.
* paper_scale -- the 2^20-particle set (CV on the first 65,536, 32
  concentrations in [1, 1e4], M = 256), for float64 and float32-rounded
  positions: the CV curve (through the oracle's Fourier-moment route, which
  the CPU tests pin to the direct sums), its first minimum kappa*, the pilot
  density at kappa*, the adaptive widths (Sec. II.C), the adaptive density,
  and the widths and the gathered adaptive density at every 4096th particle.

Usage: python tests/golden/make_bench_references.py  (about a minute).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cv as ocv, density as od  # noqa: E402

SAMPLE_EVERY = 4096


def small(x, p):
    cv, S1, S2 = ocv.cv_curve(x, p.L, p.kappas)
    grids = [od.deposit(x, p.L, p.M, kappa=float(k)).tolist() for k in p.kappas]
    return {"cv": cv.tolist(), "S1": S1.tolist(), "S2": S2.tolist(), "argmin": ocv.cv_argmin(cv), "grids": grids}


def paper(x, p):
    cv, _, _ = ocv.cv_curve_fourier(x[:p.n_cv], p.L, p.kappas)
    b = ocv.cv_argmin(cv)
    kstar = float(p.kappas[b])
    pilot = od.deposit(x, p.L, p.M, kappa=kstar)
    k_i, log_g, _ = od.adapt_widths(x, p.L, pilot, kstar, 0.5)
    rho = od.deposit(x, p.L, p.M, kappa_i=k_i)
    idx = np.arange(0, x.shape[0], SAMPLE_EVERY)
    G = od.gather(x[idx], p.L, rho, kappa_i=k_i[idx])
    return {"cv": cv.tolist(), "argmin": b, "kappa_star": kstar, "pilot": pilot.tolist(), "log_geomean": float(log_g),
            "rho": rho.tolist(), "sample_every": SAMPLE_EVERY, "kappa_i": k_i[idx].tolist(), "gather": G.tolist()}


def main():
    out = {"generator": "tests/golden/make_bench_references.py (oracle only)"}
    p = W.plain_small()
    out["precision_small"] = {"f32_positions": small(p.x.astype(np.float32).astype(np.float64), p),
                              "f64_positions": small(p.x, p)}
    q = W.plain_paper_scale()
    out["paper_scale"] = {"f64": paper(q.x, q), "f32": paper(q.x.astype(np.float32).astype(np.float64), q)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bench_reference.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
