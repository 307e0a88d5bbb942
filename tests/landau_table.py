"""Landau damping table (Sec. III.B) from a ``bench.py --form landau`` JSON line.

Test infrastructure, not collected by pytest: it sets the measured mean
energy rates of standard PIC and KDE beside the theory, 2 Im(omega) of the
least-damped root of the Maxwellian dispersion relation at k = 1, and for
KDE also the root with the kernel's response rho_1(kappa*)^2 at the mean
kappa* of the runs (both from the oracle), with the t statistic of each
mean's error against the plain theory.

    python bench.py --form landau --json-out landau.json
    python tests/landau_table.py landau.json
"""
from __future__ import annotations

import json
import math
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import landau as olandau  # noqa: E402


def cell(entry, theory):
    m, sd, n = entry["mean_rate"], entry["sd"], entry["runs_with_two_peaks"]
    if m is None:
        return "n/a"
    t = (m - theory) / (sd / math.sqrt(n)) if n > 1 and sd > 0 else float("nan")
    return f"{m:.3f} (sd {sd:.3f}, t {t:.1f})"


def table(line):
    rows = ["| v_th | theory 2 Im ω | standard PIC | KDE | KDE κ* | theory with ρ_1(κ*)² |",
            "|---|---|---|---|---|---|"]
    for r in line["damping"]:
        vth = r["v_th"]
        theory = 2 * olandau.landau_root(1.0, vth).imag
        kk = r["kde"]["mean_kappa_star"]
        resp = 2 * olandau.landau_root(1.0, vth, response=olandau.kernel_response(kk)).imag
        rows.append(f"| {vth:.2f} | {theory:.4f} | {cell(r['standard'], theory)} | {cell(r['kde'], theory)} "
                    f"| {kk:.1f} | {resp:.3f} |")
    return "\n".join(rows)


if __name__ == "__main__":
    with open(sys.argv[1]) as f:
        print(table(json.loads(f.readline())))
