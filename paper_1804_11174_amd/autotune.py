"""Autotuner for the CV pair kernel's launch shape.

Two knobs: the pass size (concentrations evaluated per pass over a tile
pair: 4, 8 or 16) and the group (concentrations one workgroup takes on,
a multiple of the pass size, or 0 for all of them; a smaller group splits
each tile pair over more workgroups, which shortens the critical path of
small sets). For each precision and particle count in a ladder it times
kde_cv_scan with every combination, keeps the fastest, and writes the
table to tune_gfx950.json beside this file; the Python binding installs
that table when it loads the library. Results do not depend on either
knob, only speed does.

Usage (on an MI355X): python -m paper_1804_11174_amd.autotune [--B 16]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CHUNKS = (4, 8, 16)
LADDER = (1024, 4096, 16384, 65536)


def shapes(B):
    """(chunk, group) combinations worth timing for B concentrations."""
    out = []
    for c in CHUNKS:
        if c > B and c != CHUNKS[0]:
            continue
        out.append((c, 0))
        for m in (1, 2, 4):
            if c * m < B:
                out.append((c, c * m))
    return out


def time_scan(kde, x, L, kappas, reps):
    import torch
    cv, sums, am = kde.cv_scan(x, L, kappas)          # warm-up
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        kde.cv_scan(x, L, kappas)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--B", type=int, default=16)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=os.path.join(HERE, "tune_gfx950.json"))
    args = ap.parse_args()
    import numpy as np
    import torch
    import paper_1804_11174_amd as kde
    import workloads as W

    kde.require_library()
    L = 4 * math.pi
    kappas = W.log_kappas(1.0, 1e4, args.B)
    table = {"arch": "gfx950", "B": args.B, "measured": {}}
    for name, dt, prec in (("f64", torch.float64, kde.KDE_F64), ("f32", torch.float32, kde.KDE_F32)):
        rows = []
        for n in LADDER:
            x = torch.from_numpy(W.cosine_positions(W.rng_for(9, n), n, L, 0.5, 0.5)).to(dt).cuda()
            times = {}
            for c, g in shapes(args.B):
                kde.kde_tune_set(prec, [1 << 62], [c], [g])
                times[(c, g)] = time_scan(kde, x, L, kappas, args.reps)
            best = min(times, key=times.get)
            rows.append({"n": n, "chunk": best[0], "group": best[1]})
            table["measured"][f"{name}/{n}"] = {f"{c}/{g}": t for (c, g), t in times.items()}
            print(name, n, {f"{c}/{g}": f"{t*1e3:.3f} ms" for (c, g), t in times.items()}, "->", best, flush=True)
        # bucket boundaries at the geometric midpoints of the ladder
        out_rows = []
        for k, r in enumerate(rows):
            n_max = int(math.sqrt(rows[k]["n"] * rows[k + 1]["n"])) if k + 1 < len(rows) else 1 << 62
            out_rows.append({"n_max": n_max, "chunk": r["chunk"], "group": r["group"]})
        table[name] = out_rows
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
