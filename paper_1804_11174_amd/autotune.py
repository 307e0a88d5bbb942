"""Autotuner for the CV pair kernel's launch shape.

Two knobs: the pass size (concentrations evaluated per pass over a tile
pair: 4, 8, or 16 in double) and the group (concentrations one workgroup takes on,
a multiple of the pass size, or 0 for all of them; a smaller group splits
each tile pair over more workgroups, which shortens the critical path of
small sets). For each precision and particle count in a ladder it times
kde_cv_scan with every combination at each concentration count of --B,
keeps the combination with the least sum over those counts of its time
relative to the fastest, and writes the
table to tune_gfx950.json beside this file (the Python binding installs it
when it loads the library) and to csrc/tune_gfx950.inc (the library's
built-in default, for callers of the C interface; rebuild after a run).
Results do not depend on either knob, only speed does.

Usage (on an MI355X): python -m paper_1804_11174_amd.autotune [--B 16,32]
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

CHUNKS = {"f64": (4, 8, 16), "f32": (4, 8)}
LADDER = (1024, 4096, 16384, 65536)


def shapes(B, chunks):
    """(chunk, group) combinations worth timing for B concentrations."""
    out = []
    for c in chunks:
        if c > B and c != chunks[0]:
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
    ap.add_argument("--B", default="16,32", help="concentration counts to tune for (comma-separated)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=os.path.join(HERE, "tune_gfx950.json"))
    ap.add_argument("--inc", default=os.path.join(HERE, "csrc", "tune_gfx950.inc"))
    args = ap.parse_args()
    import numpy as np
    import torch
    import paper_1804_11174_amd as kde
    import workloads as W

    kde.require_library()
    L = 4 * math.pi
    Bs = [int(b) for b in args.B.split(",")]
    table = {"arch": "gfx950", "B": Bs, "measured": {}}
    for name, dt, prec in (("f64", torch.float64, kde.KDE_F64), ("f32", torch.float32, kde.KDE_F32)):
        rows = []
        for n in LADDER:
            x = torch.from_numpy(W.cosine_positions(W.rng_for(9, n), n, L, 0.5, 0.5)).to(dt).cuda()
            score, common = {}, None
            for B in Bs:
                kappas = W.log_kappas(1.0, 1e4, B)
                times = {}
                for c, g in shapes(B, CHUNKS[name]):
                    kde.kde_tune_set(prec, [1 << 62], [c], [g])
                    times[(c, g)] = time_scan(kde, x, L, kappas, args.reps)
                fastest = min(times.values())
                for k, t in times.items():
                    score[k] = score.get(k, 0.0) + t / fastest
                common = set(times) if common is None else common & set(times)
                table["measured"][f"{name}/{n}/B{B}"] = {f"{c}/{g}": t for (c, g), t in times.items()}
                print(name, n, B, {f"{c}/{g}": f"{t*1e3:.3f} ms" for (c, g), t in times.items()}, flush=True)
            best = min(sorted(common), key=lambda k: score[k])  # shapes timed at every B
            rows.append({"n": n, "chunk": best[0], "group": best[1]})
            print(name, n, "->", best, flush=True)
        # bucket boundaries at the geometric midpoints of the ladder
        out_rows = []
        for k, r in enumerate(rows):
            n_max = int(math.sqrt(rows[k]["n"] * rows[k + 1]["n"])) if k + 1 < len(rows) else 1 << 62
            out_rows.append({"n_max": n_max, "chunk": r["chunk"], "group": r["group"]})
        table[name] = out_rows
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", args.out)
    write_inc(table, args.inc)
    print("wrote", args.inc)


def write_inc(table, path):
    """The table as the C initialisers the library builds in."""
    def rows(name):
        return ", ".join("{%s, {%d, %d}}" % ("INT64_MAX" if r["n_max"] >= 1 << 62 else str(r["n_max"]), r["chunk"],
                                             r["group"]) for r in table[name])
    with open(path, "w") as f:
        f.write("// Written by paper_1804_11174_amd/autotune.py from its %s run (B = %s): the\n"
                "// pair kernel's {n_max, {pass size, group}} by particle count, the last\n"
                "// entry covering every larger N.\n" % (table["arch"], ", ".join(str(b) for b in table["B"])))
        f.write("#define KDE_TUNE_F64 {%s}\n" % rows("f64"))
        f.write("#define KDE_TUNE_F32 {%s}\n" % rows("f32"))


if __name__ == "__main__":
    main()
