"""Benchmark of the KDE hot path on one MI355X.

One step is one pass of the whole path over the paper-scale workload
(1,048,576 particles drawn from (1 + 0.5 cos(0.5 x)) / L on L = 4 pi,
M = 256 grid nodes):

  1. CV scan on the first 65,536 particles over 32 concentrations
     log-spaced in [1, 1e4] (pack + sort, O(N^2) pair sums, finalize, argmin);
  2. pilot deposit of all particles at the chosen kappa*;
  3. particle-wise widths from the pilot (Silverman, alpha = 0.5);
  4. adaptive deposit with those widths;
  5. gather of the adaptive density back to all particles.

Inputs are resident in HBM before the timed region; workspaces and outputs
are allocated once, outside it. The only host round trip inside a step is
reading kappa* (4 bytes) after the scan, which the following calls take as
an argument.

Prints one JSON line. ``value`` is the whole step's throughput in CV
pair-evaluations per second: B * n_cv (n_cv - 1) / 2 per step over the step
time. Per-phase kernel times come from the library's HIP-event timing of
its dominant kernels, on the stream they are launched on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CV pair-evals/s, particles/s at 1e-6 rel err; p50/p99 solve latency vs plain"

# MI355X published vector peaks: FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s,
# counting a fused multiply-add as two flops. In lane-operations (an FMA,
# a multiply, an add, a min or a transcendental each count one) that is
# 39.3e12/s in double (256 CUs x 64 lanes x 2.4 GHz) and 78.6e12/s in float
# (twice the lanes per clock, reached with packed FP32 instructions, which
# the library's kernels are compiled not to emit). HBM3E 8 TB/s.
PEAK_LANE_OPS = {"f64": 78.6e12 / 2, "f32": 157.3e12 / 2}
PEAK_HBM = 8.0e12

# Algorithmic lane-operations of the CV pair sums, counted from the method's
# formulas in FMA-issue slots: a multiply, an add or an FMA counts one; the
# hardware float exp2 counts four (it issues at a quarter of the float FMA
# rate, measured by `--form peak`); an accumulated sum counts one add per
# term (compensation of the float sums is overhead); per-pair geometry and
# per-concentration constants are not counted.
# Terms of the other concentrations (X0 = 16 in double, 8 in float, the
# split point of the Bessel fits), priced at the large-argument branch:
#   f64: K term: exponent product 1 + exponential 14 (Tang's table method:
#        reduction 4, table index 3, polynomial and combination 5, scaling
#        1, bound 1) = 15; Kbar term: exponent product 1 + exponential 14 +
#        Bessel argument 1 + degree-11 polynomial 11 + two products = 29;
#        two accumulations 2. Total 46 per evaluated term.
#   f32: K term: product 1 + exp2 4 = 5; Kbar term: product 1 + exp2 4 +
#        argument 1 + degree-5 polynomial 5 + two products = 13; two
#        accumulations 2. Total 20 per evaluated term.
# Concentrations with 2 kappa below X0 (1.01 X0 in double, where the
# small-argument fit holds its accuracy to there) take the small-argument
# branch for every pair, and none of their terms is skipped:
#   f64: K term 15 and its accumulation 1 = 16 per term; the Kbar terms of
#        all these concentrations together 41 per pair: their terms are one
#        degree-20 polynomial of the pair's c^2 with per-concentration
#        scales, so the pair sums need only the power sums of c^2 (twenty
#        multiplies forming c^2 ... c^40 and twenty-one adds); the
#        polynomials are applied to the power sums once per thread and
#        tile pair, not per pair. The same holds, tile pair by tile pair,
#        for larger concentrations on two tiles far enough apart that every
#        pair's 2 kappa c stays below 1.01 X0 (power_sum_route counts them
#        as the kernel decides them; the rest at 46 per evaluated term).
#   f32: K term 5 + Kbar term (argument 1 + degree-10 polynomial 10 +
#        product 1) 12 + two accumulations 2 = 19 per term.
OPS_PER_TERM = {"f64": 46, "f32": 20}
BESSEL_X0 = {"f64": 16.0, "f32": 8.0}
PURE_REACH = {"f64": 1.01, "f32": 1.0}
PURE_TERM_OPS = {"f64": 16, "f32": 19}
PURE_PAIR_OPS = {"f64": 41, "f32": 0}
SKIP_EXPONENT = 70.0

# The planning cost model's ideal pair-evaluation rates, against which the
# algorithmic pair-evaluation rate B n (n - 1) / 2 / t is also stated: about
# 70 FP64 operations per pair-evaluation (5e11/s at the FP64 vector peak);
# in float 4 transcendentals at a quarter of the FMA rate plus about 22
# other operations (1.0e12/s). The model counts every (pair, kappa) term,
# while the kernel skips terms below e^-70 of their sum's scale, so a kernel
# can exceed it; `frac` itself is taken on the evaluated terms.
PLANNING_IDEAL_PAIR_EVALS = {"f64": 5.0e11, "f32": 1.0e12}

# Issue counters of the pair kernel on the paper-scale scan (rocprofv3 --pmc
# SQ_INSTS_VALU SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_SALU SQ_WAVES SQ_BUSY_CYCLES
# GRBM_GUI_ACTIVE, one dispatch): VALU lane-instructions and transcendentals
# per evaluated term, the engine clock during that dispatch (GRBM_GUI_ACTIVE
# over its duration, per XCD), and the issue fraction in that same run:
# FMA-issue slots used (each VALU instruction one, a float transcendental
# four) over those available (256 CUs x 4 SIMDs at one double instruction
# per four clocks, or one float instruction per two). Valid only for the
# kernel sources they were taken on (PAIR_KERNEL_SOURCES' digest); where a
# change to these files leaves cv_pairs_kernel's machine code the same
# (other kernels of cv.hip, comments), the digest is moved on after
# comparing that code, and the counters are kept.
PAIR_COUNTERS = {"digest": "9257d2c5f950ec86",
                 "source": "profiles/cv_pairs_valu_counters_paper_scale.md",
                 "f64": {"valu_lane_instr_per_term": 38.51, "trans_per_term": 0.0005, "engine_clock_ghz": 2.213,
                         "issue_frac": 0.940},
                 "f32": {"valu_lane_instr_per_term": 23.60, "trans_per_term": 1.842, "engine_clock_ghz": 2.135,
                         "issue_frac": 0.882}}

# HBM bytes per launch of the pair kernel on the paper-scale scan, from the
# FETCH_SIZE and WRITE_SIZE counters (rocprofv3 --pmc, one counter per run)
# scaled by a 1 GiB copy's readings (bytes read = 2.0 x FETCH_SIZE, bytes
# written = 1.0 x WRITE_SIZE); valid only for the kernel sources they were
# taken on, identified by PAIR_KERNEL_SOURCES' digest.
PAIR_KERNEL_SOURCES = ("cv.hip", "dev_cv.hpp", "dev_sum.hpp", "device_bessel.hpp", "bessel_coeffs.inc",
                       "dev_layout.hpp", "kde_internal.hpp")
PAIR_TRAFFIC = {"digest": "9257d2c5f950ec86",
                "f64": {"fetch_kib": 8690.375, "write_kib": 191780.125},
                "f32": {"fetch_kib": 1711.5, "write_kib": 22528.0}}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def pair_kernel_traffic(prec):
    """HBM bytes per pair-kernel launch, or None once its sources differ
    from those the counters were taken on."""
    if pair_kernel_digest() != PAIR_TRAFFIC["digest"]:
        return None
    c = PAIR_TRAFFIC[prec]
    return (FETCH_SCALE * c["fetch_kib"] + WRITE_SCALE * c["write_kib"]) * 1024.0


def count_evaluated_terms(x, L, kappas):
    """Exact number of (pair, kappa) terms whose convolution exponent
    -2 kappa (1 - cos(pi d / L)) is at least -70 (the terms the pair kernel
    must evaluate), from the sorted positions by binary search."""
    xs = np.sort(np.asarray(x, dtype=np.float64) % L)
    n = xs.shape[0]
    ext = np.concatenate([xs, xs + L])
    total = 0
    for k in kappas:
        lim = SKIP_EXPONENT / (2.0 * k)
        if lim >= 1.0:
            total += n * (n - 1) // 2
            continue
        dmax = (L / math.pi) * math.acos(1.0 - lim)       # circular distance bound
        dmax = min(dmax, L / 2)
        hi = np.searchsorted(ext, xs + dmax, side="right")
        cnt = np.minimum(hi - np.arange(n) - 1, n - 1)     # partners ahead within dmax
        # an unordered pair within dmax is counted once, from the particle
        # whose forward arc to the other is the shorter one (dmax <= L/2)
        total += int(cnt.sum())
    return total



CV_TILE = 256


def power_sum_route(x, L, kappas, detail=None):
    """The double pair kernel's power-sum route over the tile pairs of the
    cell-sorted positions, as the kernel decides it: per tile pair the
    concentrations with 2 kappa < 1.01 X0, and, on two tiles at least a gap
    g apart (the kernel's cell bound), also those with 2 kappa (C + 1e-12)
    < 1.01 X0, C = 1 - x^2/2 + x^4/24 >= cos(x), x = pi g, up to the first
    concentration the tile test prunes.
    Returns (terms on the route, those of them at or above the skip bound,
    pairs of the tile pairs that form power sums); a list passed as
    `detail` receives (indices of tile I, indices of tile J, concentrations
    on the route) per tile pair that has any."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    k2 = 2.0 * np.asarray(kappas, dtype=np.float64)
    reach = PURE_REACH["f64"] * BESSEL_X0["f64"]
    cells = min(max(n // 32, 1), 8192)
    w = x - L * np.floor(x / L)
    w[w >= L] = 0.0
    cell = np.clip((w * cells / L).astype(np.int64), 0, cells - 1)
    order = np.lexsort((np.arange(n), cell))
    f = w[order] * (1.0 / L)
    ntiles = (n + CV_TILE - 1) // CV_TILE
    first = f[np.arange(ntiles) * CV_TILE]
    last = f[np.minimum(np.arange(ntiles) * CV_TILE + CV_TILE, n) - 1]
    lo = (np.floor(first * cells) - 2.0) / cells
    hi = (np.floor(np.where(last < first, 1.0, last) * cells) + 3.0) / cells
    npure = int(np.count_nonzero(k2 < reach))
    terms = evaluated = wpairs = 0
    for I in range(ntiles):
        ni = min(CV_TILE, n - I * CV_TILE)
        for J in range(I, ntiles):
            nj = min(CV_TILE, n - J * CV_TILE)
            pe, tp = npure, (ni * (ni - 1) // 2 if I == J else ni * nj)
            gap = -1.0 if I == J else min(lo[J] - hi[I], 1.0 + lo[I] - hi[J])
            if gap > 0.0:
                y = 0.5 * math.pi * gap
                qmin = 2.0 * (y * (1.0 - y * y / 6.0)) ** 2
                pruned = k2 * qmin > SKIP_EXPONENT * (1.0 + 1e-6)
                be = int(np.argmax(pruned)) if pruned.any() else len(k2)
                x2 = (math.pi * gap) ** 2
                cmax = 1.0 + x2 * (-0.5 + x2 / 24.0) + 1e-12  # the kernel's bound on cos(pi gap)
                while pe < be and k2[pe] * cmax < reach:
                    pe += 1
                pe = min(pe, be)
            if pe == 0:
                continue
            if detail is not None:
                detail.append((order[I * CV_TILE:I * CV_TILE + ni], order[J * CV_TILE:J * CV_TILE + nj], pe))
            terms += pe * tp
            wpairs += tp
            for b in range(pe):
                if k2[b] <= SKIP_EXPONENT:
                    evaluated += tp
                else:
                    fi = f[I * CV_TILE:I * CV_TILE + ni]
                    fj = f[J * CV_TILE:J * CV_TILE + nj]
                    d = np.abs(fi[:, None] - fj[None, :])
                    d = np.minimum(d, 1.0 - d)
                    ok = -k2[b] * (1.0 - np.cos(math.pi * d)) >= -SKIP_EXPONENT
                    if I == J:
                        ok = np.triu(ok, 1)
                    evaluated += int(np.count_nonzero(ok))
    return terms, evaluated, wpairs


def pair_kernel_ops(x, L, kappas, prec):
    """Algorithmic lane-operations of one CV pair-sum launch over positions x
    on the basis above; returns (ops, evaluated terms, terms summed through
    power sums in double / small-argument terms in float)."""
    n = int(np.asarray(x).shape[0])
    pairs = n * (n - 1) // 2
    evaluated = count_evaluated_terms(x, L, kappas)
    if prec == "f64":
        route, route_evaluated, wpairs = power_sum_route(x, L, kappas)
        ops = ((evaluated - route_evaluated) * OPS_PER_TERM[prec] + route * PURE_TERM_OPS[prec]
               + wpairs * PURE_PAIR_OPS[prec])
        return ops, evaluated, route
    npure = sum(1 for k in kappas if 2.0 * float(k) < PURE_REACH[prec] * BESSEL_X0[prec])
    pure = npure * pairs
    ops = (evaluated - pure) * OPS_PER_TERM[prec] + pure * PURE_TERM_OPS[prec]
    return ops, evaluated, pure

# Secondary kernels of the plain pipeline, from the library's per-launch
# event averages. Algorithmic lane-operations per (particle, node)
# evaluation of the deposit and gather, on the pair kernel's basis (FMA-issue
# slots, a float exp2 as four, one add per accumulated sum):
#   f64: node sine from the node table 2, square 1, exponent product 1,
#        clamp 1, table exponential 14, weight or field product 1,
#        accumulation 1 = 21;
#   f32: node index wrap 2, node sine 2, square 1, exponent product 1,
#        exp2 4, weight or field product 1, accumulation 1 = 12.
# Algorithmic HBM bytes per launch: deposit reads the positions (and the
# widths in the adaptive one; the pipeline runs one of each, so 1.5 arrays
# on average) and writes its chunk grids (chunks x M doubles); gather reads
# positions and widths and writes the gathered values; adapt reads the
# positions twice (log sums, then widths) and writes the widths.
NODE_OPS = {"f64": 21, "f32": 12}
HBM_PEAK = 8e12


def secondary_rooflines(prec, n, M, kern):
    el = 8 if prec == "f64" else 4
    chunk = min(512, max(64, -(-n // 2048)))
    chunks = -(-n // chunk)
    out = {}
    for name, bytes_ in (("deposit", 1.5 * el * n + chunks * M * 8), ("gather", 3 * el * n + M * 8)):
        ms = kern[name]["avg_ms"]
        if not ms:
            continue
        alu = n * M * NODE_OPS[prec] / (ms * 1e-3)
        bw = bytes_ / (ms * 1e-3)
        out[name] = {"bound": "alu", "ops_per_eval": NODE_OPS[prec], "evals_per_launch": n * M,
                     "alu_frac": alu / PEAK_LANE_OPS[prec], "hbm_gbs": bw / 1e9, "hbm_frac": bw / HBM_PEAK,
                     "avg_ms": ms}
    ms = kern["adapt"]["avg_ms"]
    if ms:
        bw = 3 * el * n / (ms * 1e-3)
        out["adapt"] = {"bound": "hbm", "bytes_per_launch": 3 * el * n, "hbm_gbs": bw / 1e9, "hbm_frac": bw / HBM_PEAK,
                        "avg_ms": ms}
    return out


# Issue-rate probes: per instruction kind, the iteration count of one
# launch (about 10-40 ms on MI355X) and the published peak it is read
# against (lane-operations per second, an FMA counting as one; the
# published vector peaks: FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s of which
# half needs packed instructions; no published figure for exp2 or add).
PROBES = (("fma_f64", 0, 131072, 78.6e12 / 2), ("fma_f32", 1, 262144, 157.3e12 / 2),
          ("exp_f32", 2, 32768, None), ("add_f64", 3, 131072, 78.6e12 / 2))


def bench_peak(args, kde, torch, dev):
    """Sustained lane-operation rates of single instruction kinds (8 waves
    per SIMD, 8 independent chains per lane), timed with the library's HIP
    events over `steps` launches after one warm-up."""
    blocks = 2048
    out = torch.empty(blocks * 256, dtype=torch.float64, device=dev)
    rates, ratio, ms = {}, {}, {}
    for name, kind, iters, peak in PROBES:
        kde.kde_probe_peak(kind, blocks, 4096, out)
        torch.cuda.synchronize()
        kde.kde_timing_reset()
        kde.kde_timing_enable(True)
        for _ in range(args.steps):
            kde.kde_probe_peak(kind, blocks, iters, out)
        torch.cuda.synchronize()
        kde.kde_timing_enable(False)
        tot, cnt = kde.kde_timing_read(kde.KDE_KERNEL_PROBE)
        ops = blocks * 256 * 8 * iters * cnt
        rates[name] = ops / (tot * 1e-3)
        ms[name] = tot / cnt
        ratio[name] = rates[name] / peak if peak else None
    line = {"metric": "sustained lane-operations/s per instruction kind", "value": rates["fma_f64"],
            "unit": "lane-ops/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": True,
            "dtype": "f64", "data": "synthetic", "vs_baseline": None,
            "config": {"workload": "issue-rate probes: 2048 workgroups x 256 threads, 8 dependency chains per "
                                   "thread, one instruction kind per launch"},
            "rates": rates, "fraction_of_published_peak": ratio, "ms_per_launch": ms}
    out_s = json.dumps(line)
    print(out_s, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out_s + "\n")


def pair_kernel_digest():
    """Digest of PAIR_KERNEL_SOURCES without their comments and blank lines
    (a line's text from "//" on is dropped; the sources hold no "//" inside
    string literals), so that only a change of code moves it."""
    h = hashlib.sha256()
    for f in PAIR_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1804_11174_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def pair_kernel_issue(prec):
    """The pair kernel's issue counters, or None once its sources differ
    from those the counters were taken on."""
    if PAIR_COUNTERS.get("digest") != pair_kernel_digest() or prec not in PAIR_COUNTERS:
        return None
    return dict(PAIR_COUNTERS[prec], source=PAIR_COUNTERS["source"])


REFERENCE_FILE = os.path.join(ROOT, "tests", "golden", "bench_reference.json")


def _rel(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.abs(ref)))


def plain_errors(prec, cv, kstar, pilot, rho, k_i, G):
    """Errors of the timed step's results against the FP64 oracle's, stored
    by tests/golden/make_bench_references.py for the same positions (float32
    runs: the float32-rounded positions): the CV curve (relative, and
    relative to its range), the chosen kappa*, and when it agrees the pilot
    and adaptive densities (relative per node), the widths (relative) and the
    gathered density (normwise) at every 4096th particle."""
    with open(REFERENCE_FILE) as f:
        ref = json.load(f)["paper_scale"][prec]
    rc = np.asarray(ref["cv"])
    out = {"reference": "FP64 oracle, tests/golden/bench_reference.json",
           "cv_rel": _rel(cv, rc), "cv_over_range": float(np.max(np.abs(np.asarray(cv) - rc)) / np.ptp(rc)),
           "kappa_star_equal": bool(kstar == ref["kappa_star"])}
    if out["kappa_star_equal"]:
        e = ref["sample_every"]
        rg = np.asarray(ref["gather"])
        out.update({"pilot_rel": _rel(pilot, ref["pilot"]), "rho_rel": _rel(rho, ref["rho"]),
                    "kappa_i_rel_sampled": _rel(np.asarray(k_i)[::e], ref["kappa_i"]),
                    "gather_normwise_sampled": float(np.max(np.abs(np.asarray(G)[::e] - rg)) / np.max(np.abs(rg)))})
    return out


def host_cores():
    """The host the oracle ran on: logical CPUs, those this process may use,
    and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def _pair_rows_task(args):
    """One row block of the oracle's direct pair sums (a worker of the
    all-cores baseline)."""
    from oracle import cv as ocv
    x, L, kappas, i0, i1 = args
    return ocv.pair_sums_rows(x, L, kappas, i0, i1)


def _oracle_pair_sums(pool, x, L, kappas, block=256):
    """The oracle's direct pair sums over row blocks of ``block`` rows,
    spread over the pool's workers and added in row order (the order of the
    oracle's own loop, so the result is the one-worker result bit for bit)."""
    n = x.shape[0]
    tasks = [(x, L, kappas, i0, min(n, i0 + block)) for i0 in range(0, n, block)]
    parts = pool.map_async(_pair_rows_task, tasks, chunksize=1).get(timeout=300)
    S1 = np.zeros(len(kappas))
    S2 = np.zeros(len(kappas))
    for s1, s2 in parts:
        S1 += s1
        S2 += s2
    return S1, S2


def cpu_baseline(x, L, kappas, budget_s=10.0):
    """The oracle's direct FP64 pair sums of the same scan, timed on a
    bounded sample (the first m particles, m chosen for about budget_s
    seconds of wall time): once on one worker and once on every core this
    process may use (len(sched_getaffinity)), row blocks spread over a pool
    of spawned worker processes and reduced in row order. Pair-evaluations
    per second = B m (m - 1) / 2 over the wall time of the sums."""
    import multiprocessing as mp
    from oracle import cv as ocv
    x = np.asarray(x, dtype=np.float64)
    kappas = np.asarray(kappas, dtype=np.float64)
    B = len(kappas)
    m0 = 512
    t0 = time.perf_counter()
    ocv.pair_sums(x[:m0], L, kappas)
    rate0 = B * m0 * (m0 - 1) / 2 / max(time.perf_counter() - t0, 1e-9)

    def size_for(rate):
        return max(m0, min(int(math.sqrt(2 * budget_s * rate / B)), x.shape[0]))

    m1 = size_for(rate0)
    t0 = time.perf_counter()
    ocv.pair_sums(x[:m1], L, kappas)
    dt1 = time.perf_counter() - t0
    rate1 = B * m1 * (m1 - 1) / 2 / dt1
    P = len(os.sched_getaffinity(0))
    with mp.get_context("spawn").Pool(P) as pool:
        _oracle_pair_sums(pool, x[:256 * P], L, kappas)   # start the workers, import the oracle
        mP = size_for(rate1 * P)
        t0 = time.perf_counter()
        _oracle_pair_sums(pool, x[:mP], L, kappas)
        dtP = time.perf_counter() - t0
    rateP = B * mP * (mP - 1) / 2 / dtP
    return {"value": rateP, "unit": "CV pair-evals/s", "cores": P, "kind": "oracle",
            "sample": f"direct FP64 pair sums (NumPy/SciPy) of the first {mP} particles x {B} kappas on {P} "
                      f"worker processes (row blocks of 256, reduced in row order): "
                      f"{B * mP * (mP - 1) / 2:.3e} pair-evals in {dtP:.1f} s",
            "one_worker": {"value": rate1, "cores": 1,
                           "sample": f"the first {m1} particles x {B} kappas: {B * m1 * (m1 - 1) / 2:.3e} pair-evals "
                                     f"in {dt1:.1f} s"},
            "all_over_one": rateP / rate1,
            "host": host_cores()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", choices=["f64", "f32"], default=None,
                    help="particle precision (default: f64 for the plain form, f32 for the batching form)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--form", choices=["plain", "precision", "batch", "serve", "tri", "fourier", "landau", "copy",
                                       "peak"],
                    default="plain",
                    help="plain: the paper-scale pipeline (default); precision: the float form on the "
                         "4096-particle plain-small set (float32-rounded positions; CV scan and the density at "
                         "every concentration) with every result's error against the FP64 oracle; batch: the batching form on 512 sets; "
                         "serve: the request server beside 16 resident PIC sessions; tri: the first-order "
                         "(triangular) shape with a CV-chosen width on the paper-scale positions; fourier: the "
                         "paper-scale pipeline through the Fourier moments (refined kappa*, exact pilot); "
                         "landau: Landau-damping ensembles on resident sessions, standard PIC against KDE; "
                         "copy: a device copy of known size that calibrates the HBM byte counters; "
                         "peak: issue-rate probes (double and float FMA, float exp2, double add)")
    ap.add_argument("--sets", type=int, default=512)
    ap.add_argument("--requests", type=int, default=2000, help="serve form: requests per load point")
    ap.add_argument("--loads", default="0.5,0.8,0.95",
                    help="serve form: offered loads as fractions of the plain path's capacity")
    ap.add_argument("--slots", type=int, default=4, help="serve form: server slots (streams)")
    ap.add_argument("--max-batch", type=int, default=16, help="serve form: requests per launch at most")
    ap.add_argument("--budget-mb", type=int, default=256,
                    help="serve form: server arena budget (requests' workspaces and attached sessions' arenas)")
    ap.add_argument("--sessions", type=int, default=16, help="serve form: resident PIC sessions")
    ap.add_argument("--session-steps", type=int, default=200, help="serve form: steps of every session per run")
    ap.add_argument("--ensembles", type=int, default=30, help="landau form: ensembles per thermal velocity")
    ap.add_argument("--vths", default="0.20,0.25,0.30,0.35,0.40,0.45", help="landau form: thermal velocities")
    ap.add_argument("--workers", type=int, default=16, help="landau form: sessions stepping at once")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of this "
              "path is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1804_11174_amd as kde
    import workloads as W

    kde.require_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.form == "peak":
        return bench_peak(args, kde, torch, dev)
    if args.form == "precision":
        return bench_precision(args, kde, W, torch, dev)
    if args.form == "batch":
        args.prec = args.prec or "f32"
        return bench_batch(args, kde, W, torch, dev)
    if args.form == "serve":
        args.prec = args.prec or "f32"
        return bench_serve(args, kde, W, torch, dev)
    if args.form == "copy":
        return bench_copy(args, torch, dev)
    if args.form == "tri":
        args.prec = args.prec or "f64"
        return bench_tri(args, kde, W, torch, dev)
    if args.form == "fourier":
        args.prec = args.prec or "f64"
        return bench_fourier(args, kde, W, torch, dev)
    if args.form == "landau":
        args.prec = args.prec or "f64"
        return bench_landau(args, kde, W, torch, dev)
    args.prec = args.prec or "f64"
    prob = W.plain_paper_scale()
    L, M, kappas, n, n_cv = prob.L, prob.M, prob.kappas, prob.x.shape[0], prob.n_cv
    tdt = torch.float64 if args.prec == "f64" else torch.float32
    prec = kde.KDE_F64 if args.prec == "f64" else kde.KDE_F32
    x = torch.from_numpy(prob.x).to(dev).to(tdt).contiguous()
    x_cv = x[:n_cv]
    B = len(kappas)

    dom_cv = kde.kde_domain(L, M, prec)
    dom = kde.kde_domain(L, M, prec)
    ws_cv, ws_dep, ws_ad = kde.Workspace(dev), kde.Workspace(dev), kde.Workspace(dev)
    p_cv, b_cv = ws_cv.get(kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom_cv, n_cv, B))
    p_dep, b_dep = ws_dep.get(kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, dom, n))
    p_ad, b_ad = ws_ad.get(kde.kde_workspace_size(kde.KDE_OP_ADAPT, dom, n))
    cv = torch.empty(B, dtype=torch.float64, device=dev)
    sums = torch.empty(2 * B, dtype=torch.float64, device=dev)
    am = torch.empty(1, dtype=torch.int32, device=dev)
    am_h = torch.empty(1, dtype=torch.int32, pin_memory=True)
    pilot = torch.empty(M, dtype=torch.float64, device=dev)
    rho = torch.empty(M, dtype=torch.float64, device=dev)
    k_i = torch.empty(n, dtype=tdt, device=dev)
    G = torch.empty(n, dtype=tdt, device=dev)
    lg = torch.empty(1, dtype=torch.float64, device=dev)
    nf = torch.empty(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        kde.kde_cv_scan(dom_cv, n_cv, x_cv, kappas, cv, sums, am, p_cv, b_cv, stream)
        am_h.copy_(am, non_blocking=True)
        stream.synchronize()
        kstar = float(kappas[int(am_h[0])])
        kde.kde_deposit(dom, n, x, None, kstar, pilot, p_dep, b_dep, stream)
        kde.kde_adapt_widths(dom, n, x, pilot, kstar, 0.5, k_i, lg, nf, p_ad, b_ad, stream)
        kde.kde_deposit(dom, n, x, k_i, 0.0, rho, p_dep, b_dep, stream)
        kde.kde_gather(dom, n, x, k_i, 0.0, rho, G, None, 0, stream)
        return kstar

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kde.kde_timing_reset()
    kde.kde_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_steps = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        kstar = step()
        torch.cuda.synchronize()
        t_steps.append((time.perf_counter() - ts) * 1e3)
    t1 = time.perf_counter()
    kde.kde_timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    kern = {}
    for name, kid in (("cv_pairs", kde.KDE_KERNEL_CV_PAIRS), ("deposit", kde.KDE_KERNEL_DEPOSIT),
                      ("gather", kde.KDE_KERNEL_GATHER), ("adapt", kde.KDE_KERNEL_ADAPT)):
        tot, cnt = kde.kde_timing_read(kid)
        kern[name] = {"launches": cnt, "avg_ms": tot / cnt if cnt else None}
    secondary = secondary_rooflines(args.prec, n, M, kern)

    pair_evals = B * n_cv * (n_cv - 1) / 2
    value = pair_evals / (ms_step * 1e-3)
    ops, evaluated, pure_terms = pair_kernel_ops(prob.x[:n_cv], L, kappas, args.prec)
    pair_ms = kern["cv_pairs"]["avg_ms"]
    achieved = ops / (pair_ms * 1e-3)
    peak = PEAK_LANE_OPS[args.prec]
    pe_rate = pair_evals / (pair_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": "cv_pairs_kernel", "achieved": achieved / 1e12,
                "peak": peak / 1e12, "unit": "T lane-ops/s (FMA = 1)",
                "frac": achieved / peak, "traffic": pair_kernel_traffic(args.prec),
                "traffic_unit": "bytes per launch",
                "basis": "algorithmic lane-operations of the method's formulas in FMA-issue slots (a float exp2 "
                         "as 4, one add per accumulated sum) over the terms at or above e^-70 of their sum's "
                         "scale, counted from the sorted positions: large-argument terms at ops_per_term, "
                         "small-argument terms (2 kappa below the Bessel split) at their own formulas",
                "evaluated_terms_per_launch": evaluated, "evaluated_fraction": evaluated / pair_evals,
                "small_argument_terms_per_launch": pure_terms, "ops_per_launch": ops,
                "ops_per_term": OPS_PER_TERM[args.prec], "ops_per_evaluated_term": ops / evaluated,
                "kernel_avg_ms": pair_ms,
                "pair_evals_per_s": pe_rate, "planning_ideal_pair_evals_per_s": PLANNING_IDEAL_PAIR_EVALS[args.prec],
                "frac_of_planning_ideal": pe_rate / PLANNING_IDEAL_PAIR_EVALS[args.prec],
                "issue": pair_kernel_issue(args.prec)}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "CV pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "plain KDE at paper scale: N=1,048,576 (CV on first 65,536), L=4pi, "
                               "M=256, 32 kappas in [1,1e4], f=(1+0.5cos(0.5x))/L",
                   "n": n, "n_cv": n_cv, "M": M, "B": B, "prec": args.prec, "parallelism": "single GPU"},
        "particles_per_s": n / (ms_step * 1e-3),
        "kappa_star": kstar,
        "kernels": kern,
        "cv_pair_kernel_pair_evals_per_s": pair_evals / (pair_ms * 1e-3),
        "step_ms": {"p10": float(np.percentile(t_steps, 10)), "p50": float(np.percentile(t_steps, 50)),
                    "p90": float(np.percentile(t_steps, 90))},
        "roofline": roofline,
        "secondary": secondary,
        "errors_vs_oracle": plain_errors(args.prec, cv.cpu().numpy(), kstar, pilot.cpu().numpy(),
                                         rho.cpu().numpy(), k_i.cpu().numpy(), G.cpu().numpy()),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob.x[:n_cv], L, kappas)
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out + "\n")


def precision_errors(cv, sums, am, grids, ref):
    """Per-result errors of the plain-small form against the oracle's: every
    grid value (relative; max over nodes, per concentration and overall),
    every CV value (relative, and relative to the curve's range max - min),
    the pair sums (relative) and whether the first minimum is the same."""
    rc = np.asarray(ref["cv"])
    rg = np.asarray(ref["grids"])
    g = np.asarray(grids)
    B = rc.shape[0]
    grid_rel = np.max(np.abs(g - rg) / np.abs(rg), axis=1)
    cv_rel = np.abs(np.asarray(cv) - rc) / np.abs(rc)
    cv_range = np.abs(np.asarray(cv) - rc) / np.ptp(rc)
    return {"grid_rel_max": float(grid_rel.max()), "grid_rel_per_kappa": grid_rel.tolist(),
            "cv_rel_max": float(cv_rel.max()), "cv_rel": cv_rel.tolist(),
            "cv_over_range_max": float(cv_range.max()), "cv_over_range": cv_range.tolist(),
            "S1_rel_max": _rel(sums[:B], ref["S1"]), "S2_rel_max": _rel(sums[B:], ref["S2"]),
            "argmin": int(am), "argmin_oracle": int(ref["argmin"]), "argmin_equal": bool(int(am) == ref["argmin"])}


def bench_precision(args, kde, W, torch, dev):
    """The precision form on the plain-small set: the 4096 float64 positions
    of the plain-small draw rounded to float32, the CV scan over its 8
    concentrations and the grid density (M = 64) at every one of them, in
    the float form (float terms, compensated float sums per thread, FP64
    normalisers, cross-thread reductions and CV combination). Errors against
    the FP64 oracle (stored by tests/golden/make_bench_references.py) on the
    same rounded positions (the float form's own error) and on the float64
    positions (adding the rounding of the input); the float64 path on the
    float64 positions alongside. A step is the scan plus the 8 deposits."""
    p = W.plain_small()
    with open(REFERENCE_FILE) as f:
        ref = json.load(f)["precision_small"]
    kappas, L, M, n = p.kappas, p.L, p.M, p.x.shape[0]
    B = len(kappas)
    runs = {}
    for name, td, prec in (("f32", torch.float32, kde.KDE_F32), ("f64", torch.float64, kde.KDE_F64)):
        x = torch.from_numpy(p.x).to(dev).to(td).contiguous()
        dom = kde.kde_domain(L, M, prec)
        wcv, wdep = kde.Workspace(dev), kde.Workspace(dev)
        p_cv, b_cv = wcv.get(kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom, n, B))
        p_dep, b_dep = wdep.get(kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, dom, n))
        cv = torch.empty(B, dtype=torch.float64, device=dev)
        sums = torch.empty(2 * B, dtype=torch.float64, device=dev)
        am = torch.empty(1, dtype=torch.int32, device=dev)
        grids = torch.empty((B, M), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream()

        def step():
            kde.kde_cv_scan(dom, n, x, kappas, cv, sums, am, p_cv, b_cv, stream)
            for b in range(B):
                kde.kde_deposit(dom, n, x, None, float(kappas[b]), grids[b], p_dep, b_dep, stream)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        out = (cv.cpu().numpy(), sums.cpu().numpy(), int(am.cpu()[0]), grids.cpu().numpy())
        runs[name] = {"ms_per_step": ms, "out": out}
    f32 = runs["f32"]["out"]
    pair_evals = B * n * (n - 1) / 2
    ms = runs["f32"]["ms_per_step"]
    line = {"metric": METRIC, "value": pair_evals / (ms * 1e-3), "unit": "CV pair-evals/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "precision form of plain-small: N=4096 positions drawn in float64 and rounded to "
                                   "float32, L=4pi, M=64, 8 kappas in [1,1e3]; CV scan + density at all 8 kappas",
                       "n": n, "M": M, "B": B, "prec": "f32", "parallelism": "single GPU"},
            "particles_per_s": n * (B + 1) / (ms * 1e-3),
            "errors_vs_oracle_same_positions": precision_errors(*f32, ref["f32_positions"]),
            "errors_vs_oracle_float64_positions": precision_errors(*f32, ref["f64_positions"]),
            "f64_path": {"ms_per_step": runs["f64"]["ms_per_step"],
                         "errors_vs_oracle": precision_errors(*runs["f64"]["out"], ref["f64_positions"])},
            "oracle_reference": "FP64 oracle, tests/golden/bench_reference.json"}
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out + "\n")


# Triangle shape, algorithmic lane-operations per evaluated (pair, width)
# term, on the basis of OPS_PER_TERM: a = max(0, 1 - u/2) and c = max(0,
# 1 - u), each a multiply-add of the distance clamped to [0, 1], 2; their
# cubes 4; the spline difference 1 (an FMA); two accumulations 2. A width
# above L/4 adds its periodic image for every pair: the image's a and the
# cube added, 3. The per-pair distance (3-4 operations) is shared by all
# widths and not counted.
TRI_OPS_PER_TERM = {"f64": 9, "f32": 9}
TRI_OPS_PER_IMAGE_TERM = 3


def count_tri_terms(x, L, widths):
    """Exact number of (pair, width) terms of the triangle CV sums that are
    not identically zero: pairs closer than 2 h_b, and every pair for
    widths above L/4 (whose periodic image reaches back)."""
    xs = np.sort(np.asarray(x, dtype=np.float64) % L)
    n = xs.shape[0]
    ext = np.concatenate([xs, xs + L])
    total = 0
    for h in widths:
        if 2.0 * h >= L / 2:
            total += n * (n - 1) // 2
            continue
        hi = np.searchsorted(ext, xs + 2.0 * h, side="left")
        total += int(np.minimum(hi - np.arange(n) - 1, n - 1).sum())
    return total


def tri_cpu_baseline(x, L, widths, budget_s=12.0):
    """The triangle oracle's direct pair sums timed on a bounded sample."""
    from oracle import triangle as otri
    m0 = 512
    t0 = time.perf_counter()
    otri.pair_sums(x[:m0], L, widths)
    dt0 = time.perf_counter() - t0
    rate0 = len(widths) * m0 * (m0 - 1) / 2 / max(dt0, 1e-9)
    m = max(m0, min(int(math.sqrt(2 * budget_s * rate0 / len(widths))), x.shape[0]))
    t0 = time.perf_counter()
    otri.pair_sums(x[:m], L, widths)
    dt = time.perf_counter() - t0
    evals = len(widths) * m * (m - 1) / 2
    return {"value": evals / dt, "unit": "CV pair-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"direct FP64 triangle pair sums (NumPy, one thread) over the first {m} particles "
                      f"x {len(widths)} half-widths: {evals:.3e} pair-evals in {dt:.1f} s",
            "host": host_cores()}


def bench_tri(args, kde, W, torch, dev):
    """The first-order (triangular) shape with its half-width chosen by CV
    on the paper-scale positions: CV scan of the first 65,536 particles
    over 32 half-widths log-spaced in [L/(4M), L/2], the host reading h*,
    then deposit of all 1,048,576 particles at h* and the gather of that
    density back to them."""
    prob = W.plain_paper_scale()
    L, M, n, n_cv = prob.L, prob.M, prob.x.shape[0], prob.n_cv
    widths = np.geomspace(0.25 * L / M, 0.5 * L, 32)
    B = len(widths)
    tdt = torch.float64 if args.prec == "f64" else torch.float32
    prec = kde.KDE_F64 if args.prec == "f64" else kde.KDE_F32
    x = torch.from_numpy(prob.x).to(dev).to(tdt).contiguous()
    x_cv = x[:n_cv]
    dom = kde.kde_domain(L, M, prec, kde.KDE_SHAPE_TRIANGLE, 0)
    ws_cv, ws_dep = kde.Workspace(dev), kde.Workspace(dev)
    p_cv, b_cv = ws_cv.get(kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, dom, n_cv, B))
    p_dep, b_dep = ws_dep.get(kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, dom, n))
    cv = torch.empty(B, dtype=torch.float64, device=dev)
    am = torch.empty(1, dtype=torch.int32, device=dev)
    am_h = torch.empty(1, dtype=torch.int32, pin_memory=True)
    rho = torch.empty(M, dtype=torch.float64, device=dev)
    G = torch.empty(n, dtype=tdt, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        kde.kde_cv_scan(dom, n_cv, x_cv, widths, cv, None, am, p_cv, b_cv, stream)
        am_h.copy_(am, non_blocking=True)
        stream.synchronize()
        hstar = float(widths[int(am_h[0])])
        kde.kde_deposit(dom, n, x, None, hstar, rho, p_dep, b_dep, stream)
        kde.kde_gather(dom, n, x, None, hstar, rho, G, None, 0, stream)
        return hstar

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kde.kde_timing_reset()
    kde.kde_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hstar = step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    kde.kde_timing_enable(False)
    kern = {}
    for name, kid in (("tri_pairs", kde.KDE_KERNEL_CV_PAIRS), ("deposit", kde.KDE_KERNEL_DEPOSIT),
                      ("gather", kde.KDE_KERNEL_GATHER)):
        tot, cnt = kde.kde_timing_read(kid)
        kern[name] = {"launches": cnt, "avg_ms": tot / cnt if cnt else None}
    pair_evals = B * n_cv * (n_cv - 1) / 2
    evaluated = count_tri_terms(prob.x[:n_cv], L, widths)
    image_terms = int(np.sum(widths > 0.25 * L)) * n_cv * (n_cv - 1) // 2
    pair_ms = kern["tri_pairs"]["avg_ms"]
    achieved = (evaluated * TRI_OPS_PER_TERM[args.prec] + image_terms * TRI_OPS_PER_IMAGE_TERM) / (pair_ms * 1e-3)
    peak = PEAK_LANE_OPS[args.prec]
    line = {
        "metric": METRIC, "form": "tri",
        "value": pair_evals / (ms_step * 1e-3), "unit": "CV pair-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "first-order (triangular) shape, CV-chosen half-width, paper-scale positions: "
                               "N=1,048,576 (CV on first 65,536), L=4pi, M=256, 32 half-widths in [L/(4M), L/2]",
                   "n": n, "n_cv": n_cv, "M": M, "B": B, "prec": args.prec, "parallelism": "single GPU"},
        "particles_per_s": n / (ms_step * 1e-3),
        "h_star": hstar,
        "kernels": kern,
        "tri_pair_kernel_pair_evals_per_s": pair_evals / (pair_ms * 1e-3),
        "roofline": {"bound": "alu", "kernel": "tri_pairs_kernel", "achieved": achieved / 1e12,
                     "peak": peak / 1e12, "unit": "T lane-ops/s (FMA = 1)", "frac": achieved / peak,
                     "traffic": None, "evaluated_terms_per_launch": evaluated,
                     "image_terms_per_launch": image_terms, "ops_per_term": TRI_OPS_PER_TERM[args.prec],
                     "ops_per_image_term": TRI_OPS_PER_IMAGE_TERM, "kernel_avg_ms": pair_ms},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = tri_cpu_baseline(prob.x[:n_cv], L, widths)
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out + "\n")


# Fourier moments, algorithmic lane-operations per (particle, m): the
# rotation of exp(i m theta) by exp(i theta) (two products, two FMAs) and
# the two accumulations. The exact phase at the start of each run of 16 m
# (two sincos per particle) is not counted.
MOMENT_OPS = 6


def fourier_order(kmax):
    """Series order of the Fourier route for concentrations up to kmax: the
    smallest m where the product of Amos's bounds on I_nu/I_{nu-1} drops
    below 1e-18 (the rule the library applies)."""
    lg, m = 0.0, 0
    while True:
        m += 1
        nu = m - 0.5
        lg += math.log(kmax / (nu + math.sqrt(nu * nu + kmax * kmax)))
        if lg < math.log(1e-18):
            return m


def bench_fourier(args, kde, W, torch, dev):
    """The paper-scale pipeline through the Fourier moments: kde_cv_refine
    on the first 65,536 particles (scan of 32 kappas + Newton on log kappa,
    all on the device; the host reads kappa*), the exact pilot widths of all
    1,048,576 particles (kde_adapt_widths_exact), the adaptive deposit and
    the gather. Also times the Fourier scan alone against the pair-kernel
    scan of the same positions and concentrations."""
    prob = W.plain_paper_scale()
    L, M, kappas, n, n_cv = prob.L, prob.M, prob.kappas, prob.x.shape[0], prob.n_cv
    B = len(kappas)
    tdt = torch.float64 if args.prec == "f64" else torch.float32
    prec = kde.KDE_F64 if args.prec == "f64" else kde.KDE_F32
    x = torch.from_numpy(prob.x).to(dev).to(tdt).contiguous()
    x_cv = x[:n_cv]
    dom = kde.kde_domain(L, M, prec)
    wsr, wsa, wsd, wss = kde.Workspace(dev), kde.Workspace(dev), kde.Workspace(dev), kde.Workspace(dev)
    p_r, b_r = wsr.get(kde.kde_workspace_size(kde.KDE_OP_CV_REFINE, dom, n_cv, B))
    p_a, b_a = wsa.get(kde.kde_workspace_size(kde.KDE_OP_ADAPT_EXACT, dom, n))
    p_d, b_d = wsd.get(kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, dom, n))
    p_s, b_s = wss.get(kde.kde_workspace_size(kde.KDE_OP_CV_FOURIER, dom, n_cv, B))
    res = torch.empty(5, dtype=torch.float64, device=dev)
    res_h = torch.empty(5, dtype=torch.float64, pin_memory=True)
    cv = torch.empty(B, dtype=torch.float64, device=dev)
    am = torch.empty(1, dtype=torch.int32, device=dev)
    k_i = torch.empty(n, dtype=tdt, device=dev)
    rho = torch.empty(M, dtype=torch.float64, device=dev)
    G = torch.empty(n, dtype=tdt, device=dev)
    lg = torch.empty(1, dtype=torch.float64, device=dev)
    nf = torch.empty(1, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        kde.kde_cv_refine(dom, n_cv, x_cv, kappas, res, cv, am, p_r, b_r, stream)
        res_h.copy_(res, non_blocking=True)
        stream.synchronize()
        kstar = float(res_h[0])
        kde.kde_adapt_widths_exact(dom, n, x, kstar, 0.5, k_i, lg, nf, p_a, b_a, stream)
        kde.kde_deposit(dom, n, x, k_i, 0.0, rho, p_d, b_d, stream)
        kde.kde_gather(dom, n, x, k_i, 0.0, rho, G, None, 0, stream)
        return kstar

    def timed(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, out

    scan = lambda: kde.kde_cv_scan_fourier(dom, n_cv, x_cv, kappas, cv, None, am, p_s, b_s, stream)
    ms_scan, _ = timed(scan, max(args.steps, 10))
    kde.kde_timing_reset()
    kde.kde_timing_enable(True)
    ms_step, kstar = timed(step, args.steps)
    kde.kde_timing_enable(False)
    kern = {}
    for name, kid in (("moments", kde.KDE_KERNEL_MOMENTS), ("pilot_exact", kde.KDE_KERNEL_ADAPT),
                      ("deposit", kde.KDE_KERNEL_DEPOSIT), ("gather", kde.KDE_KERNEL_GATHER)):
        tot, cnt = kde.kde_timing_read(kid)
        kern[name] = {"launches": cnt, "avg_ms": tot / cnt if cnt else None}
    # the moment launches alternate between the CV subsample (series order of
    # the list's largest kappa) and all particles (order of kappa*)
    m_cv, m_star = fourier_order(float(kappas[-1])), fourier_order(kstar)
    work = (n_cv * m_cv + n * m_star) * MOMENT_OPS / 2.0  # per launch, averaged over the two kinds
    mom_ms = kern["moments"]["avg_ms"]
    peak = PEAK_LANE_OPS["f64"]
    achieved = work / (mom_ms * 1e-3)
    pair_evals = B * n_cv * (n_cv - 1) / 2
    line = {
        "metric": METRIC, "form": "fourier",
        "value": pair_evals / (ms_step * 1e-3), "value_kind": "equivalent CV pair-evals/s (no pairs are evaluated)",
        "unit": "CV pair-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "paper-scale pipeline through Fourier moments: N=1,048,576 (CV refine on first "
                               "65,536 over 32 kappas in [1,1e4]), exact pilot widths, adaptive deposit and "
                               "gather, L=4pi, M=256", "n": n, "n_cv": n_cv, "M": M, "B": B,
                   "positions": args.prec, "parallelism": "single GPU"},
        "particles_per_s": n / (ms_step * 1e-3),
        "kappa_star_refined": kstar, "refine_steps": int(res_h[3]), "kappa_star_grid": float(kappas[int(res_h[4])]),
        "scan_ms": ms_scan, "series_order_cv": m_cv, "series_order_pilot": m_star,
        "kernels": kern,
        "roofline": {"bound": "alu", "kernel": "moments_kernel", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "T lane-ops/s (FMA = 1)", "frac": achieved / peak, "traffic": None,
                     "ops_per_particle_mode": MOMENT_OPS, "kernel_avg_ms": mom_ms},
    }
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out + "\n")


def bench_landau(args, kde, W, torch, dev):
    """Linear Landau damping (Sec. III.B): for each thermal velocity, the
    same seeded ensembles (common random numbers: the same positions and
    unit-normal velocity draws for every v_th and both methods) run as
    resident sessions with standard PIC (linear weighting) and with KDE
    (CV width at t = 0 and the update rule): 2^15 particles, 256 nodes,
    dt = 0.01, 1500 steps, density perturbation 0.02 cos x. Each run's
    damping rate is the slope of log field energy through its first two
    peaks (kde_damping_rate, = 2 Im(omega)), reported per method as mean,
    spread and, for KDE, the kappa* in force between the peaks; the
    comparison with the dispersion relation's roots is made afterwards from
    this JSON line by tests/landau_table.py. Sessions step concurrently, one
    per worker thread, each on its own stream."""
    import concurrent.futures as cf
    vths = [float(v) for v in args.vths.split(",")]
    ens = [W.landau_ensemble(i) for i in range(args.ensembles)]
    e0 = ens[0]
    tdt = torch.float64 if args.prec == "f64" else torch.float32
    kappas = W.log_kappas(1.0, 1e4, 16)
    chunk = 100
    xs = [torch.from_numpy(e.x).to(dev).to(tdt).contiguous() for e in ens]
    zs = [torch.from_numpy(e.z).to(dev) for e in ens]

    def run(e_idx, vth, method):
        e = ens[e_idx]
        v = (zs[e_idx] * vth).to(tdt).contiguous()
        kw = dict(method=kde.KDE_PIC_STANDARD) if method == "standard" else dict(kappas=kappas, n_cv=e.x.shape[0])
        s = kde.Session(xs[e_idx], v, e.L, e.M, e.dt, history=e.steps, **kw)
        ks = []
        try:
            for _ in range(e.steps // chunk):
                ks.append(s.state()["kappa_star"])
                s.step(chunk)
            Wt = s.read(kde.KDE_SESSION_ENERGY).cpu().numpy()
        finally:
            s.close()
        rate, peaks = kde.kde_damping_rate(Wt, e.dt)
        kstar = float(np.mean(ks[peaks[0] // chunk: peaks[1] // chunk + 1])) if peaks[1] > 0 else float("nan")
        return rate, kstar

    jobs = [(i, vth, m) for vth in vths for i in range(args.ensembles) for m in ("standard", "kde")]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=args.workers) as ex:
        results = list(ex.map(lambda j: run(*j), jobs))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    table = []
    for vth in vths:
        row = {"v_th": vth}
        for m in ("standard", "kde"):
            r = np.array([res[0] for (i, v, mm), res in zip(jobs, results) if v == vth and mm == m])
            k = np.array([res[1] for (i, v, mm), res in zip(jobs, results) if v == vth and mm == m])
            ok = np.isfinite(r)
            sd = float(np.std(r[ok], ddof=1)) if ok.sum() > 1 else float("nan")
            entry = {"mean_rate": float(np.mean(r[ok])) if ok.any() else None, "sd": sd,
                     "runs_with_two_peaks": int(ok.sum())}
            if m == "kde":
                entry["mean_kappa_star"] = float(np.nanmean(k))
            row[m] = entry
        table.append(row)
    steps = len(jobs) * e0.steps
    line = {
        "metric": METRIC, "form": "landau",
        "value": steps * e0.x.shape[0] / wall, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": e0.steps, "warmup": 0, "ms_per_step": wall * 1e3 / e0.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "Landau damping: 2^15 particles, M=256, dt=0.01, 1500 steps, 0.02 cos x, L=2pi; "
                               f"{args.ensembles} ensembles x {len(vths)} thermal velocities x (standard PIC, KDE)",
                   "ensembles": args.ensembles, "vths": vths, "workers": args.workers, "parallelism": "single GPU"},
        "session_steps_per_s": steps / wall, "wall_s": wall, "sessions": len(jobs),
        "damping": table,
    }
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out + "\n")


def bench_batch(args, kde, W, torch, dev):
    """The batching form on independent sets (N log-uniform in [1e3, 1e5],
    alpha ~ U[0.01, 0.5], k in {0.5, 1, 2}, L = 2 pi / k, M in {64, 128, 256};
    16 kappas in [1, 1e4]; float form by default): one graph launch per step,
    against the same sets through the one-set calls, one set after another
    (the plain path: per set a CV scan, the host reading kappa*, the pilot
    deposit, the widths and the adaptive deposit)."""
    prec_name = args.prec
    tdt = torch.float64 if prec_name == "f64" else torch.float32
    sets = W.batch_sets(args.sets)
    kappas = sets[0].problem.kappas
    xs = [torch.from_numpy(s.problem.x).to(dev).to(tdt).contiguous() for s in sets]
    Ls = [s.problem.L for s in sets]
    Ms = [s.problem.M for s in sets]
    ns = np.array([x.shape[0] for x in xs], dtype=np.float64)
    B = len(kappas)
    pair_evals = float(B * np.sum(ns * (ns - 1) / 2))
    bt = kde.Batch(xs, Ls, Ms, kappas)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        bt.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bt.run(stream)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / args.steps

    # the plain path: one set after another through the one-set calls
    ws_cv, ws_dep, ws_ad = kde.Workspace(dev), kde.Workspace(dev), kde.Workspace(dev)
    prec = kde.KDE_F64 if prec_name == "f64" else kde.KDE_F32
    cv = torch.empty(B, dtype=torch.float64, device=dev)
    am = torch.empty(1, dtype=torch.int32, device=dev)
    am_h = torch.empty(1, dtype=torch.int32, pin_memory=True)
    outs = []
    for x, L, M in zip(xs, Ls, Ms):
        outs.append((torch.empty(M, dtype=torch.float64, device=dev), torch.empty(M, dtype=torch.float64, device=dev),
                     torch.empty(x.shape[0], dtype=tdt, device=dev)))

    def plain_all():
        for x, L, M, (pil, rho, k_i) in zip(xs, Ls, Ms, outs):
            n = x.shape[0]
            d = kde.kde_domain(L, M, prec)
            p1, b1 = ws_cv.get(kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, d, n, B))
            kde.kde_cv_scan(d, n, x, kappas, cv, None, am, p1, b1, stream)
            am_h.copy_(am, non_blocking=True)
            stream.synchronize()
            kstar = float(kappas[int(am_h[0])])
            p2, b2 = ws_dep.get(kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, d, n))
            kde.kde_deposit(d, n, x, None, kstar, pil, p2, b2, stream)
            p3, b3 = ws_ad.get(kde.kde_workspace_size(kde.KDE_OP_ADAPT, d, n))
            kde.kde_adapt_widths(d, n, x, pil, kstar, 0.5, k_i, None, None, p3, b3, stream)
            kde.kde_deposit(d, n, x, k_i, 0.0, rho, p2, b2, stream)

    plain_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_all()
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) * 1e3
    same = all(torch.equal(bt.rho[s], outs[s][1]) for s in range(len(xs)))
    line = {"metric": METRIC, "form": "batch", "value": pair_evals / (ms_batch * 1e-3), "unit": "CV pair-evals/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec_name,
            "data": "synthetic",
            "config": {"workload": f"batching form: {len(xs)} sets, N log-uniform in [1e3,1e5], M in {{64,128,256}}, "
                                   "16 kappas in [1,1e4]; CV scan + pilot + widths + adaptive deposit per set",
                       "sets": len(xs), "particles": int(ns.sum()), "B": B},
            "particles_per_s": float(ns.sum()) / (ms_batch * 1e-3),
            "plain_path_ms": ms_plain, "batched_over_plain_speedup": ms_plain / ms_batch,
            "batched_equals_plain_bitwise": bool(same)}
    bt.close()
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out + "\n")


COPY_BYTES = 1 << 30


def bench_copy(args, torch, dev):
    """A device-to-device copy of COPY_BYTES (torch's copy kernel), the
    reference for scaling the FETCH_SIZE / WRITE_SIZE counters: it reads and
    writes exactly COPY_BYTES per launch."""
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(json.dumps({"form": "copy", "bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES, "ms_per_copy": ms,
                      "GB_per_s": 2 * COPY_BYTES / (ms * 1e-3) / 1e9}), flush=True)


def _latency_summary(lat, t_end, reqs, B):
    lat = np.asarray(lat)
    ncv = np.array([r.problem.n_cv for r in reqs], dtype=np.float64)
    ns = np.array([r.problem.x.shape[0] for r in reqs], dtype=np.float64)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
            "requests_per_s": len(reqs) / t_end, "pair_evals_per_s": float(B * np.sum(ncv * (ncv - 1) / 2)) / t_end,
            "particles_per_s": float(ns.sum()) / t_end}


class _SessionThreads:
    """The plain path's resident sessions: a thread per session steps it
    `steps` times back to back (each step synchronous, on the session's own
    stream), recording every step's latency."""

    def __init__(self, sessions, steps):
        import threading
        self.sessions, self.nsteps, self.threading = sessions, steps, threading
        self.lat = [[] for _ in sessions]
        self.errors = []

    def _run(self, k):
        try:
            s, lat = self.sessions[k], self.lat[k]
            for _ in range(self.nsteps):
                t = time.perf_counter()
                s.step(1)
                lat.append(time.perf_counter() - t)
        except Exception as e:  # reported by join()
            self.errors.append(e)

    def start(self):
        self.threads = [self.threading.Thread(target=self._run, args=(k,), daemon=True)
                        for k in range(len(self.sessions))]
        for t in self.threads:
            t.start()

    def join(self):
        for t in self.threads:
            t.join()
        if self.errors:
            raise self.errors[0]
        lat = np.concatenate([np.asarray(v) for v in self.lat])
        return {"session_steps": int(lat.size), "session_step_p50_ms": float(np.percentile(lat, 50) * 1e3),
                "session_step_p99_ms": float(np.percentile(lat, 99) * 1e3)}


def bench_serve(args, kde, W, torch, dev):
    """The serving form: a Poisson stream of one-shot KDE requests (N
    log-uniform in [1e3, 1e6], M in {64, 128, 256, 512}, float form, CV on
    min(N, 65536) particles over 16 kappas, then pilot deposit, widths and
    adaptive deposit) beside resident PIC sessions (N = 262,144, M = 128,
    dt = 0.1), each of which takes `--session-steps` steps in every run.

    Served path: a fresh server per run with an arena of `--budget-mb`
    (256 MiB by default); the sessions are attached to it at the start of
    the run (kde_server_attach), so their arenas are charged against the
    same budget as the requests' workspaces and the scheduler steps them
    beside the request slots. Plain path: the same arrival trace FIFO
    through the one-set calls on one stream, one request at a time, while a
    thread per session steps it back to back on the session's own stream.
    The plain capacity is measured first (all requests waiting at time 0);
    each load point then replays the trace at that fraction of it through
    both paths. Request latency is completion minus arrival on the host's
    monotonic clock; a run's wall time ends when its requests and its
    session steps are all done."""
    prec = kde.KDE_F32 if args.prec == "f32" else kde.KDE_F64
    tdt = torch.float32 if args.prec == "f32" else torch.float64
    R, S = args.requests, args.session_steps
    t_gen = time.perf_counter()
    trace = W.request_stream(R, 1.0)          # arrivals at rate 1, rescaled per load point
    base_arrival = np.array([r.arrival_s for r in trace])
    kappas = trace[0].problem.kappas
    B = len(kappas)
    n_cv_cap = 65536
    budget = args.budget_mb << 20
    xs = [torch.from_numpy(r.problem.x).to(dev).to(tdt).contiguous() for r in trace]

    def outputs():
        return [(torch.empty(B, dtype=torch.float64, device=dev), torch.empty(r.problem.M, dtype=torch.float64, device=dev),
                 torch.empty(r.problem.M, dtype=torch.float64, device=dev),
                 torch.empty(r.problem.x.shape[0], dtype=tdt, device=dev), torch.empty(1, dtype=torch.float64, device=dev))
                for r in trace]

    out_srv, out_pl = outputs(), outputs()
    sess_init = [W.pic_session(i) for i in range(args.sessions)]
    sessions = [kde.Session(torch.from_numpy(si.x).to(dev).to(tdt).contiguous(),
                            torch.from_numpy(si.v).to(dev).to(tdt).contiguous(),
                            si.L, si.M, si.dt, si.kappas, si.n_cv) for si in sess_init]
    session_bytes = sum(kde.kde_session_bytes(s_.params) for s_ in sessions)
    gen_s = time.perf_counter() - t_gen

    # ---- plain path: FIFO, one request at a time, one stream
    stream = torch.cuda.Stream(device=dev)
    am = torch.empty(1, dtype=torch.int32, device=dev)
    am_h = torch.empty(1, dtype=torch.int32, pin_memory=True)
    sz_cv = sz_dep = sz_ad = 0
    for r in trace:
        d = kde.kde_domain(r.problem.L, r.problem.M, prec)
        n = r.problem.x.shape[0]
        sz_cv = max(sz_cv, kde.kde_workspace_size(kde.KDE_OP_CV_SCAN, d, min(n, n_cv_cap), B))
        sz_dep = max(sz_dep, kde.kde_workspace_size(kde.KDE_OP_DEPOSIT, d, n))
        sz_ad = max(sz_ad, kde.kde_workspace_size(kde.KDE_OP_ADAPT, d, n))
    ws = [kde.Workspace(dev) for _ in range(3)]
    (p1, b1), (p2, b2), (p3, b3) = ws[0].get(sz_cv), ws[1].get(sz_dep), ws[2].get(sz_ad)

    def plain_one(i):
        r = trace[i].problem
        x, n = xs[i], r.x.shape[0]
        ncv = min(n, n_cv_cap)
        cv, pil, rho, k_i, ks = out_pl[i]
        d = kde.kde_domain(r.L, r.M, prec)
        kde.kde_cv_scan(d, ncv, x[:ncv], kappas, cv, None, am, p1, b1, stream)
        am_h.copy_(am, non_blocking=True)
        stream.synchronize()
        kstar = float(kappas[int(am_h[0])])
        kde.kde_deposit(d, n, x, None, kstar, pil, p2, b2, stream)
        kde.kde_adapt_widths(d, n, x, pil, kstar, 0.5, k_i, None, None, p3, b3, stream)
        kde.kde_deposit(d, n, x, k_i, 0.0, rho, p2, b2, stream)
        ks.fill_(kstar)
        stream.synchronize()

    def wait_until(target):
        while True:
            d = target - time.perf_counter()
            if d <= 0:
                return
            time.sleep(min(d, 2e-4))

    def run_plain(arrival, steps=S):
        lat = np.empty(R)
        load = _SessionThreads(sessions, steps)
        t0 = time.perf_counter()
        load.start()
        with torch.cuda.stream(stream):
            for i in range(R):
                target = t0 + arrival[i]
                wait_until(target)
                plain_one(i)
                lat[i] = time.perf_counter() - target
        t_req = time.perf_counter() - t0
        sess = load.join()
        wall = time.perf_counter() - t0
        out = _latency_summary(lat, t_req, trace, B)
        out.update(sess, wall_s=wall, session_steps_per_s=sess["session_steps"] / wall)
        return out

    # ---- served path
    reqs = [kde.Server.request(xs[i], trace[i].problem.L, trace[i].problem.M, out_srv[i]) for i in range(R)]

    def run_served(arrival, steps=S, **policy):
        srv = kde.Server(kappas, prec=prec, budget_bytes=budget, nslots=args.slots, max_batch=args.max_batch,
                         n_cv=n_cv_cap, alpha=0.5, device=dev, **policy)
        try:
            lag = np.empty(R)
            t0 = time.perf_counter()
            attached = [srv.attach(s_, steps) for s_ in sessions] if steps else []
            tickets = []
            for i in range(R):
                target = t0 + arrival[i]
                wait_until(target)
                lag[i] = time.perf_counter() - target
                tickets.append(srv.submit(reqs[i]))
            res = [srv.wait(t) for t in tickets]
            sres = [srv.wait(t) for t in attached]
            wall = time.perf_counter() - t0
            if any(r["status"] != 0 for r in res + sres):
                raise RuntimeError("a served request or session step did not complete")
            st = srv.stats()
        finally:
            srv.close()
        lat = lag + np.array([r["latency_s"] for r in res])
        out = _latency_summary(lat, float(np.max(arrival + lat)), trace, B)
        out.update(session_steps=int(st["session_steps"]), session_step_p50_ms=st["session_p50_s"] * 1e3,
                   session_step_p99_ms=st["session_p99_s"] * 1e3, wall_s=wall,
                   session_steps_per_s=st["session_steps"] / wall,
                   mean_batch=float(np.mean([r["batch_size"] for r in res])), launches=int(st["launches"]))
        return out

    # warm-up: a few requests through both paths and one step of every session
    zero = np.zeros(R)
    for i in range(min(R, 32)):
        plain_one(i)
    srv = kde.Server(kappas, prec=prec, budget_bytes=budget, nslots=args.slots, max_batch=args.max_batch,
                     n_cv=n_cv_cap, alpha=0.5, device=dev)
    warm = [srv.submit(reqs[i]) for i in range(min(R, 32))]
    if any(srv.wait(t)["status"] != 0 for t in warm):
        raise RuntimeError("a warm-up request did not complete")
    srv.close()
    for s_ in sessions:
        s_.step(1)
    torch.cuda.synchronize()

    def progress(tag, sv, pl=None):
        msg = {"point": tag, "served_p99_ms": sv["p99_ms"], "served_req_per_s": sv["requests_per_s"]}
        if pl:
            msg.update(plain_p99_ms=pl["p99_ms"], plain_req_per_s=pl["requests_per_s"])
        print(json.dumps(msg), file=sys.stderr, flush=True)

    points = []
    sat_pl = run_plain(zero)
    cap_plain = sat_pl["requests_per_s"]
    sat_sv = run_served(zero)
    same = all(torch.equal(out_srv[i][2], out_pl[i][2]) and torch.equal(out_srv[i][3], out_pl[i][3]) and
               torch.equal(out_srv[i][4], out_pl[i][4]) for i in range(R))
    progress("saturated", sat_sv, sat_pl)
    points.append({"offered_load": "saturated (all requests waiting at t=0)", "served": sat_sv, "plain": sat_pl})
    # the same saturated trace under a throughput policy: no request is
    # large, so every one may batch with requests of similar cost and run
    # concurrently with other batches
    sat_tp = run_served(zero, large_terms=1e300)
    progress("saturated, throughput policy", sat_tp)
    for f in [float(v) for v in args.loads.split(",") if v]:
        rate = f * cap_plain
        arrival = base_arrival / rate
        sv = run_served(arrival)
        pl = run_plain(arrival)
        progress(f, sv, pl)
        points.append({"offered_load": f, "rate_per_s": rate, "served": sv, "plain": pl})
    ns = np.array([r.problem.x.shape[0] for r in trace], dtype=np.float64)
    line = {"metric": METRIC, "form": "serve", "value": sat_sv["pair_evals_per_s"], "unit": "CV pair-evals/s",
            "n_gpus": 1, "steps": R, "warmup": 0, "ms_per_step": 1e3 / sat_sv["requests_per_s"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
            "data": "synthetic",
            "config": {"workload": f"serving form: Poisson stream of {R} KDE/CV requests (N log-uniform in "
                                   "[1e3,1e6], M in {64,128,256,512}, CV on min(N,65536), 16 kappas in [1,1e4]) "
                                   f"beside {len(sessions)} resident PIC sessions (N=262,144, M=128, dt=0.1), "
                                   f"{S} steps each per run",
                       "requests": R, "mean_N": float(ns.mean()), "slots": args.slots, "max_batch": args.max_batch,
                       "budget_mb": args.budget_mb, "sessions": len(sessions), "session_steps_per_run": S,
                       "session_arena_mb": session_bytes / 2**20},
            "plain_capacity_requests_per_s": cap_plain,
            "served_over_plain_throughput": sat_sv["requests_per_s"] / sat_pl["requests_per_s"],
            "served_over_plain_wall": sat_pl["wall_s"] / sat_sv["wall_s"],
            "saturated_throughput_policy": sat_tp,
            "throughput_policy_over_plain": sat_tp["requests_per_s"] / sat_pl["requests_per_s"],
            "served_equals_plain_bitwise": bool(same),
            "load_points": points, "input_generation_s": gen_s}
    for s_ in sessions:
        s_.close()
    out = json.dumps(line)
    print(out, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(out + "\n")


if __name__ == "__main__":
    main()
