#!/usr/bin/env python3
"""Benchmark of the MI355X pair-counting path.

Default workload (the headline): xi(r) auto-count of 10^6 Neyman-Scott points
(2*10^4 parents, mean 50 children, sigma 1.5) in a periodic cube of side 420,
14 log bins over [0.1, 25], weights U(0.5, 1.5) with the weighted mean
separation per bin.  A step is one countpairs_xi call: cell build, pruned
cell-pair walk, pair kernel and reduction, with the inputs already resident in
HBM.  The weighted mean needs the binary64 separation of every counted pair,
so this workload runs in binary64 in either precision mode.

Also reported (one JSON line on stdout, progress on stderr): the same
catalogue unweighted with binary32 distances and binary64 edge recheck against
plain binary64, the wp(rp) 2-D histogram on the same generator, the float32
non-periodic cross count D(10^6) x R(10^7), the batch of 256 mocks
(mocks/s), the roofline of the dominant kernel, and the CPU oracle timed on a
bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1911_08275_amd import synth  # noqa: E402

# VALU issue peak of the MI355X: 256 CUs x 64 lanes per clock x 2.4 GHz =
# 39.3e12 lane-operations per second (one unpacked, unfused vector operation
# per lane and clock; an FMA counts once).  Published FLOP peaks (an FMA
# counts twice): binary64 vector 78.6, binary32 vector 157.3 (packed) TFLOP/s.
PEAK_LANE_OPS = 256 * 64 * 2.4e9
PEAK_FLOPS = {"f64": 78.6e12, "f32": 157.3e12}
# Algorithmic work per pair (lane-operations, flops):
#   xi binary64 candidate: 3 sub, 3 mul, 2 add, 1 compare      -> 9 ops, 8 flops
#   xi binary32 candidate: 3 FMA, 1 add, 1 compare (Gram form,
#     unpacked: packed binary32 arithmetic is not used)          -> 5 ops, 7 flops
#   wp binary64 candidate: 3 sub, 2 mul, 1 add, 2 compares       -> 8 ops, 6 flops
#   wp binary32 candidate: 2 FMA, 1 add, 1 sub, 2 compares       -> 6 ops, 6 flops
#   in-range pair: bin locate + count (wp: two bins)             -> 2 (3) ops
#   weighted in-range pair: bin + count, sqrt, w_i w_j, x r, 2 sums -> 7 ops, 5 flops
WORK = {("xi", "f64"): (9, 8), ("xi", "f32"): (5, 7), ("wp", "f64"): (8, 6), ("wp", "f32"): (6, 6)}
INRANGE_OPS = {"xi": 2, "wp": 3}
WEIGHTED_OPS, WEIGHTED_FLOPS = 7, 5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(fn())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, stats


TRAFFIC_FILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "k_pairs_xi_weighted_1e6_traffic*.md")))
KERNEL_SRC = os.path.join(ROOT, "paper_1911_08275_amd", "csrc", "pair_kernels.hip")


def measured_traffic(refine):
    """HBM bytes per launch of the headline pair kernel from a committed
    FETCH_SIZE / WRITE_SIZE counter summary taken at these refine factors, or
    None when none matches the kernel source and the refine factors."""
    import hashlib
    try:
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    want = ",".join(str(r) for r in refine)
    for path in TRAFFIC_FILES:
        try:
            text = open(path).read()
        except OSError:
            continue
        vals = {}
        for line in text.splitlines():
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
        if vals.get("pair_kernels.hip sha256") != src or vals.get("refine") != want:
            continue
        try:
            return int(vals["fetch bytes per launch"]) + int(vals["write bytes per launch"])
        except (KeyError, ValueError):
            continue
    return None


def roofline(stat, prec, cand, inrange, ms_pairs, weighted=False):
    """Algorithmic work of one pair-kernel launch over its HIP-event time.
    cand: candidate pairs evaluated (cp_stats.candidates); inrange: pairs
    counted by the kernel (unique pairs for an auto-count)."""
    cop, cfl = WORK[(stat, prec)]
    ops = cop * cand + (WEIGHTED_OPS if weighted else INRANGE_OPS[stat]) * inrange
    flops = cfl * cand + (WEIGHTED_FLOPS if weighted else 0) * inrange
    t = ms_pairs * 1e-3
    ach = ops / t / 1e12
    peak = PEAK_LANE_OPS / 1e12
    return {"bound": "alu", "achieved": round(ach, 3), "peak": round(peak, 3),
            "unit": "T lane-ops/s", "frac": round(ach / peak, 4), "traffic": None,
            "kernel": "k_pairs (pair kernel)", "ops_per_launch": int(ops),
            "flops_per_launch": int(flops), "flop_frac": round(flops / t / PEAK_FLOPS[prec], 4),
            "flop_peak_tflops": PEAK_FLOPS[prec] / 1e12, "ms_kernel": round(ms_pairs, 4)}


def smi_query():
    """Shader and memory clock (MHz) and power cap (W) of GPU 0 from
    rocm-smi, or None."""
    import re
    import subprocess
    try:
        out = subprocess.run(["rocm-smi", "--showclocks", "--showmaxpower", "--json"],
                             capture_output=True, text=True, timeout=30).stdout
        d = json.loads(out[out.index("{"):])
    except Exception:
        return None
    card = next((v for k, v in d.items() if k.lower().startswith("card")), None)
    if not isinstance(card, dict):
        return None
    res = {}
    for k, v in card.items():
        kl, vs = k.lower(), str(v).lower()
        m = re.search(r"(\d+(?:\.\d+)?)\s*mhz", vs)
        if "sclk" in kl and m:
            res["sclk_mhz"] = float(m.group(1))
        elif "mclk" in kl and m:
            res["mclk_mhz"] = float(m.group(1))
        elif "power" in kl and "max" in kl:
            n = re.search(r"\d+(?:\.\d+)?", vs)
            if n:
                res["power_cap_w"] = float(n.group(0))
    return res or None


def clocks_under_load(fn, seconds):
    """Runs fn() back to back for about `seconds` while a thread samples
    rocm-smi; returns the shader clocks seen (MHz) and the power cap."""
    import threading
    import torch
    samples, caps = [], []
    stop = threading.Event()

    def poll():
        while not stop.is_set():
            q = smi_query()
            if q and "sclk_mhz" in q:
                samples.append(q["sclk_mhz"])
                if "power_cap_w" in q:
                    caps.append(q["power_cap_w"])
            if q is None:
                return
    th = threading.Thread(target=poll, daemon=True)
    th.start()
    t0 = time.time()
    while time.time() - t0 < seconds:
        fn()
    torch.cuda.synchronize()
    stop.set()
    th.join(timeout=40)
    return samples, (caps[0] if caps else None)


def rocm_version():
    try:
        return open("/opt/rocm/.info/version").read().strip()
    except OSError:
        return None


def _median_call(fn, steps):
    """Median device time of the whole call (ms_total) and the last result."""
    fn()
    res = [fn() for _ in range(steps)]
    return float(np.median([r.stats["ms_total"] for r in res])), res[-1]


def sweep_refine(native, steps):
    """Refine factors and bounding-box pruning on the headline catalogue
    (the paper's refine-factor and pruning experiments of Sections 3.1 and 3.2, on
    the MI355X): device time of one call per refine (r_x, r_y, r_z), pruning
    on and off, for weighted binary64 xi and unweighted binary32+recheck xi.
    Every configuration must give identical counts."""
    c2 = synth.config2()
    d2 = native.to_device(c2["cat"])
    e2 = c2["edges"]
    log("c2 generated, n =", c2["cat"].n)
    ref = None
    rows = []
    grid = [(rx, ry, rz) for rz in (1, 2, 3) for rx in (1, 2, 3) for ry in (1, 2, 3)]
    for refine in grid:
        row = {"refine": list(refine)}
        for label, prec, w in (("w64", "fp64", True), ("u32", "fp32", False)):
            for prune in (True, False):
                ms, g = _median_call(lambda: native.countpairs_xi(
                    d2, e2, precision=prec, periodic=True, boxsize=420.0, need_ravg=w,
                    refine=refine, no_prune=not prune), steps)
                if ref is None:
                    ref = g.npairs.copy()
                same = bool((g.npairs == ref).all())
                key = f"{label}_{'prune' if prune else 'noprune'}"
                row[key] = {"ms": round(ms, 4), "candidates": g.stats["candidates"],
                            "units": g.stats["cell_pairs"],
                            "pruned": g.stats["cell_pairs_pruned"], "same_counts": same}
        log(json.dumps(row))
        rows.append(row)
    auto = {}
    for label, prec, w in (("w64", "fp64", True), ("u32", "fp32", False)):
        g = native.countpairs_xi(d2, e2, precision=prec, periodic=True, boxsize=420.0,
                                 need_ravg=w, refine="auto")
        auto[label] = g.stats["refine"]
    all_same = all(r[k]["same_counts"] for r in rows for k in r if k != "refine")
    print("| refine | w64 pruned ms | w64 unpruned ms | u32 pruned ms | u32 unpruned ms | "
          "candidates pruned / unpruned (u32) | units skipped |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {tuple(r['refine'])} | {r['w64_prune']['ms']:.3f} | {r['w64_noprune']['ms']:.3f} "
              f"| {r['u32_prune']['ms']:.3f} | {r['u32_noprune']['ms']:.3f} | "
              f"{r['u32_prune']['candidates'] / 1e9:.2f}e9 / "
              f"{r['u32_noprune']['candidates'] / 1e9:.2f}e9 | {r['u32_prune']['pruned']} |")
    print(json.dumps({"sweep": "refine", "rows": rows, "autotuned": auto,
                      "counts_identical": all_same}), flush=True)


def sweep_rmax(native, steps):
    """R_max scaling (the paper's Section 3.3 experiment, on the MI355X): xi
    with 14 log bins over [0.1, R] and wp with pi_max = R, 1-wide pi bins, on
    the headline catalogue, binary64 and binary32+recheck, refine from the
    autotuner; the CPU oracle is timed on a random sample of primaries against
    the whole catalogue, and the GPU cross count of that sample must equal it."""
    import oracle
    c2 = synth.config2()
    cat = c2["cat"]
    d2 = native.to_device(cat)
    log("c2 generated, n =", cat.n)
    rng = np.random.Generator(np.random.PCG64(77))
    rows = []
    for R in (10.0, 20.0, 40.0, 80.0, 100.0):
        edges = synth.log_edges(0.1, R, 14)
        npi = int(R)
        row = {"rmax": R}
        for stat in ("xi", "wp"):
            def call(prec, refine="auto", d=d2):
                if stat == "xi":
                    return native.countpairs_xi(d, edges, precision=prec, periodic=True,
                                                boxsize=420.0, refine=refine)
                return native.countpairs_wp(d, edges, R, npi, precision=prec, periodic=True,
                                            boxsize=420.0, refine=refine)
            res = {}
            for prec in ("fp64", "fp32"):
                ms, g = _median_call(lambda: call(prec), steps)
                res[prec] = (ms, g)
            pairs = int(res["fp64"][1].npairs.sum())
            # oracle on a sample of primaries sized for about a second of CPU work
            per = max(1.0, pairs / cat.n)
            nprim = int(min(cat.n, max(2000, 3e8 / per)))
            idx = np.sort(rng.choice(cat.n, nprim, replace=False))
            sub = cat.subset(idx)
            t = time.perf_counter()
            if stat == "xi":
                ref = oracle.xi(sub, edges, periodic=True, box=420.0, other=cat)
            else:
                ref = oracle.wp(sub, edges, R, npi, periodic=True, box=420.0, other=cat)
            tcpu = time.perf_counter() - t
            if stat == "xi":
                gs = native.countpairs_cross(native.to_device(sub), d2, edges, periodic=True,
                                             boxsize=420.0)
            else:
                gs = native.countpairs_cross_wp(native.to_device(sub), d2, edges, R, npi,
                                                periodic=True, boxsize=420.0)
            row[stat] = {
                "pairs": pairs,
                "fp64_ms": round(res["fp64"][0], 4), "fp32_ms": round(res["fp32"][0], 4),
                "refine_fp64": res["fp64"][1].stats["refine"],
                "refine_fp32": res["fp32"][1].stats["refine"],
                "fp64_pairs_per_s": pairs / (res["fp64"][0] * 1e-3),
                "fp32_pairs_per_s": pairs / (res["fp32"][0] * 1e-3),
                "candidates_fp32": res["fp32"][1].stats["candidates"],
                "recheck_fraction": res["fp32"][1].stats["rechecks"] / max(1, pairs // 2),
                "counts_equal_fp32_fp64": bool((res["fp64"][1].npairs ==
                                                res["fp32"][1].npairs).all()),
                "oracle_pairs_per_s": float(ref.npairs.sum()) / tcpu,
                "oracle_sample": f"{nprim} primaries, {tcpu:.2f} s",
                "gpu_matches_oracle_on_sample": bool(
                    (gs.npairs.reshape(ref.npairs.shape) == ref.npairs).all())}
        log(json.dumps(row))
        rows.append(row)
    print("| R_max | stat | in-range pairs | fp64 ms | fp32 ms | fp32 pairs/s | refine (fp32) | "
          "oracle pairs/s (sample) | GPU fp32 / oracle | exact |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        for stat in ("xi", "wp"):
            v = r[stat]
            ok = v["counts_equal_fp32_fp64"] and v["gpu_matches_oracle_on_sample"]
            print(f"| {r['rmax']:g} | {stat} | {v['pairs']:.3e} | {v['fp64_ms']:.3f} | "
                  f"{v['fp32_ms']:.3f} | {v['fp32_pairs_per_s']:.3e} | "
                  f"{tuple(v['refine_fp32'])} | {v['oracle_pairs_per_s']:.3e} | "
                  f"{v['fp32_pairs_per_s'] / v['oracle_pairs_per_s']:.0f} | {ok} |")
    print(json.dumps({"sweep": "rmax", "rows": rows, "oracle_threads": oracle.num_threads()}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-mock batch")
    ap.add_argument("--refine", type=str, default=None, help="e.g. 2,2,1")
    ap.add_argument("--no-clock", action="store_true",
                    help="skip rocm-smi (shader clock under load, power cap): profiled runs")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--sweep", choices=("refine", "rmax"), default=None,
                    help="instead of the benchmark: refine/pruning sweep or R_max scaling "
                         "sweep (markdown table and one JSON line on stdout)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the pair counts "
              "of this workload fit one MI355X and the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_1911_08275_amd import native
    native.lib()  # fails loudly when the HIP library is missing
    if args.sweep == "refine":
        sweep_refine(native, max(3, args.steps // 3))
        return
    if args.sweep == "rmax":
        sweep_rmax(native, max(3, args.steps // 3))
        return
    refine = tuple(int(v) for v in args.refine.split(",")) if args.refine else None
    # refine factors: given, or picked by the autotuner on first use (during
    # warm-up, outside the timed steps)
    rk = {"refine": refine if refine is not None else "auto"}

    # ---------------------------------------------------------- headline: C2
    c2 = synth.config2()
    d2 = native.to_device(c2["cat"])
    e2 = c2["edges"]
    log("c2 generated, n =", c2["cat"].n)

    def step(prec, weighted=True):
        def f():
            return native.countpairs_xi(d2, e2, precision=prec, periodic=True, boxsize=420.0,
                                        need_ravg=weighted, **rk)
        return f

    def mean_ms(stats, key="ms_pairs"):
        return float(np.mean([x.stats[key] for x in stats]))

    # Headline: weighted xi.  Every counted pair needs its binary64 separation;
    # the library runs the binary64 kernel in either precision mode (measured
    # faster on gfx950) unless CP_XI_WEIGHTED_BINARY32=1 selects the binary32
    # screen, which is timed beside it.
    dtw, sw = time_steps(step("fp64"), args.steps, args.warmup)
    log(f"c2 weighted (binary64): {dtw * 1e3:.3f} ms/step", sw[-1].stats)
    os.environ["CP_XI_WEIGHTED_BINARY32"] = "1"
    try:
        dtws, sws = time_steps(step("fp32"), max(3, args.steps // 2), 1)
    finally:
        del os.environ["CP_XI_WEIGHTED_BINARY32"]
    log(f"c2 weighted (binary32 screen): {dtws * 1e3:.3f} ms/step", sws[-1].stats)
    dt32, s32 = time_steps(step("fp32", False), max(3, args.steps // 2), 1)
    log(f"c2 unweighted fp32+recheck: {dt32 * 1e3:.3f} ms/step", s32[-1].stats)
    dt64, s64 = time_steps(step("fp64", False), max(3, args.steps // 2), 1)
    log(f"c2 unweighted fp64: {dt64 * 1e3:.3f} ms/step", s64[-1].stats)
    gw, gws, g32, g64 = sw[-1], sws[-1], s32[-1], s64[-1]
    exact = bool((g32.npairs == g64.npairs).all() and (gw.npairs == g64.npairs).all()
                 and (gws.npairs == g64.npairs).all())
    pairs = int(gw.npairs.sum())                  # ordered in-range pairs
    uniq = pairs // 2                             # pairs the kernel counts
    ms_w = mean_ms(sw)
    st = gw.stats
    roof = roofline("xi", "f64", st["candidates"], uniq, ms_w, weighted=True)
    roof["traffic"] = measured_traffic(st["refine"])
    roof_ws = roofline("xi", "f32", gws.stats["candidates"], uniq, mean_ms(sws), weighted=True)
    roof32 = roofline("xi", "f32", g32.stats["candidates"], uniq, mean_ms(s32))
    roof64 = roofline("xi", "f64", g64.stats["candidates"], uniq, mean_ms(s64))

    # shader clock under load (rocm-smi sampled while the headline runs back
    # to back, outside the timed steps), power cap, ROCm version
    # (rocm-smi is a script started through /usr/bin/env: profiled runs skip it)
    idle = None if args.no_clock else smi_query()
    sclk, cap = ([], None) if args.no_clock else clocks_under_load(step("fp64"), 3.0)
    machine = {"rocm": rocm_version(),
               "sclk_mhz_under_load": {"min": min(sclk), "median": float(np.median(sclk)),
                                       "max": max(sclk), "samples": len(sclk)} if sclk else None,
               "sclk_mhz_idle": (idle or {}).get("sclk_mhz"),
               "mclk_mhz_idle": (idle or {}).get("mclk_mhz"),
               "power_cap_w": cap if cap is not None else (idle or {}).get("power_cap_w"),
               "peak_assumes_sclk_mhz": 2400}
    log("machine:", machine)

    out = {
        "metric": "pair evaluations/sec and mocks/sec, FP32+recheck vs FP64, counts bit-exact",
        "value": pairs / dtw,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dtw * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "xi(r) auto-count, 1e6 Neyman-Scott points (2e4 parents, "
                               "Poisson(50) children, sigma 1.5), periodic L=420, 14 log bins "
                               "0.1-25, weights U(0.5,1.5) with weighted mean r; binary64 kernel "
                               "(what either precision mode runs for weighted xi)",
                   "n": c2["cat"].n, "nbins": 14, "rmax": 25.0, "box": 420.0,
                   "grid": st["grid"], "refine": st["refine"]},
        "pairs_per_step": pairs,
        "candidates_per_step": st["candidates"],
        "candidate_rate": st["candidates"] / dtw,
        "candidates_per_inrange_pair": st["candidates"] / max(1, uniq),
        "ms_pairs_kernel": ms_w,
        "ms_grid": mean_ms(sw, "ms_grid"),
        "weighted_binary32_screen": {
            "value": pairs / dtws, "ms_per_step": dtws * 1e3, "ms_pairs_kernel": mean_ms(sws),
            "precision_ran": gws.stats["precision"],
            "recheck_fraction": gws.stats["rechecks"] / max(1, uniq),
            "roofline_frac": roof_ws["frac"], "flop_frac": roof_ws["flop_frac"],
            "over_binary64": dtw / dtws},
        "unweighted": {
            "fp32": {"value": pairs / dt32, "ms_per_step": dt32 * 1e3,
                     "ms_pairs_kernel": mean_ms(s32), "refine": g32.stats["refine"],
                     "candidates": g32.stats["candidates"],
                     "recheck_fraction": g32.stats["rechecks"] / max(1, uniq),
                     "roofline_frac": roof32["frac"], "flop_frac": roof32["flop_frac"]},
            "fp64": {"value": pairs / dt64, "ms_per_step": dt64 * 1e3,
                     "ms_pairs_kernel": mean_ms(s64), "refine": g64.stats["refine"],
                     "candidates": g64.stats["candidates"],
                     "roofline_frac": roof64["frac"], "flop_frac": roof64["flop_frac"]},
            "fp32_over_fp64": dt64 / dt32},
        "counts_equal_fp32_fp64_weighted": exact,
        "machine": machine,
        "roofline": roof,
    }

    extras = {}
    if not args.quick:
        # ------------------------------------------------------ C3: wp 2-D
        c3 = synth.config3()
        d3 = native.to_device(c3["cat"])
        res = {}
        for prec in ("fp32", "fp64"):
            dt, ss = time_steps(lambda: native.countpairs_wp(
                d3, c3["edges"], 40.0, 40, precision=prec, periodic=True, boxsize=420.0, **rk),
                max(3, args.steps // 2), 1)
            res[prec] = (dt, ss[-1])
            log(f"c3 wp {prec}: {dt * 1e3:.3f} ms/step", ss[-1].stats)
        p3 = int(res["fp32"][1].npairs.sum())

        def leg(stat, prec, pairs_, counted, dt, g):
            r = roofline(stat, "f32" if prec == "fp32" else "f64", g.stats["candidates"],
                         counted, g.stats["ms_pairs"])
            return {"value": pairs_ / dt, "ms": dt * 1e3, "ms_pairs_kernel": g.stats["ms_pairs"],
                    "candidates": g.stats["candidates"], "refine": g.stats["refine"],
                    "precision_ran": g.stats["precision"],
                    "recheck_fraction": g.stats["rechecks"] / max(1, counted),
                    "roofline_frac": r["frac"], "flop_frac": r["flop_frac"]}
        extras["wp_c3"] = {"pairs_per_step": p3,
                           "fp32": leg("wp", "fp32", p3, p3 // 2, *res["fp32"]),
                           "fp64": leg("wp", "fp64", p3, p3 // 2, *res["fp64"]),
                           "counts_equal": bool((res["fp32"][1].npairs ==
                                                 res["fp64"][1].npairs).all())}
        del d3
        # ---------------------------------------------------- C4: cross DR
        c4 = synth.config4()
        dd, dr = native.to_device(c4["d"]), native.to_device(c4["r"])
        res = {}
        for prec in ("fp32", "fp64"):
            dt, ss = time_steps(lambda: native.countpairs_cross(
                dd, dr, c4["edges"], precision=prec, periodic=False, **rk),
                max(2, args.steps // 3), 1)
            res[prec] = (dt, ss[-1])
            log(f"c4 cross {prec}: {dt * 1e3:.3f} ms/step", ss[-1].stats)
        p4 = int(res["fp32"][1].npairs.sum())
        extras["cross_c4"] = {"pairs_per_step": p4,
                              "fp32": leg("xi", "fp32", p4, p4, *res["fp32"]),
                              "fp64": leg("xi", "fp64", p4, p4, *res["fp64"]),
                              "counts_equal": bool((res["fp32"][1].npairs ==
                                                    res["fp64"][1].npairs).all())}
        del dd, dr
        torch.cuda.empty_cache()
        # ---------------------------------------------------- C5: 256 mocks
        if not args.no_batch:
            specs = synth.mock_specs()
            t = time.perf_counter()
            with ThreadPoolExecutor(8) as ex:
                cats = list(ex.map(synth.mock, specs))
            log(f"c5 generated {len(cats)} mocks, {sum(c.n for c in cats)} points in "
                f"{time.perf_counter() - t:.1f}s")
            devs = [native.to_device(c) for c in cats]
            del cats
            xe = synth.log_edges(0.1, 25.0, 14)
            bres = {}
            for prec in ("fp32", "fp64"):
                plan = native.Plan(devs, xi_edges=xe, wp_edges=xe, pimax=40.0, npibins=40,
                                   precision=prec, periodic=True, boxsize=420.0, **rk)
                nrep = 2 if prec == "fp32" else 1
                plan.execute()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(nrep):
                    plan.execute()
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t) / nrep
                xi, wp = plan.results()
                sx, sw = plan.stats()
                bres[prec] = (dt, xi, wp, sx, sw)
                log(f"c5 batch {prec}: {dt:.3f} s per evaluation of 256 mocks")
                plan.close()
            dt = bres["fp32"][0]
            pairs5 = int(bres["fp32"][1].sum() + bres["fp32"][2].sum())
            extras["batch_c5"] = {
                "mocks": len(devs), "points": int(sum(d.n for d in devs)),
                "mocks_per_s": len(devs) / dt, "s_per_eval": dt,
                "pairs_per_eval": pairs5, "pairs_per_s": pairs5 / dt,
                "fp64_mocks_per_s": len(devs) / bres["fp64"][0],
                "counts_equal": bool((bres["fp32"][1] == bres["fp64"][1]).all() and
                                     (bres["fp32"][2] == bres["fp64"][2]).all()),
                "graph_ms": bres["fp32"][3]["ms_total"],
                "xi_candidates": bres["fp32"][3]["candidates"],
                "wp_candidates": bres["fp32"][4]["candidates"]}
            # roofline of the whole evaluation (cell builds included, so a
            # lower bound for the pair kernels): binary32 work of both
            # statistics over the wall time of one graph replay
            px, pw = int(bres["fp32"][1].sum()) // 2, int(bres["fp32"][2].sum()) // 2
            ops = (WORK[("xi", "f32")][0] * bres["fp32"][3]["candidates"] + INRANGE_OPS["xi"] * px +
                   WORK[("wp", "f32")][0] * bres["fp32"][4]["candidates"] + INRANGE_OPS["wp"] * pw)
            extras["batch_c5"]["roofline_frac_incl_build"] = round(ops / dt / PEAK_LANE_OPS, 4)
            extras["batch_c5"]["recheck_fraction"] = (
                (bres["fp32"][3]["rechecks"] + bres["fp32"][4]["rechecks"]) / max(1, px + pw))
            del devs
            torch.cuda.empty_cache()
    if extras:
        out["extras"] = extras

    if args.copy_calib:
        # a plain copy kernel of known size (reads and writes 256 MiB each), to
        # scale the FETCH_SIZE / WRITE_SIZE memory counters
        a = torch.empty(256 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = a.numel() * 4

    # ------------------------------------------------- CPU oracle baseline
    if not args.no_cpu:
        import oracle
        rng = np.random.Generator(np.random.PCG64(123))
        frac = 0.25
        idx = np.sort(rng.choice(c2["cat"].n, int(frac * c2["cat"].n), replace=False))
        sub = c2["cat"].subset(idx)
        t = time.perf_counter()
        ref = oracle.xi(sub, e2, periodic=True, box=420.0, other=c2["cat"])
        tcpu = time.perf_counter() - t
        # the same sample through the GPU cross path must agree exactly
        gs = native.countpairs_cross(native.to_device(sub), d2, e2, periodic=True, boxsize=420.0,
                                     need_ravg=True, **rk)
        same = bool((gs.npairs == ref.npairs).all())
        rel = float(np.max(np.abs(gs.wsum - ref.wsum) / np.maximum(ref.wsum, 1e-300)))
        out["cpu_baseline"] = {
            "value": float(ref.npairs.sum()) / tcpu, "unit": "pairs/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{len(idx)} random primaries (25%) of the headline catalogue against all "
                      f"1e6 points (cross count, weighted, periodic); {tcpu:.1f} s",
            "gpu_matches_oracle_on_sample": same, "wsum_max_rel_err": rel}
        # per-core rate: one thread on a 2 % sample
        idx1 = np.sort(rng.choice(c2["cat"].n, c2["cat"].n // 50, replace=False))
        sub1 = c2["cat"].subset(idx1)
        t = time.perf_counter()
        ref1 = oracle.xi(sub1, e2, periodic=True, box=420.0, other=c2["cat"], nthreads=1)
        t1 = time.perf_counter() - t
        out["cpu_baseline"]["one_thread"] = {
            "value": float(ref1.npairs.sum()) / t1, "unit": "pairs/s",
            "sample": f"{len(idx1)} random primaries (2%) against all 1e6 points; {t1:.1f} s"}
        log(f"cpu oracle: {tcpu:.1f} s on {oracle.num_threads()} threads, match={same}; "
            f"one thread {t1:.1f} s")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
