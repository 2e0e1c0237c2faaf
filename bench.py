"""Benchmark: exact 2D hulls of the paper's 20M-point workloads on one MI355X.

One step = one hull2d_compute of each set of the workload (20,000,000 points
uniform in [0,1)^2 and 20,000,000 points uniform in the unit disk, the shapes
and sizes of the paper's Section 4 groups 1 and 2), inputs resident in HBM.
The step covers every stage: extremes, round-1 discard with exact keys, the
round-2 filter over the candidates of the angle buckets (sorted in the exact
angular order), the copy of the kept points to the host and the host stack
scan.

Prints one JSON line: the headline rate over both sets, the roofline of the
dominant kernel (algorithmic bytes over its measured time, and its counted
HBM traffic), per-kernel times, the other legs (full sort, four-region
variant, adversarial inputs, the batched form with both engines, the learned
filter) and the CPU oracle's rate.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpoints/s exact 2D hull at 20M pts (plain vs learned-filter/batched); HBM GB/s"
HBM_PEAK_GBPS = 8000.0
# The paper's gScan total (GPU + CPU) at 20M points on its faster platform
# (GeForce GT 640, Tables 3 and 5): 446.4 ms (square) + 418.1 ms (disk).
PAPER_MS_SQUARE_DISK_20M = 446.4 + 418.1

# HBM traffic of one launch from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0, the factors a plain 320 MB copy gives), averaged over the
# square and disk launches, with the SHA-256 of every source the kernel is
# built from: once a source differs, the figure no longer describes the
# kernel and `traffic` is null.
TRAFFIC = {
    "filter1": {
        "bytes": 534_000_000,  # 320.3 MB fetched + 213.7 MB written
        "profile": "profiles/hull_square_disk_20M_hbm_counters.md",
        "sources": {
            "paper_1508_05931_amd/csrc/kernels_filter.hip":
                "0228e0b387a19da152fc4287fc4d55071941023087765fb771ee816d1db5c34d",
            "paper_1508_05931_amd/csrc/steps.hpp":
                "33fa676280d55236357f5fab49d6890917f601f226406e1aaa653063fafa9744",
            "paper_1508_05931_amd/csrc/exact.hpp":
                "492fba6ee743cba0bb741d699072aaffa58163bfd2ddf06fa43db6642a3a9861",
            "paper_1508_05931_amd/csrc/common.hpp":
                "b945234c8a977df749c303e9fadbe0b97853518d9b1324d8323dd32fc2e11fd8",
            "paper_1508_05931_amd/csrc/kernels.hpp":
                "bec1a4687ab4f3693c831227513bcb66ff7d49d6249bcd3441975fde7968e309",
        },
    },
}


TRAFFIC["batch_tiled"] = {
    # all kernels of one hull2d_batch call of the tiled engine on the 4096-set
    # workload with the tuned schedule (both streams), same scale factors
    "bytes": 8_918_800_000,  # 6,830.8 MB fetched + 2,088.0 MB written
    "profile": "profiles/hull_batch_4096_sets_kernel_trace.md",
    "sources": {
        "paper_1508_05931_amd/csrc/kernels_batch.hip":
            "683f6205368a9b5ef8020fa5d5e6642693f3e9b15d15280ce9f1634b00b30dae",
        "paper_1508_05931_amd/csrc/kernels.hpp":
            "bec1a4687ab4f3693c831227513bcb66ff7d49d6249bcd3441975fde7968e309",
        "paper_1508_05931_amd/csrc/steps.hpp":
            "33fa676280d55236357f5fab49d6890917f601f226406e1aaa653063fafa9744",
        "paper_1508_05931_amd/csrc/exact.hpp":
            "492fba6ee743cba0bb741d699072aaffa58163bfd2ddf06fa43db6642a3a9861",
        "paper_1508_05931_amd/csrc/common.hpp":
            "b945234c8a977df749c303e9fadbe0b97853518d9b1324d8323dd32fc2e11fd8",
        "paper_1508_05931_amd/csrc/hull2d_api.cpp":
            "3f83169190397b1c42e80633cd7d8c280a665c6a93955c82e538221767ac8be6",
        "paper_1508_05931_amd/tuning/batch.json":
            "d53dc0fcea061e10bd57df56b5b7370304b9f75d4147c3b108c3426c8ef753de",
    },
}


def measured_traffic(kernel: str):
    """Profiled HBM bytes per launch of `kernel`, or None when there is no
    profile or the kernel's sources changed since it was taken."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None or t["bytes"] is None:
        return None
    for rel, digest in t["sources"].items():
        path = os.path.join(ROOT, rel)
        if not os.path.exists(path):
            return None
        with open(path, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return t["bytes"]


KERNEL_STAGES = ["extremes", "filter1", "longest", "buckets", "histogram", "sort0", "sort1",
                 "sort2", "sort3", "ties", "ties_long", "round2", "compact", "tail", "scan"]


def kernel_bytes(stage: str, n: int, ms: int, nc: int, m2: int, full: bool) -> float:
    """Algorithmic HBM bytes of one launch: what the kernel must read and
    write at least once (float64 x,y = 16 B, index/key/slot = 4 B, flag = 1 B).
    n points, ms sorted round-1 survivors, nc points sorted for round 2
    (= ms when every survivor is sorted), m2 kept points."""
    return {
        "extremes": 16.0 * n,
        "filter1": 16.0 * n + 24.0 * ms,
        "longest": 0.0,
        # bucketed: maxima over a 1/8 sample of the survivors (20 B each),
        # then every survivor classified, candidates written (28 B each)
        "buckets": 12.0 * ms if full else 22.5 * ms + 28.0 * nc,
        "histogram": 4.0 * nc,
        "sort0": 12.0 * nc,
        "sort1": 16.0 * nc,
        "sort2": 16.0 * nc,
        "sort3": 16.0 * nc,
        "ties": 8.0 * nc,
        "ties_long": 0.0,
        "round2": 21.0 * nc,
        "compact": 1.0 * nc + 44.0 * m2,
        # candidates' keys read, kept points read and written to the host
        "tail": 8.0 * nc + 40.0 * m2,
        # Step 8 on the device: the kept points read (20 B each)
        "scan": 20.0 * m2,
    }[stage]


def cpu_baseline(sets, names, reps: int):
    """The oracle (single-threaded C monotone chain) on the full sets of the
    workload, timed on this host: the median of `reps` runs per set."""
    import numpy as np
    import oracle
    total_pts, total_s, per = 0, 0.0, {}
    for nm, pts in zip(names, sets):
        ts = []
        for _ in range(max(1, reps)):
            t0 = time.perf_counter()
            oracle.hull(pts)
            ts.append(time.perf_counter() - t0)
        med = float(np.median(ts))
        progress(f"oracle on {nm}: {med:.1f} s")
        per[nm] = round(med, 2)
        total_s += med
        total_pts += pts.shape[0]
    return {"value": round(total_pts / total_s / 1e6, 3), "unit": "Mpoints/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the full sets {' + '.join(names)} ({total_pts} points), median of "
                      f"{max(1, reps)} run(s) per set, seconds {per}, on "
                      f"{platform.processor() or platform.machine()} "
                      f"({os.cpu_count()} logical CPUs, one used)"}


def learned(steps: int):
    """The learned first-round filter against the quadrilateral on the 20M
    anisotropic Gaussian mixture (the shape the paper's third group stands in
    for), with the weights shipped in the package."""
    import numpy as np
    import torch
    import paper_1508_05931_amd as hx
    import synth
    w = os.path.join(ROOT, "paper_1508_05931_amd", "weights", "filter16.f32")
    if not os.path.exists(w):
        return None
    d = torch.from_numpy(synth.workload("mixture_20M")).cuda()
    out = {"workload": "mixture_20M", "weights": "paper_1508_05931_amd/weights/filter16.f32"}
    hulls = {}
    for key, ctx in (("quad", hx.Hull2D(profile=2)),
                     ("learned", hx.Hull2D(profile=2, learned=True, weights=w))):
        hulls[key] = ctx.compute(d)
        torch.cuda.synchronize()
        reps = max(3, steps // 2)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            ctx.compute(d)
            ts.append(time.perf_counter() - t0)
        st = ctx.last_stats
        ms = float(np.median(ts)) * 1e3
        out[key] = {"ms_median": round(ms, 4), "Mpoints_per_s": round(d.shape[0] / (ms * 1e-3) / 1e6, 1),
                    "survivors_round1": int(st.n_round1), "n_hull": int(st.n_hull),
                    "survivors_round2": int(st.n_round2), "sorted_for_round2": int(st.n_candidates)}
        ctx.close()
    out["identical_output"] = bool(np.array_equal(hulls["quad"], hulls["learned"]))
    return out


def batched(steps: int):
    """The batched form on 4096 independent sets (sizes log-uniform in
    [64, 200000], squares, disks, Gaussians and thin annuli; 99.9M points),
    inputs resident in HBM: one hull2d_batch call per step."""
    import numpy as np
    import torch
    import paper_1508_05931_amd as hx
    import synth
    pts, offs, _ = synth.batch(4096)
    d = torch.from_numpy(pts).cuda()
    reps = max(3, steps // 4)

    def run(engine):
        c = hx.Hull2D(batch_engine=engine)
        c.batch(d, offs)
        torch.cuda.synchronize()
        ts, dev = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            c.batch(d, offs)
            ts.append(time.perf_counter() - t0)
            dev.append(float(c.last_stats.ms_device))
        return c, float(np.median(ts)) * 1e3, float(np.median(dev))

    # the persistent engine (one workgroup per set) for comparison, then the
    # default tiled engine, whose context the per-set loop below reuses
    cp, ms_p, dev_p = run(1)
    cp.close()
    ctx, ms, dev_ms = run(0)
    st = ctx.last_stats
    # the same sets through the plain single-hull path, one call per set
    views = [d[offs[i]:offs[i + 1]] for i in range(len(offs) - 1)]
    for v in views[:64]:
        ctx.compute(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v in views:
        ctx.compute(v)
    loop_ms = (time.perf_counter() - t0) * 1e3
    ctx.close()
    # every point is read twice (Step 1, then Steps 2-3): 32 bytes a point
    alg = 32.0 * float(offs[-1])
    achieved = alg / (dev_ms * 1e-3) / 1e9
    # the HBM bytes all kernels of one call move, from the counters
    traffic = measured_traffic("batch_tiled")
    traffic_frac = None if traffic is None else round(traffic / (dev_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    return {"workload": "4096 sets, sizes log-uniform 64..200000, 4 distributions",
            "engine": "tiled (batch_engine=0)",
            "n_points": int(offs[-1]), "n_hull": int(st.n_hull), "reps": reps,
            "ms_median": round(ms, 3), "ms_device": round(dev_ms, 3),
            "Mpoints_per_s": round(offs[-1] / (ms * 1e-3) / 1e6, 1),
            "sets_on_host_path": int(st.n_candidates),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                         "traffic_frac": traffic_frac,
                         "basis": "32 B per point (two reads of the input) over the device time of a call; "
                                  "traffic_frac: the counted bytes of all kernels of a call over the same time"},
            "persistent_engine": {"ms_median": round(ms_p, 3), "ms_device": round(dev_p, 3),
                                  "Mpoints_per_s": round(offs[-1] / (ms_p * 1e-3) / 1e6, 1)},
            "per_set_loop": {"ms": round(loop_ms, 2),
                             "Mpoints_per_s": round(offs[-1] / (loop_ms * 1e-3) / 1e6, 1)}}


def profiled_pass(hx, names, host, dev, reps: int, warmup: int, **kw):
    """Per-kernel device times from a pass with one HIP event per stage
    (outside any timed region; the events cost the stream a little), and each
    kernel's algorithmic bytes for the sizes of that call."""
    import numpy as np
    pctx = hx.Hull2D(profile=1, **kw)
    for _ in range(max(1, warmup)):
        for d in dev:
            pctx.compute(d)
    stage_ms = {nm: {k: [] for k in KERNEL_STAGES + ["d2h", "host_scan"]} for nm in names}
    pstats = {}
    for _ in range(max(3, reps)):
        for nm, d in zip(names, dev):
            pctx.compute(d)
            pstats[nm] = pctx.last_stats
            for k in stage_ms[nm]:
                stage_ms[nm][k].append(pstats[nm].ms_stage[k])
    pctx.close()
    full = bool(kw.get("full_sort") or kw.get("round2_chunk", 0) != 0)
    kern = {}
    for k in KERNEL_STAGES:
        ms_sum, bytes_sum = 0.0, 0.0
        for nm, a in zip(names, host):
            st = pstats[nm]
            ms_sum += float(np.mean(stage_ms[nm][k]))
            bytes_sum += kernel_bytes(k, a.shape[0], st.n_sorted, st.n_candidates,
                                      st.n_round2 - 1, full)
        kern[k] = {"ms": ms_sum / len(names), "bytes": bytes_sum / len(names)}
    # filter + sort segment (Steps 1-7): the kernels that ran, their
    # algorithmic bytes (what those kernels must move), and the bytes of the
    # method's own formula for comparison
    seg_ms, seg_bytes, formula = 0.0, 0.0, 0.0
    for nm, a in zip(names, host):
        st = pstats[nm]
        n = a.shape[0]
        for k in KERNEL_STAGES:
            ms = float(np.mean(stage_ms[nm][k]))
            seg_ms += ms
            if ms > 0.0:
                seg_bytes += kernel_bytes(k, n, st.n_sorted, st.n_candidates, st.n_round2 - 1, full)
        formula += 32.0 * n + 80.0 * st.n_round1 + 20.0 * st.n_round2
    seg = {"ms_per_hull": round(seg_ms / len(names), 4),
           "bytes_run_per_hull": round(seg_bytes / len(names)),
           "GBps_run": round(seg_bytes / (seg_ms * 1e-3) / 1e9, 1),
           "frac_of_peak": round(seg_bytes / (seg_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "bytes_formula_per_hull": round(formula / len(names)),
           "GBps_formula": round(formula / (seg_ms * 1e-3) / 1e9, 1),
           "formula": "32n + 80*round1 + 20*round2 (every survivor written, sorted, walked)"}
    return kern, pstats, stage_ms, seg


def dominant(kern, ms_override=None):
    """The kernel with the longest average duration, and its roofline."""
    dom = max(KERNEL_STAGES, key=lambda k: kern[k]["ms"])
    dom_ms = kern[dom]["ms"] if ms_override is None or dom not in ms_override else ms_override[dom]
    achieved = kern[dom]["bytes"] / (dom_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(dom), "algorithmic_bytes": round(kern[dom]["bytes"]),
            "ms_per_launch": round(dom_ms, 4),
            "ms_from": "timed region" if ms_override and dom in ms_override else "profiled pass"}


def timed_sets(hx, names, dev, steps: int, warmup: int, **kw):
    """Median wall time of hull2d_compute per set and the last call's stats."""
    import numpy as np
    import torch
    ctx = hx.Hull2D(**kw)
    for _ in range(max(1, warmup)):
        for d in dev:
            ctx.compute(d)
    torch.cuda.synchronize()
    out = {}
    for nm, d in zip(names, dev):
        ts = []
        for _ in range(max(1, steps)):
            t0 = time.perf_counter()
            ctx.compute(d)
            ts.append(time.perf_counter() - t0)
        st = ctx.last_stats
        ms = float(np.median(ts)) * 1e3
        n = int(d.shape[0])
        out[nm] = {"n": n, "h": int(st.n_hull), "ms_median": round(ms, 4),
                   "Mpoints_per_s": round(n / (ms * 1e-3) / 1e6, 1),
                   "survivors_round1": round(st.n_round1 / n, 5),
                   "survivors_round2": round(st.n_round2 / n, 7),
                   "sorted_for_round2": int(st.n_candidates),
                   "ms_host_scan": round(float(st.ms_stage["host_scan"]), 4)}
    ctx.close()
    return out


def progress(msg: str):
    """A line on stderr after each leg (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--round2-chunk", type=int, default=0)
    ap.add_argument("--full-sort", action="store_true",
                    help="sort every round-1 survivor (Step 4 as printed)")
    ap.add_argument("--no-full-sort-line", action="store_true",
                    help="skip the extra timing of the full-sort mode")
    ap.add_argument("--cpu-reps", type=int, default=1,
                    help="oracle runs per 20M set for cpu_baseline (median)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-filter comparison on the 20M mixture")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the timing of the batched form (4096 sets)")
    ap.add_argument("--no-four-region", action="store_true",
                    help="skip the four-region variant (Section 5.1) on the 20M sets")
    ap.add_argument("--no-adversarial", action="store_true",
                    help="skip the adversarial workloads (annulus + 2^20-gon, integer grid)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 320 MB device buffer three times (reference for HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the hull path has no multi-GPU form "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        src = torch.empty(40_000_000, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 8}), flush=True)
        return

    import paper_1508_05931_amd as hx
    import synth

    names = ["square_20M", "disk_20M"]
    host = [synth.workload(nm) for nm in names]
    dev = [torch.from_numpy(a).cuda() for a in host]
    torch.cuda.synchronize()
    full = bool(args.full_sort or args.round2_chunk != 0)
    mode = dict(round2_chunk=args.round2_chunk, full_sort=args.full_sort)
    kern, pstats, stage_ms, seg = profiled_pass(hx, names, host, dev, args.steps // 4, args.warmup,
                                                **mode)

    # The timed region: events only around Step 1 and Steps 2-3, the two
    # streaming passes over the input (the dominant kernel is one of them).
    ctx = hx.Hull2D(profile=2, **mode)
    for _ in range(args.warmup):
        for d in dev:
            ctx.compute(d)
    per_set = {nm: {"ms": [], "stats": None, "extremes": [], "filter1": []} for nm in names}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for nm, d in zip(names, dev):
            ctx.compute(d)
            st = ctx.last_stats
            per_set[nm]["ms"].append(st.ms_total)
            per_set[nm]["stats"] = st
            per_set[nm]["extremes"].append(st.ms_stage["extremes"])
            per_set[nm]["filter1"].append(st.ms_stage["filter1"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.close()

    n_total = sum(a.shape[0] for a in host)
    ms_per_step = elapsed * 1e3 / args.steps
    value = n_total / (ms_per_step * 1e-3) / 1e6
    timed = {k: float(np.mean([np.mean(per_set[nm][k]) for nm in names]))
             for k in ("extremes", "filter1")}
    roof = dominant(kern, timed)
    progress(f"timed region done: {value:.0f} Mpoints/s")

    sets_out = {}
    for nm, a in zip(names, host):
        st = per_set[nm]["stats"]
        n = a.shape[0]
        sets_out[nm] = {
            "n": n, "h": st.n_hull,
            "ms_median": round(float(np.median(per_set[nm]["ms"])), 4),
            "Mpoints_per_s": round(n / (float(np.median(per_set[nm]["ms"])) * 1e-3) / 1e6, 1),
            "survivors_round1": round(st.n_round1 / n, 5),
            "survivors_round2": round(st.n_round2 / n, 7),
            "sorted_for_round2": st.n_candidates,
            "ms_filter_sort": round(sum(float(np.mean(stage_ms[nm][k])) for k in KERNEL_STAGES), 4),
            "ms_d2h": round(float(np.mean(stage_ms[nm]["d2h"])), 4),
            "ms_host_scan": round(float(np.mean(stage_ms[nm]["host_scan"])), 4),
        }

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / (n_total / (PAPER_MS_SQUARE_DISK_20M * 1e-3) / 1e6), 1),
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "square_20M + disk_20M (one hull each per step)",
                   "n_per_set": int(host[0].shape[0]),
                   "round2": "single walk per region" if args.round2_chunk == 0
                   else f"subsets ({args.round2_chunk})",
                   "sort": "every round-1 survivor" if full else
                   "candidates of the bucketed filter"},
        "roofline": roof,
        "filter_sort": seg,
        "kernels_ms": {k: round(v["ms"], 4) for k, v in kern.items()},
        "sets": sets_out,
    }
    if not full and not args.no_full_sort_line:
        # the paper's Step 4 as printed: every round-1 survivor sorted; its
        # own per-kernel breakdown, roofline and segment figures
        fk, _, _, fseg = profiled_pass(hx, names, host, dev, args.steps // 4, 1, full_sort=True)
        fctx = hx.Hull2D(full_sort=True)
        for d in dev:
            fctx.compute(d)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        reps = max(1, args.steps // 4)
        for _ in range(reps):
            for d in dev:
                fctx.compute(d)
        torch.cuda.synchronize()
        fms = (time.perf_counter() - t1) * 1e3 / reps
        fctx.close()
        out["full_sort"] = {"ms_per_step": round(fms, 4),
                            "Mpoints_per_s": round(n_total / (fms * 1e-3) / 1e6, 1),
                            "roofline": dominant(fk), "filter_sort": fseg,
                            "kernels_ms": {k: round(v["ms"], 4) for k, v in fk.items()}}
        progress("full-sort leg done")
    if not args.no_four_region:
        # the paper's comparison method (Section 5.1, Table 8) on the same sets
        fr = timed_sets(hx, names, dev, max(3, args.steps // 2), 1, method=1)
        fr_ms = sum(v["ms_median"] for v in fr.values())
        out["four_region"] = {"ms_per_step": round(fr_ms, 4),
                              "Mpoints_per_s": round(n_total / (fr_ms * 1e-3) / 1e6, 1),
                              "sets": fr}
        progress("four-region leg done")
    if not args.no_adversarial:
        # the all-extreme limitation the paper discusses (Section 5.3) and
        # exact ties: 10M annulus points + 10M vertices of a 2^20-gon, and a
        # 500 x 500 integer grid with every cell four times
        adv_names = ["annulus_ngon_20M", "grid_500x4"]
        adv_dev = [torch.from_numpy(synth.workload(nm)).cuda() for nm in adv_names]
        adv = timed_sets(hx, adv_names, adv_dev, max(3, args.steps // 4), 1)
        # the annulus is where the sort and round 2 see ~10M points
        ak, _, _, aseg = profiled_pass(hx, adv_names[:1], adv_dev[:1], adv_dev[:1], 1, 1)
        adv["annulus_ngon_20M"].update({"roofline": dominant(ak), "filter_sort": aseg,
                                        "kernels_ms": {k: round(v["ms"], 4) for k, v in ak.items()}})
        out["adversarial"] = adv
        progress("adversarial leg done")
        del adv_dev
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = batched(args.steps)
        progress("batched leg done")
    if not args.no_learned:
        out["learned_filter"] = learned(args.steps)
        progress("learned leg done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(host, names, args.cpu_reps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
