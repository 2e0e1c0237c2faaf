"""Autotuner of the batched form's schedule (off the timed path).

    python -m paper_1508_05931_amd.autotune [--sets 4096] [--reps 5] [--out PATH]

Times hull2d_batch on the batch workload (the 4096 sets of synth.batch:
sizes log-uniform in [64, 200000], square, disk, Gaussian and thin-annulus
sets), each schedule as a captured graph, for both engines:

* the persistent engine (batch_engine=1): workgroups per compute unit of the
  persistent launch (1 or 2) times the order in which workgroups take the
  sets (0 by size class, largest first; 1 by exact size, largest first; 2
  input order);
* the tiled engine (batch_engine=0, the default): points per tile of the
  passes over points, the largest number of filter buckets per region
  (2^bits) of Steps 6-7, the largest number of angle buckets per region of
  the grouping before the sort, and how many of the largest sets run on the
  second stream (-1: one stream); then, at the fastest of those, the points
  each thread takes per round in the passes over points (2, 4 or 8).

Every schedule must give the same hulls as the first; the fastest of each
engine (median device time of `reps` calls after two warm-up calls, from
the library's events around the call's device work: steadier than the
wall clock) goes to tuning/batch.json, which Hull2D reads as its default
schedule.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PERSISTENT = [dict(batch_engine=1, batch_blocks_per_cu=b, batch_order=o) for b in (1, 2) for o in (0, 1, 2)]
TILE_SIZES = (4096, 8192, 16384, 32768)
FILTER_BITS = (13, 14)
SORT_BITS = (11, 12)
SIDE_SETS = (-1, 256, 384, 512)
ITEMS = (2, 4, 8)
TILED = [dict(batch_engine=0, batch_tile=t, batch_filter_bits=f, batch_sort_bits=s, batch_side_sets=g)
         for t, f, s, g in itertools.product(TILE_SIZES, FILTER_BITS, SORT_BITS, SIDE_SETS)]


def _name(kw: dict) -> str:
    return "_".join(f"{k.replace('batch_', '')}{v}" for k, v in kw.items() if k != "batch_engine")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "batch.json"))
    args = ap.parse_args(argv)
    import torch
    import paper_1508_05931_amd as hx
    import synth

    pts, offs, _ = synth.batch(args.sets)
    d = torch.from_numpy(pts).cuda()
    ref = None
    timings = {"persistent": {}, "tiled": {}}
    best = {}
    def stages():
        yield "persistent", PERSISTENT
        yield "tiled", TILED
        # points per thread, at the fastest tiled schedule so far
        yield "tiled", [dict(best["tiled"][1], batch_items=i) for i in ITEMS]

    for engine, grid in stages():
        for kw in grid:
            # every knob given, so the stored tuning does not leak into the run
            full = {k: 0 for k in hx.TUNED_KEYS}
            full.update(kw)
            c = hx.Hull2D(batch_graph=True, **full)
            for _ in range(2):
                h, oo = c.batch(d, offs)
            if ref is None:
                ref = (h.copy(), oo.copy())
            elif not (np.array_equal(h, ref[0]) and np.array_equal(oo, ref[1])):
                raise SystemExit(f"schedule {kw} changed the hulls")
            ts = []
            for _ in range(args.reps):
                c.batch(d, offs)
                ts.append(float(c.last_stats.ms_device))
            c.close()
            ms = round(float(np.median(ts)), 3)
            timings[engine][_name(kw)] = ms
            print(f"{engine} {_name(kw)}: {ms:.3f} ms", flush=True)
            if engine not in best or ms < best[engine][0]:
                best[engine] = (ms, kw)
    out = {k: v for k, v in best["persistent"][1].items() if k != "batch_engine"}
    out.update({k: v for k, v in best["tiled"][1].items() if k != "batch_engine"})
    out.update({"workload": f"synth.batch({args.sets}): {int(offs[-1])} points",
                "ms_median_per_call": timings, "reps": args.reps,
                "device": torch.cuda.get_device_name(0)})
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "ms_median_per_call"}), flush=True)


if __name__ == "__main__":
    main()
