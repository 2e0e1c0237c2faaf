"""Autotuner of the batched form's schedule (off the timed path).

    python -m paper_1508_05931_amd.autotune [--sets 4096] [--reps 5] [--out PATH]

Times hull2d_batch on the batch workload (the 4096 sets of synth.batch:
sizes log-uniform in [64, 200000], square, disk, Gaussian and thin-annulus
sets) for every schedule the library offers: workgroups per compute unit
of the persistent launch (1 or 2) times the order in which workgroups take
the sets (0 by size class, largest first; 1 by exact size, largest first;
2 input order), each as a captured graph.  Every schedule must give the
same hulls as the first; the fastest (median of `reps` timed calls after
two warm-up calls) goes to tuning/batch.json, which Hull2D reads as its
default schedule.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CANDIDATES = [(b, o) for b in (1, 2) for o in (0, 1, 2)]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "batch.json"))
    args = ap.parse_args(argv)
    import torch
    import paper_1508_05931_amd as hx
    import synth

    pts, offs, _ = synth.batch(args.sets)
    d = torch.from_numpy(pts).cuda()
    ref = None
    timings = {}
    for b, o in CANDIDATES:
        c = hx.Hull2D(batch_blocks_per_cu=b, batch_order=o, batch_graph=True)
        for _ in range(2):
            h, oo = c.batch(d, offs)
        if ref is None:
            ref = (h.copy(), oo.copy())
        elif not (np.array_equal(h, ref[0]) and np.array_equal(oo, ref[1])):
            raise SystemExit(f"schedule blocks={b} order={o} changed the hulls")
        ts = []
        for _ in range(args.reps):
            t0 = time.perf_counter()
            c.batch(d, offs)
            ts.append(time.perf_counter() - t0)
        c.close()
        timings[f"blocks{b}_order{o}"] = round(float(np.median(ts)) * 1e3, 3)
        print(f"blocks per CU {b}, order {o}: {timings[f'blocks{b}_order{o}']:.3f} ms", flush=True)
    best = min(CANDIDATES, key=lambda bo: timings[f"blocks{bo[0]}_order{bo[1]}"])
    out = {"batch_blocks_per_cu": best[0], "batch_order": best[1],
           "workload": f"synth.batch({args.sets}): {int(offs[-1])} points",
           "ms_median_per_call": timings, "reps": args.reps,
           "device": torch.cuda.get_device_name(0)}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
