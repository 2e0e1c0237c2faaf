"""Writes tests/golden/hulls.json: the oracle's canonical hull of every named
workload (size, vertex count, SHA-256 of the int32 index list, and the first
indices).  Calls only the seeded generators and the oracle.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def digest(idx: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(idx, dtype="<i4").tobytes()).hexdigest()


def main(names=None):
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hulls.json")
    data = {}
    if os.path.exists(out_path):
        with open(out_path) as f:
            data = json.load(f)
    for name in names or sorted(synth.WORKLOADS):
        t = time.time()
        pts = synth.workload(name)
        h = oracle.hull(pts)
        data[name] = {
            "n": int(pts.shape[0]),
            "input_hash": synth.content_hash(pts),
            "h": int(h.shape[0]),
            "sha256": digest(h),
            "head": h[:16].tolist(),
        }
        print(f"{name}: n={pts.shape[0]} h={h.shape[0]} ({time.time() - t:.1f} s)", flush=True)
    with open(out_path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or None)
