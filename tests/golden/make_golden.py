"""Writes tests/golden/hulls.json: the oracle's canonical hull of every named
workload (size, vertex count, SHA-256 of the int32 index list, and the first
indices), and tests/golden/batch.json: the oracle's hulls of the 4096-set
batch (set-local indices concatenated in set order, and the output offsets).
Calls only the seeded generators and the oracle.

    python tests/golden/make_golden.py            # every single workload
    python tests/golden/make_golden.py batch      # the batch only
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


def batch_golden():
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch.json")
    t = time.time()
    pts, offs, kinds = synth.batch(4096)
    hulls = []
    out_offs = np.zeros(len(offs), dtype=np.int64)
    for s in range(len(offs) - 1):
        h = oracle.hull(np.ascontiguousarray(pts[offs[s]:offs[s + 1]]))
        hulls.append(h)
        out_offs[s + 1] = out_offs[s] + len(h)
    allh = np.concatenate(hulls).astype(np.int32)
    data = {"batch_4096": {
        "S": int(len(offs) - 1),
        "N": int(offs[-1]),
        "input_hash": synth.content_hash(pts),
        "total": int(out_offs[-1]),
        "sha256": digest(allh),
        "offsets_sha256": hashlib.sha256(np.ascontiguousarray(out_offs, dtype="<i8").tobytes()).hexdigest(),
    }}
    with open(out_path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(f"batch_4096: N={offs[-1]} total={out_offs[-1]} ({time.time() - t:.1f} s)", flush=True)


def main(names=None):
    if names == ["batch"]:
        batch_golden()
        return
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
