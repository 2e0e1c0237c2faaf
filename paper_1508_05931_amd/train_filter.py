"""Training of the learned first-round filter (off the timed path).

    python -m paper_1508_05931_amd.train_filter --out DIR

Data: 10,000 sets of 65,536 points from the anisotropic Gaussian mixture
generator (set i from stream (1000 + i, 2)), the shape where the axis
quadrilateral is weakest.  For each set the library computes the network
input (hull2d_histogram) and the exact hull (hull2d_batch); the label is 16
directions read off the hull: 16 hull vertices chosen to enclose a large
area (evenly spaced along the perimeter, then each moved to the vertex
farthest from the chord of its neighbours), and for each the bisector of its
two edge normals (the middle of the directions in which it is extreme),
sorted by angle.  Training runs on the device (hull2d_train_step: float32
forward and backward passes, Adam); inference uses bfloat16 weights.

Writes DIR/filter16.f32 (HULL2D_MLP_PARAMS little-endian float32 values, the
layout hull2d_load_weights reads) and DIR/filter16.json (shapes, recipe,
losses and a held-out comparison of first-round survivors against the
quadrilateral and against 16 evenly spaced directions).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_IN, N_H, N_OUT, K = 1024, 256, 32, 16


def label_directions(hv: np.ndarray) -> np.ndarray:
    """16 unit directions (float32 [32], sorted by angle) from the hull's
    vertex coordinates hv [h, 2] (counter-clockwise)."""
    h = hv.shape[0]
    if h == 0:
        ang = np.linspace(-math.pi, math.pi, K, endpoint=False) + math.pi / K
        return np.stack([np.cos(ang), np.sin(ang)], 1).astype(np.float32).ravel()
    if h < 3:
        hv = np.concatenate([hv, hv[::-1]])[:max(h, 2)]
        h = hv.shape[0]
    nxt = np.roll(hv, -1, axis=0)
    prv = np.roll(hv, 1, axis=0)
    # outward normals of the edges (v -> next) and (prev -> v) of a CCW polygon
    e1 = nxt - hv
    e0 = hv - prv
    n1 = np.stack([e1[:, 1], -e1[:, 0]], 1)
    n0 = np.stack([e0[:, 1], -e0[:, 0]], 1)
    n1 /= np.maximum(np.linalg.norm(n1, axis=1, keepdims=True), 1e-300)
    n0 /= np.maximum(np.linalg.norm(n0, axis=1, keepdims=True), 1e-300)
    bis = n0 + n1
    bis /= np.maximum(np.linalg.norm(bis, axis=1, keepdims=True), 1e-300)
    if h <= K:
        pick = np.arange(K) % h
    else:
        per = np.linalg.norm(e1, axis=1)
        cum = np.concatenate([[0.0], np.cumsum(per)])[:-1]
        tot = per.sum()
        pick = np.searchsorted(cum, np.arange(K) * tot / K, side="right") - 1
        pick = np.unique(np.clip(pick, 0, h - 1))
        while pick.size < K:  # pad with the largest gaps' midpoints
            gaps = np.diff(np.concatenate([pick, [pick[0] + h]]))
            g = int(np.argmax(gaps))
            pick = np.unique(np.append(pick, (pick[g] + gaps[g] // 2) % h))
        for _ in range(3):
            for j in range(K):
                a, b = pick[j - 1], pick[(j + 1) % K]
                lo, hi = (a + 1), (b if b > a else b + h)
                cand = np.arange(lo, hi) % h
                if cand.size == 0:
                    continue
                pa, pb = hv[a], hv[b]
                d = (pb[0] - pa[0]) * (hv[cand, 1] - pa[1]) - (pb[1] - pa[1]) * (hv[cand, 0] - pa[0])
                pick[j] = cand[int(np.argmax(d))]
            pick = np.sort(pick)
    u = bis[pick]
    order = np.argsort(np.arctan2(u[:, 1], u[:, 0]), kind="stable")
    return u[order].astype(np.float32).ravel()


def init_params(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    W1 = rng.normal(scale=math.sqrt(2.0 / N_IN), size=(N_H, N_IN))
    W2 = rng.normal(scale=math.sqrt(2.0 / N_H), size=(N_H, N_H))
    W3 = rng.normal(scale=0.01, size=(N_OUT, N_H))
    ang = np.linspace(-math.pi, math.pi, K, endpoint=False) + math.pi / K
    b3 = np.stack([np.cos(ang), np.sin(ang)], 1).ravel()
    # untrained, the network proposes 16 evenly spaced directions
    return np.concatenate([W1.ravel(), np.zeros(N_H), W2.ravel(), np.zeros(N_H), W3.ravel(),
                           b3]).astype(np.float32)


def make_data(ctx, first: int, count: int, n: int, chunk: int = 256):
    """Histograms [count, 1024] (device) and labels [count, 32] for sets
    first .. first + count - 1."""
    import torch
    import synth
    X = torch.empty((count, N_IN), dtype=torch.float32, device="cuda")
    T = np.empty((count, N_OUT), dtype=np.float32)
    for c0 in range(0, count, chunk):
        m = min(chunk, count - c0)
        pts = np.empty((m * n, 2), dtype=np.float64)
        for j in range(m):
            pts[j * n:(j + 1) * n] = synth.mixture(n, (first + c0 + j, 2))
        d = torch.from_numpy(pts).cuda()
        offs = np.arange(m + 1, dtype=np.int64) * n
        hulls, hoffs = ctx.batch(d, offs)
        for j in range(m):
            X[c0 + j] = ctx.histogram(d[j * n:(j + 1) * n])
            hv = pts[j * n + hulls[hoffs[j]:hoffs[j + 1]]]
            T[c0 + j] = label_directions(hv)
    return X, torch.from_numpy(T).cuda()


def survivors(hx, ctx_q, ctx_l, ctx_u, first: int, count: int, n: int):
    """First-round survivors of held-out sets: quadrilateral, learned, and
    16 evenly spaced directions (a network with zero weights)."""
    import torch
    import synth
    out = {"quad": [], "learned": [], "uniform": []}
    for i in range(count):
        d = torch.from_numpy(synth.mixture(n, (first + i, 2))).cuda()
        for key, c in (("quad", ctx_q), ("learned", ctx_l), ("uniform", ctx_u)):
            c.compute(d)
            out[key].append(c.last_stats.n_round1)
    return {k: float(np.mean(v)) for k, v in out.items()}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--sets", type=int, default=10_000)
    ap.add_argument("--points", type=int, default=65_536)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=17)
    ap.add_argument("--eval-sets", type=int, default=200)
    args = ap.parse_args(argv)
    import torch
    import paper_1508_05931_amd as hx

    t0 = time.time()
    ctx = hx.Hull2D()
    p0 = init_params(args.seed)
    ctx.set_weights(p0)
    X, T = make_data(ctx, 1000, args.sets, args.points)
    print(f"data: {args.sets} sets in {time.time() - t0:.1f} s", flush=True)
    rng = np.random.default_rng(args.seed)
    losses = []
    for ep in range(args.epochs):
        perm = torch.from_numpy(rng.permutation(args.sets)).cuda()
        tot, nb = 0.0, 0
        for b0 in range(0, args.sets - args.batch + 1, args.batch):
            idx = perm[b0:b0 + args.batch]
            loss, _ = ctx.train_step(X[idx], T[idx], lr=args.lr)
            tot += loss
            nb += 1
        losses.append(tot / max(nb, 1))
        print(f"epoch {ep}: loss {losses[-1]:.5f}", flush=True)
    params = ctx.get_weights()
    os.makedirs(args.out, exist_ok=True)
    wpath = os.path.join(args.out, "filter16.f32")
    params.astype("<f4").tofile(wpath)

    ctx_q = hx.Hull2D(profile=False)
    ctx_l = hx.Hull2D(learned=True, weights=params)
    zero = init_params(args.seed)
    zero[:-N_OUT] = 0.0
    ctx_u = hx.Hull2D(learned=True, weights=zero)
    ev = survivors(hx, ctx_q, ctx_l, ctx_u, 2000, args.eval_sets, args.points)
    meta = {
        "format": "HULL2D_MLP_PARAMS little-endian float32: W1[256][1024] b1[256] W2[256][256] "
                  "b2[256] W3[32][256] b3[32]",
        "shapes": {"in": N_IN, "hidden": [N_H, N_H], "out": N_OUT, "directions": K},
        "histogram": "32x32 occupancy of the sample (all points when n <= 4096, else 16 blocks "
                     "of 256 consecutive points starting at floor(b*n/16)) over its bounding box, "
                     "count*1024/sample_size, cell = cy*32+cx",
        "train_sets": f"{args.sets} mixture sets of {args.points} points, streams (1000+i, 2)",
        "eval_sets": f"{args.eval_sets} mixture sets of {args.points} points, streams (2000+i, 2)",
        "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "seed": args.seed,
        "loss_first_epoch": losses[0] if losses else None,
        "loss_last_epoch": losses[-1] if losses else None,
        "mean_round1_survivors": ev,
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(args.out, "filter16.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
