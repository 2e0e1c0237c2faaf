"""Reference of the learned filter's network (test infrastructure only).

Plain numpy, float64 unless stated.  The network maps a 32 x 32 occupancy
histogram (1024 inputs) through two hidden layers of 256 ReLU units to 32
outputs, read as 16 direction vectors (y[2j], y[2j+1]):

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3

with W1 [256, 1024], W2 [256, 256], W3 [32, 256] (row = output unit).  The
training loss is the mean squared error over the batch and the 32 outputs.
Parameters travel as one flat float32 vector in the order
W1, b1, W2, b2, W3, b3 (row-major), the layout of the library's weights.

`forward_bf16` models the inference precision: weights and every layer input
rounded to bfloat16 (round to nearest, ties to even), products summed in
float64 here (in float32 on the device; the tests allow for the difference),
biases float32.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 1024, 256, 32
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64).ravel()
    assert flat.size == N_PARAMS, flat.size
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = flat[o:o + k].reshape(shp)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(flat, x):
    """Outputs [B, 32] and the hidden activations, in float64."""
    p = unpack(flat)
    x = np.asarray(x, dtype=np.float64).reshape(-1, N_IN)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(flat, x, t) -> float:
    y, _ = forward(flat, x)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(flat, x, t) -> np.ndarray:
    """Gradient of the mean squared error by the chain rule (flat, float64)."""
    p = unpack(flat)
    y, (x, z1, h1, z2, h2) = forward(flat, x)
    t = np.asarray(t, dtype=np.float64).reshape(y.shape)
    d3 = 2.0 * (y - t) / y.size                 # dL/dy
    g = {"W3": d3.T @ h2, "b3": d3.sum(0)}
    d2 = (d3 @ p["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return pack(g)


def bf16(a) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(flat, x):
    p = unpack(np.asarray(flat, dtype=np.float32).astype(np.float64))
    a = bf16(np.asarray(x, dtype=np.float32).reshape(-1, N_IN))
    for wn, bn, act in (("W1", "b1", True), ("W2", "b2", True), ("W3", "b3", False)):
        z = a @ bf16(p[wn]).T + p[bn]
        if act:
            a = bf16(np.maximum(z, 0.0).astype(np.float32))
        else:
            a = z
    return a


def sample_index(n: int) -> np.ndarray:
    """The histogram's sample: all points when n <= 4096, else 16 blocks of
    256 consecutive points, block b starting at floor(b * n / 16) (4096
    points whatever n; for n = 65536 every 16th block of 256)."""
    if n <= 4096:
        return np.arange(n)
    starts = [(b * n) // 16 for b in range(16)]
    return np.concatenate([np.arange(st, st + 256) for st in starts])


def histogram(xy) -> np.ndarray:
    """32 x 32 occupancy histogram (float32 [1024], cell row-major in y) of
    the sample over the sample's bounding box; a cell holds its count times
    1024 / (sample size), so the cells average 1."""
    a = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    h = np.zeros(N_IN, dtype=np.float32)
    s = sample_index(a.shape[0])
    if s.size == 0:
        return h
    p = a[s]
    lo = p.min(axis=0)
    hi = p.max(axis=0)
    w = hi - lo
    sc = np.where(w > 0, 32.0 / np.where(w > 0, w, 1.0), 0.0)
    cell = np.floor((p - lo) * sc)
    cell = np.clip(cell, 0, 31).astype(np.int64)
    cnt = np.bincount(cell[:, 1] * 32 + cell[:, 0], minlength=N_IN).astype(np.float64)
    return (cnt * (1024.0 / s.size)).astype(np.float32)
