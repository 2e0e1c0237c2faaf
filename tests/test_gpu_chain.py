"""GPU parity of the four-region variant (Section 5.1, Table 8's comparison
method; options.method = 1) against the oracle's model of it
(oracle.chain): the first-round count, the survivors per region, every
region's kept points in walking order, m2 and the canonical hull; plus the
full-size workloads against the oracle-written golden hashes."""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "hulls.json")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    import paper_1508_05931_amd as hx
    return hx.Hull2D(method=1)


def to_dev(torch, pts):
    return torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).cuda()


def _cases():
    t = np.arange(-700, 800, dtype=np.float64)
    near = synth.square(4000, (75, 1))
    near[::3] = near[0]  # 1334 copies of one point
    return {
        "square_100k": synth.square(100_000, (1, 1)),
        "square_100003": synth.square(100_003, (51, 1)),
        "disk_100k": synth.disk(100_000, (52, 1)),
        "gauss_50k": synth.gaussian(50_000, 1.0, (53, 1)),
        "mixture_100k": synth.mixture(100_000, (54, 1)),
        "annulus_ngon_100k": synth.annulus_ngon(50_000, 50_000, 14, ((55, 1), (56, 1), (57, 1))),
        "grid_draws_100k": synth.grid_draws(100_000, 64, (58, 1)),
        "grid_200x3": synth.grid(200, 3, (59, 1)),
        "ngon_4096": synth.ngon(4096, 12, (60, 1)),
        "annulus_300k": synth.annulus(300_000, 0.9999, (76, 1)),
        "collinear_1500": np.stack([t, 2 * t - 5], axis=1)[np.random.default_rng(1).permutation(1500)],
        "collinear_dups": np.repeat(np.stack([t[:40], -t[:40]], axis=1), 3, axis=0),
        "dup_heavy": np.concatenate([np.full((5000, 2), 0.25), synth.square(3000, (65, 1)),
                                     np.full((3000, 2), 1.0)])[np.random.default_rng(3).permutation(11_000)],
        "repeats_in_a_region": near,
        "all_equal_1000": np.full((1000, 2), 0.375),
        "one": np.array([[0.25, -0.5]]),
        "two": np.array([[1.0, 3.0], [-1.0, 2.0]]),
        "three_collinear": np.array([[0.0, 0.0], [2.0, 2.0], [1.0, 1.0]]),
        "triangle_interior": np.array([[0.0, 0.0], [4.0, 0.0], [0.0, 4.0], [1.0, 1.0], [-0.0, 0.0]]),
        "tiny_magnitudes": (1.0 + synth.square(5000, (61, 1))) * math.ldexp(1.0, -290),
        "huge_magnitudes": (synth.disk(5000, (62, 1)) - 0.5) * math.ldexp(1.0, 290),
    }


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_chain_equals_oracle(torch_dev, ctx, name):
    pts = CASES[name]
    say(f"four-region {name} n={len(pts)}")
    got = ctx.compute(to_dev(torch_dev, pts))
    want = oracle.chain(pts)
    assert got.tolist() == want["hull"].tolist()
    assert got.tolist() == oracle.hull(pts).tolist()
    info = ctx.chain_info()
    assert info["m1"] == want["m1"]
    assert info["n_region"] == want["n_region"]
    for k in range(4):
        assert info["kept"][k].tolist() == want["kept"][k].tolist(), k
    assert info["m2"] == want["m2"]
    st = ctx.last_stats
    assert st.n_round1 == want["m1"] and st.n_hull == len(want["hull"])
    assert st.n_candidates >= sum(len(k) for k in want["kept"])


def test_chain_many_repeats_in_one_bucket(torch_dev, ctx):
    """Over 4096 candidates in one bucket (repeats of a point beyond the
    quadrilateral): taken in rounds of the smallest remaining ones."""
    base = synth.disk(20_000, (77, 1))
    far = np.array([[-0.75, -0.75]])
    pts = np.concatenate([base, np.repeat(far, 9000, axis=0), base[:100] * 1.001])
    pts = pts[np.random.default_rng(4).permutation(len(pts))]
    got = ctx.compute(to_dev(torch_dev, pts))
    want = oracle.chain(pts)
    assert got.tolist() == want["hull"].tolist()
    info = ctx.chain_info()
    for k in range(4):
        assert info["kept"][k].tolist() == want["kept"][k].tolist()
    assert max(info["n_cand"]) > 9000


def test_chain_domain_errors(torch_dev, ctx):
    import paper_1508_05931_amd as hx
    pts = synth.square(10_000, (78, 1))
    pts[17, 0] = float("nan")
    with pytest.raises(hx.HullError) as e:
        ctx.compute(to_dev(torch_dev, pts))
    assert e.value.status == hx.NONFINITE
    ok = synth.square(1000, (79, 1))
    assert ctx.compute(to_dev(torch_dev, ok)).tolist() == oracle.hull(ok).tolist()


@pytest.mark.parametrize("name", ["square_20M", "disk_20M", "mixture_20M", "grid_500x4"])
def test_chain_full_size_matches_golden(torch_dev, ctx, name):
    with open(GOLDEN) as f:
        g = json.load(f)[name]
    say(f"four-region full size {name}")
    pts = synth.workload(name)
    assert synth.content_hash(pts) == g["input_hash"]
    got = ctx.compute(to_dev(torch_dev, pts))
    assert len(got) == g["h"]
    assert hashlib.sha256(np.ascontiguousarray(got, dtype="<i4").tobytes()).hexdigest() == g["sha256"]
    st = ctx.last_stats
    say(f"  round1={st.n_round1} candidates={st.n_candidates} kept+corners={st.n_round2} h={st.n_hull}")
