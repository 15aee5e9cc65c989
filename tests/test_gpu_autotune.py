"""GPU: the tile / batch-depth / chunk autotuner picks one of its candidates,
the pick renders the default settings' image bit for bit (the image does not
depend on any of the three), and its JSON cache round-trips."""
import json

import pytest
import torch

import synth
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def test_autotune_returns_a_candidate_that_renders_the_same_image(tmp_path):
    from paper_2410_04974_amd import Renderer
    from paper_2410_04974_amd.autotune import CANDIDATES, autotune
    w = synth.workload("c3", n_override=30000)
    cams = w.cameras[:4]
    p = G.to_dev(synth.make_scene(w.scene))
    cache = str(tmp_path / "tune.json")
    cands = [c for c in CANDIDATES if c[1] in (256, 128)]  # 16x16, 32x8, 8x32 at two depths
    res = autotune(p, cams, candidates=cands, iters=2, cache=cache)
    print("autotune", {k: round(v, 3) for k, v in res["timings"].items()}, "->", res["tile"], res["batch"],
          res["chunk"], flush=True)
    assert (tuple(res["tile"]), res["batch"], res["chunk"]) in cands
    assert len(res["timings"]) == len(cands) and all(t > 0 for t in res["timings"].values())
    assert res["ms"] == min(res["timings"].values())
    ref = Renderer().forward(p, cams)
    got = Renderer(tile=res["tile"], batch=res["batch"], chunk=res["chunk"]).forward(p, cams)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    # the cache holds the pick under this device and workload, and a second call returns it untimed
    with open(cache) as f:
        data = json.load(f)
    assert len(data) == 1
    (entry,) = data.values()
    assert (tuple(entry["tile"]), entry["batch"], entry["chunk"]) == (tuple(res["tile"]), res["batch"], res["chunk"])
    again = autotune(p, cams, candidates=[], iters=1, cache=cache)
    assert (tuple(again["tile"]), again["batch"], again["chunk"]) == (tuple(res["tile"]), res["batch"], res["chunk"])
    # another workload misses the cache and is timed afresh
    other = autotune(p, cams[:2], candidates=cands[:1], iters=1, cache=cache)
    assert (tuple(other["tile"]), other["batch"], other["chunk"]) == cands[0]
    with open(cache) as f:
        assert len(json.load(f)) == 2
