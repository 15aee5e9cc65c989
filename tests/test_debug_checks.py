"""The debug mode's binning invariants (sixdgs_debug_check_bins), run on host
arrays without a GPU: a consistent binning passes, and each planted mistake
(an index, an order, a count or a work item) is reported."""
import numpy as np
import pytest

from paper_2410_04974_amd import _lib as L


def _binning(seed=0, E=60, T=96, chunk=4, ties=True):
    """A consistent binning built directly from its definition: each entry
    touches a random set of tiles; pairs sorted by (tile, depth, entry); the
    tiles ordered by the bit length of their runs; chunk counts at most
    ceil(run / chunk); the work items listed in that order."""
    rng = np.random.default_rng(seed)
    depth = rng.uniform(0.5, 5.0, E).astype(np.float32)
    if ties:
        depth[1::7] = depth[0]  # equal depths: ties go by entry id
    tiles = np.zeros(E, np.uint32)
    pairs = []
    for e in range(E):
        if rng.random() < 0.2:
            continue  # not binned
        ts = rng.choice(T, size=rng.integers(1, 6), replace=False)
        tiles[e] = len(ts)
        pairs += [(int(t), float(depth[e]), e) for t in ts]
    pairs.sort()
    keys = np.array([p[0] for p in pairs], np.uint32)
    vals = np.array([p[2] for p in pairs], np.uint32)
    ranges = np.zeros((T, 2), np.uint32)
    for t in range(T):
        idx = np.nonzero(keys == t)[0]
        if len(idx):
            ranges[t] = (idx[0], idx[-1] + 1)
    run = ranges[:, 1] - ranges[:, 0]
    bits = np.array([int(r).bit_length() for r in run])
    order = np.argsort(-bits, kind="stable").astype(np.uint32)
    nch = np.array([rng.integers(0, -(-int(r) // chunk) + 1) for r in run], np.uint32)
    items = np.array([(t, c) for t in order for c in range(nch[t])], np.uint32).reshape(-1, 2)
    return dict(tiles=tiles, depth=depth, keys=keys, values=vals, ranges=ranges, order=order, chunk=chunk, nch=nch,
                items=items)


def _check(b):
    return L.check_bins(**b)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_consistent_binning_passes(seed):
    b = _binning(seed)
    assert _check(b) == (L.OK, "")
    # also without the work items, without the order, and with the items in any order
    assert _check(dict(b, nch=None, items=None))[0] == L.OK
    assert _check(dict(b, order=None, nch=None, items=None))[0] == L.OK
    perm = np.random.default_rng(seed).permutation(len(b["items"]))
    assert _check(dict(b, items=b["items"][perm], order=None))[0] == L.OK


def _first_tile_with(b, at_least):
    run = b["ranges"][:, 1] - b["ranges"][:, 0]
    return int(np.nonzero(run >= at_least)[0][0])


def _plant(b, what):
    b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in b.items()}
    if what == "depth order":
        t = _first_tile_with(b, 2)
        s = b["ranges"][t, 0]
        v = b["values"]
        # make the first two entries of the tile strictly out of depth order
        b["depth"][v[s]] = b["depth"][v[s + 1]] + 1.0
    elif what == "tie order":
        t = _first_tile_with(b, 2)
        s = b["ranges"][t, 0]
        v = b["values"]
        b["depth"][v[s]] = b["depth"][v[s + 1]]
        v[s], v[s + 1] = max(v[s], v[s + 1]), min(v[s], v[s + 1])
    elif what == "tile count":
        e = int(np.nonzero(b["tiles"])[0][0])
        b["tiles"][e] += 1
    elif what == "entry id":
        b["values"][3] = len(b["tiles"])
    elif what == "tile id":
        b["keys"][-1] = len(b["ranges"])
    elif what == "tile order":
        i = len(b["keys"]) // 2
        b["keys"][i], b["keys"][i + 1] = b["keys"][i] + 1, b["keys"][i]
    elif what == "multiplicity":
        # one entry's count one lower, another's one higher: the same total
        e1, e2 = np.nonzero(b["tiles"])[0][:2]
        b["tiles"][e1] -= 1
        b["tiles"][e2] += 1
    elif what == "range end":
        t = _first_tile_with(b, 1)
        b["ranges"][t, 1] += 1
    elif what == "range start":
        t = _first_tile_with(b, 2)
        b["ranges"][t, 0] += 1
    elif what == "empty range":
        t = int(np.nonzero(b["ranges"][:, 1] == b["ranges"][:, 0])[0][0])
        b["ranges"][t] = (5, 5)
    elif what == "order duplicate":
        b["order"][1] = b["order"][0]
    elif what == "order weight":
        b["order"][0], b["order"][-1] = b["order"][-1], b["order"][0]
    elif what == "chunk count":
        t = _first_tile_with(b, 1)
        run = int(b["ranges"][t, 1] - b["ranges"][t, 0])
        b["nch"][t] = -(-run // b["chunk"]) + 1
    elif what == "item count":
        b["items"] = b["items"][:-1]
    elif what == "item":
        b["items"][len(b["items"]) // 2, 1] += 1
    elif what == "item twice":
        b["items"][1] = b["items"][0]
    elif what == "item tile":
        b["items"][0, 0] = len(b["ranges"])
    return b


# each planted mistake and a word of the message of the check that must catch it
PLANTS = {"depth order": "order", "tie order": "order", "tile count": "sum to", "entry id": "entry id",
          "tile id": "tile id", "tile order": "tile id", "multiplicity": "appears in", "range end": "range",
          "range start": "range", "empty range": "no pairs", "order duplicate": "twice",
          "order weight": "longer list", "chunk count": "chunks for a run", "item count": "work items",
          "item": "work item", "item twice": "twice", "item tile": "out of range"}


@pytest.mark.parametrize("what", list(PLANTS))
def test_planted_mistake_is_reported(what):
    b = _binning(3)
    assert _check(b)[0] == L.OK
    rc, msg = _check(_plant(b, what))
    assert rc == L.ERR_DEBUG, what
    assert PLANTS[what] in msg, (what, msg)


def test_inconsistent_state_is_an_argument_error():
    b = L.BinState()
    b.E, b.P, b.T = 4, 0, 0
    assert L.lib().sixdgs_debug_check_bins(b, None, 0) == L.ERR_INVALID_ARG  # NULL tiles with E > 0
    assert L.lib().sixdgs_debug_check_bins(None, None, 0) == L.ERR_INVALID_ARG
    empty = L.BinState()
    assert L.lib().sixdgs_debug_check_bins(empty, None, 0) == L.OK  # nothing binned
