"""Leaf-merge configurations, the captured (HIP graph) batched merge and the
autotuner: every result is compared with the CPU oracle element by element.

* each of the four leaf configurations (8 or 4 waves per tile, large or
  half-size tiles, pipeline depth 2 or 3) is forced in turn on single pairs (several tiles, ragged
  tails, division levels via IM_LEAF_TILES), key+payload pairs and batches;
* a graph is recorded once and replayed several times on new contents of the
  same buffers, with eager merges and other device work between the replays;
  every replay is checked against the oracle;
* the autotuner times the configurations on a copy (the input is unchanged),
  and the following merge of that workload class uses its choice.
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2005_12648_amd as im

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def d(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def h(t):
    return t.cpu().numpy()


@pytest.fixture
def leaf_cfg():
    def setter(c):
        im.set_config(c)
    yield setter
    im.set_config(-1)


@pytest.fixture
def leaf_tiles(monkeypatch):
    def setter(v):
        if v is None:
            monkeypatch.delenv("IM_LEAF_TILES", raising=False)
        else:
            monkeypatch.setenv("IM_LEAF_TILES", str(v))
    return setter


def check_batch(got, data, off, label):
    n = (off.size - 1) // 2
    for q in range(n):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        want = oracle.merge(data[o0:o2], int(o1 - o0))
        bad = np.flatnonzero(got[o0:o2] != want)
        assert bad.size == 0, "%s: instance %d, %d mismatches" % (label, q, bad.size)


# ------------------------------------------------------ forced configurations
@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
@pytest.mark.parametrize("tiles", [None, 3, 1])
@pytest.mark.parametrize("dt", [np.int32, np.uint64])
def test_config_pairs(dev, leaf_cfg, leaf_tiles, cfg, tiles, dt):
    leaf_cfg(cfg)
    leaf_tiles(tiles)
    for la, lb, seed in [(70001, 50007, 1), (5, 123457, 2), (200003, 3, 3), (31337, 31337, 4)]:
        data = gen.pair_uniform(la, lb, seed, dtype=dt)
        say("cfg", cfg, "tiles", tiles, dt.__name__, la, lb)
        t = d(data, dev)
        im.inplace_merge(t, la)
        st = im.fetch_stats()
        assert st["leaf_config"] == cfg
        got = h(t)
        want = oracle.merge(data, la)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, "%d mismatches, first at %d" % (bad.size, bad[0])


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
@pytest.mark.parametrize("vdt", [np.uint32, np.uint64])
def test_config_kv(dev, leaf_cfg, leaf_tiles, cfg, vdt):
    leaf_cfg(cfg)
    leaf_tiles(2)
    keys, vals = gen.pair_kv(60000, 45001, 11)
    vals = vals.astype(vdt)
    say("kv cfg", cfg, vdt.__name__)
    tk, tv = d(keys, dev), d(vals, dev)
    im.inplace_merge_kv(tk, tv, 60000)
    torch.cuda.synchronize()
    wk, wv = oracle.merge_kv(keys, vals, 60000)
    assert np.array_equal(h(tk), wk)
    assert np.array_equal(h(tv), wv)


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_config_batched(dev, leaf_cfg, cfg):
    leaf_cfg(cfg)
    data, off = gen.batch(200, 51, lo_exp=0.0, hi_exp=16.0)
    say("batched cfg", cfg, data.size)
    t = d(data, dev)
    im.batched_inplace_merge(t, d(off, dev))
    assert im.fetch_stats()["leaf_config"] == cfg
    check_batch(h(t), data, off, "cfg %d" % cfg)


# ------------------------------------------------------------ captured graph
@pytest.mark.parametrize("cfg", [-1, 1])
def test_graph_replays(dev, leaf_cfg, cfg):
    leaf_cfg(cfg)
    n = 96
    data0, off0 = gen.batch(n, 61, lo_exp=0.0, hi_exp=15.0)
    total = data0.size
    max_inst = int(np.max(off0[2::2] - off0[:-1:2]))
    buf = d(data0, dev)
    offs = d(off0, dev)
    g = im.MergeGraph(buf, offs, max_instance=max_inst)
    say("graph recorded, cooperative leaf node:", g.cooperative)
    other = d(gen.pair_uniform(40000, 30000, 62), dev)
    try:
        for r in range(4):
            # new contents each replay: the same offsets with new keys, then
            # (replay 3) new offsets with the same count and no larger sizes
            if r < 3:
                off = off0
                rng = np.random.default_rng(100 + r)
                data = rng.integers(0, 2 ** 31, size=total).astype(np.int32)
                for q in range(n):
                    data[off[2 * q]:off[2 * q + 1]].sort()
                    data[off[2 * q + 1]:off[2 * q + 2]].sort()
            else:
                rng = np.random.default_rng(200)
                sizes = (off0[1:] - off0[:-1]) // 2
                off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
                data = rng.integers(0, 50, size=total).astype(np.int32)
                for q in range(n):
                    data[off[2 * q]:off[2 * q + 1]].sort()
                    data[off[2 * q + 1]:off[2 * q + 2]].sort()
                offs.copy_(d(off, dev))
            buf.copy_(d(data, dev))
            say("replay", r)
            g.launch()
            # eager work between replays: another merge and a library op
            other_h = h(other)
            im.inplace_merge(other, 40000)
            _ = torch.sort(other.to(torch.int64)).values.sum()
            torch.cuda.synchronize()
            check_batch(h(buf), data, off, "replay %d" % r)
            assert np.array_equal(h(other), oracle.merge(other_h, 40000))
            st = im.fetch_stats()
            assert st["leaf_elems"] >= 0
    finally:
        g.close()


def test_graph_single_instance_division(dev, leaf_tiles):
    # one large instance: the captured chain holds several division levels
    leaf_tiles(2)
    la, lb = 300007, 260001
    data = gen.pair_uniform(la, lb, 71)
    off = np.array([0, la, la + lb], dtype=np.int64)
    buf, offs = d(data, dev), d(off, dev)
    g = im.MergeGraph(buf, offs)
    try:
        for r in range(3):
            x = gen.pair_uniform(la, lb, 72 + r)
            buf.copy_(d(x, dev))
            say("single-instance replay", r)
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(h(buf), oracle.merge(x, la)), r
    finally:
        g.close()


@pytest.mark.parametrize("tiles", [None, 4])
def test_graph_single_pair_cells(dev, leaf_tiles, tiles):
    # one pair in a graph is tiled by cells of the whole output, as in the
    # eager call (four-tile leaves: several division levels); replays with
    # new keys, then offsets that move the pair, shrink it, leave it in
    # order, or put all of B first
    leaf_tiles(tiles)
    la, lb = 700001, 650003
    total = la + lb
    base = gen.pair_uniform(la, lb, 91)
    buf = d(base, dev)
    offs = d(np.array([0, la, total], dtype=np.int64), dev)
    g = im.MergeGraph(buf, offs)
    try:
        cases = [(0, la, lb, "uniform"), (0, la, lb, "uniform"), (7, 400000, 900000, "uniform"),
                 (0, 3, total - 3, "uniform"), (0, la, lb, "ordered"), (11, 500000, 500000, "inverted")]
        for r, (o0, a, b, kind) in enumerate(cases):
            x = np.random.default_rng(300 + r).integers(0, 2 ** 31, size=total).astype(np.int32)
            pair = gen.pair_uniform(a, b, 310 + r)
            if kind == "ordered":
                pair = np.sort(pair)
            elif kind == "inverted":
                pair = np.concatenate([np.sort(pair)[b:], np.sort(pair)[:b]])
                a, b = pair.size - b, b
            x[o0:o0 + a + b] = pair
            offs.copy_(d(np.array([o0, o0 + a, o0 + a + b], dtype=np.int64), dev))
            buf.copy_(d(x, dev))
            say("single-pair graph replay", r, o0, a, b, kind)
            g.launch()
            torch.cuda.synchronize()
            want = x.copy()
            want[o0:o0 + a + b] = oracle.merge(pair, a)
            assert np.array_equal(h(buf), want), r
    finally:
        g.close()


# ----------------------------------------------------------------- autotune
def test_autotune_choice_is_used(dev):
    data, off = gen.batch(128, 81, lo_exp=2.0, hi_exp=14.0)
    t, to = d(data, dev), d(off, dev)
    chosen, ms = im.autotune(t, to, reps=2)
    say("autotune ms per config", ms, "chosen", chosen)
    assert 0 <= chosen < im.LEAF_CONFIGS
    assert all(m > 0 for m in ms)
    assert ms[chosen] == min(ms)
    assert np.array_equal(h(t), data)        # input untouched
    im.batched_inplace_merge(t, to)
    assert im.fetch_stats()["leaf_config"] == chosen
    check_batch(h(t), data, off, "tuned")


# ------------------------------------------------------------ leaf counters
def expected_leaves(data, off, tile, max_levels):
    """Leaves, tiles and leaf elements that the instances fix when every one
    is small enough to be a leaf at the first level: a pair with both parts
    non-empty that is out of order is one leaf of ceil(S / tile) tiles, except
    a pair with every B before every A, which is one exchange while a
    further level exists."""
    leaves = tiles = elems = 0
    for q in range((off.size - 1) // 2):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        a, b = data[o0:o1], data[o1:o2]
        if a.size == 0 or b.size == 0 or a[-1] <= b[0]:
            continue
        if a[0] > b[-1] and max_levels > 1:
            continue
        s = int(o2 - o0)
        leaves += 1
        tiles += -(-s // tile)
        elems += s
    return leaves, tiles, elems


@pytest.mark.parametrize("cfg", [0, 1])
def test_batched_leaf_counters(dev, leaf_cfg, cfg):
    # leaves are laid out in tiles as the division emits them (one counter
    # gives a leaf its index and its first tile): the counts must be exact
    leaf_cfg(cfg)
    rng = np.random.default_rng(501 + cfg)
    n = 2500
    sizes = rng.integers(0, 1500, size=2 * n)
    sizes[rng.random(2 * n) < 0.05] = 0
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    data = rng.integers(0, 1 << 20, size=int(off[-1])).astype(np.int32)
    kind = rng.integers(0, 8, size=n)
    for q in range(n):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        data[o0:o1].sort()
        data[o1:o2].sort()
        if kind[q] == 0:
            data[o1:o2] += 1 << 21            # in order
        elif kind[q] == 1:
            data[o0:o1] += 1 << 21            # every B before every A
    t, to = d(data, dev), d(off, dev)
    say("leaf counters cfg", cfg, "instances", n, "elements", int(off[-1]))
    im.batched_inplace_merge(t, to)
    st = im.fetch_stats()
    leaves, tiles, elems = expected_leaves(data, off, st["tile"], st["max_levels"])
    assert (st["leaves"], st["tiles"], st["leaf_elems"]) == (leaves, tiles, elems), st
    check_batch(h(t), data, off, "leaf counters")


@pytest.mark.parametrize("tiles", [1, 3])
def test_leaf_counters_bounds_several_levels(dev, leaf_tiles, tiles):
    # several division levels: every leaf element is in one leaf, and the
    # tiles are the cells of the whole output that each leaf meets: between
    # leaf_elems / tile and that plus two per leaf (a leaf of S elements
    # meets at most ceil(S / tile) + 1 cells)
    leaf_tiles(tiles)
    la, lb = 1000003, 700001
    data = gen.pair_uniform(la, lb, 97)
    t = d(data, dev)
    say("leaf counter bounds, leaf tiles", tiles)
    im.inplace_merge(t, la)
    st = im.fetch_stats()
    assert st["levels_used"] >= 2, st
    assert 0 < st["leaf_elems"] <= la + lb
    lo = -(-st["leaf_elems"] // st["tile"])
    assert lo <= st["tiles"] <= lo + 2 * st["leaves"] - 1, st
    assert np.array_equal(h(t), oracle.merge(data, la))
