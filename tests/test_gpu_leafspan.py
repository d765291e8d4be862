"""The leaf merge's read-ahead bound, checked against the CPU oracle.

Every workgroup of the persistent leaf merge reads `depth` tiles (2, 3 or
4, by configuration and element size) ahead of its oldest unstored one, so a
leaf may span up to depth x G tiles (G resident workgroups, the default
capacity) and still never block for good.  The IM_LEAF_GRID hook shrinks G so
that small inputs put readers up to depth x G - 1 slots ahead of the tiles
they wait on (IM_LEAF_TILES=2G checks a smaller capacity); the full-size
cases check balanced leaves between G and 4G tiles at the real grid, one of
them with readers more than 3G slots ahead.
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


@pytest.fixture
def small_grid(monkeypatch):
    def setter(g):
        monkeypatch.setenv("IM_LEAF_GRID", str(g))
    yield setter
    im.set_config(-1)


CASES = [(100_000, 90_001), (7, 200_000), (200_000, 7), (150_000, 150_000), (1, 1), (17_920, 17_921)]


DEPTH = {0: 4, 1: 2, 2: 2, 3: 3}      # pipeline depth of each leaf configuration (int32 keys)


def single_pair_capacity(tiles_per_leaf, tile):
    # a single pair's tiles are cells of the whole output, so a leaf may meet
    # one cell more than ceil(S / tile): its size bound is one tile less
    # (when the read-ahead spans at least three tiles)
    return (tiles_per_leaf - 1) * tile if tiles_per_leaf >= 3 else tiles_per_leaf * tile


@pytest.mark.parametrize("grid", [1, 2, 3, 5, 16])
@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_small_grid_pairs(dev, small_grid, grid, cfg):
    small_grid(grid)
    im.set_config(cfg)
    for la, lb in CASES:
        for kind in ("uniform", "dup"):
            hi = 2 ** 31 if kind == "uniform" else 64
            data = gen.pair_uniform(la, lb, 3 * la + lb + grid, hi=hi)
            say("grid", grid, "cfg", cfg, kind, la, lb)
            t = d(data, dev)
            im.inplace_merge(t, la)
            st = im.fetch_stats()
            assert st["leaf_grid"] == grid
            assert st["leaf_capacity"] == single_pair_capacity(DEPTH[cfg] * grid, st["tile"])
            got = t.cpu().numpy()
            want = oracle.merge(data, la)
            bad = np.flatnonzero(got != want)
            assert bad.size == 0, "%d mismatches, first at %d" % (bad.size, bad[0])


@pytest.mark.parametrize("grid", [1, 2, 3, 5])
def test_small_grid_reduced_capacity(dev, small_grid, monkeypatch, grid):
    # a capacity below the read-ahead limit of configuration 0 (2G tiles per leaf)
    small_grid(grid)
    im.set_config(0)
    monkeypatch.setenv("IM_LEAF_TILES", str(2 * grid))
    for la, lb in CASES:
        data = gen.pair_uniform(la, lb, 5 * la + lb + grid)
        say("grid", grid, "2G tiles per leaf", la, lb)
        t = d(data, dev)
        im.inplace_merge(t, la)
        st = im.fetch_stats()
        assert st["leaf_capacity"] == single_pair_capacity(2 * grid, st["tile"])
        assert np.array_equal(t.cpu().numpy(), oracle.merge(data, la))


@pytest.mark.parametrize("grid", [2, 5])
def test_small_grid_kv_and_batched(dev, small_grid, grid):
    small_grid(grid)
    keys, vals = gen.pair_kv(120_000, 95_003, 17 + grid)
    tk, tv = d(keys, dev), d(vals, dev)
    im.inplace_merge_kv(tk, tv, 120_000)
    torch.cuda.synchronize()
    wk, wv = oracle.merge_kv(keys, vals, 120_000)
    assert np.array_equal(tk.cpu().numpy(), wk)
    assert np.array_equal(tv.cpu().numpy(), wv)
    data, off = gen.batch(150, 90 + grid, lo_exp=0.0, hi_exp=16.5)
    t = d(data, dev)
    im.batched_inplace_merge(t, d(off, dev))
    got = t.cpu().numpy()
    for q in range(150):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        assert np.array_equal(got[o0:o2], oracle.merge(data[o0:o2], int(o1 - o0))), q


@pytest.mark.parametrize("half", [2 ** 22 + 2 ** 21 + 12345, 2 ** 23 + 2 ** 22 + 777])
def test_balanced_leaf_beyond_g_tiles(dev, half):
    # one leaf of about 1.4 G (or 2.8 G) tiles with equal halves at the real
    # grid: the windows around the middle of A are read by tiles about 0.7 G
    # (1.4 G) slots ahead
    im.set_config(0)
    try:
        la = lb = half
        data = gen.pair_uniform(la, lb, 4242 + half % 97)
        t = d(data, dev)
        im.inplace_merge(t, la)
        st = im.fetch_stats()
        say(st)
        G = st["leaf_grid"]
        assert st["leaves"] == 1 and st["levels_used"] <= 1
        assert G * st["tile"] < la + lb <= st["leaf_capacity"]
        got = t.cpu().numpy()
        want = oracle.merge(data, la)
        assert np.array_equal(got, want)
    finally:
        im.set_config(-1)


def test_balanced_leaf_readers_beyond_3g(dev):
    # one leaf of 2^25 + 2^25 int32 at the real grid (the leaves of the
    # 2^27 + 2^27 merge): the last windows of A are read by tiles about
    # L_A / tile = 3.9 G slots ahead, which only depth 4 reaches
    im.set_config(0)
    try:
        la = lb = 2 ** 25
        data = gen.pair_uniform(la, lb, 4343)
        t = d(data, dev)
        im.inplace_merge(t, la)
        st = im.fetch_stats()
        say(st)
        G = st["leaf_grid"]
        assert st["leaves"] == 1 and st["levels_used"] <= 1
        assert la > 3 * G * st["tile"]
        got = t.cpu().numpy()
        want = oracle.merge(data, la)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, "%d mismatches, first at %d" % (bad.size, bad[0])
    finally:
        im.set_config(-1)


@pytest.mark.parametrize("grid", [1, 3, 7])
@pytest.mark.parametrize("kd,vd", [(np.int64, np.uint32), (np.int32, np.uint64)])
def test_small_grid_key_payload(dev, small_grid, monkeypatch, grid, kd, vd):
    # key+payload leaves with readers far ahead at a tiny grid, and leaf
    # capacities of a few tiles so that the exchanges of 1024-thread
    # workgroups run several levels
    small_grid(grid)
    for tiles in (None, 3):
        if tiles is None:
            monkeypatch.delenv("IM_LEAF_TILES", raising=False)
        else:
            monkeypatch.setenv("IM_LEAF_TILES", str(tiles))
        for la, lb in [(60_001, 59_999), (5, 90_000), (90_000, 5)]:
            keys = gen.pair_uniform(la, lb, 11 * la + lb + grid, hi=512, dtype=kd)
            vals = np.arange(la + lb, dtype=vd)
            say("kv grid", grid, "tiles", tiles, kd.__name__, vd.__name__, la, lb)
            tk, tv = d(keys, dev), d(vals, dev)
            im.inplace_merge_kv(tk, tv, la)
            wk, wv = oracle.merge_kv(keys, vals, la)
            assert np.array_equal(tk.cpu().numpy(), wk)
            assert np.array_equal(tv.cpu().numpy(), wv)
