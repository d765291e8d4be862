"""Fused two-level exchanges against the CPU oracle.

Where a node and both of its children split symmetrically, k_split fuses the
two levels of exchanges into one permutation moved as cycles of contiguous
pieces.  Small leaf capacities (IM_LEAF_TILES) force many levels, so fusion
happens at every other level; every result must equal the stable merge with
fusion on and off (IM_FUSE=0), for keys, key+payload and batches.
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
def env(monkeypatch):
    def setter(tiles, fuse):
        monkeypatch.setenv("IM_LEAF_TILES", str(tiles))
        if fuse:
            monkeypatch.delenv("IM_FUSE", raising=False)
        else:
            monkeypatch.setenv("IM_FUSE", "0")
    return setter


INPUTS = [
    ("balanced", lambda: (gen.pair_uniform(300000, 300000, 1), 300000)),
    ("balanced odd", lambda: (gen.pair_uniform(277777, 290001, 2), 277777)),
    ("ties", lambda: (gen.pair_uniform(250000, 250000, 3, hi=50), 250000)),
    ("w1", lambda: (gen.paper_w1_pair(500000, 0.5, 4), 250000)),
    ("w1 3/4", lambda: (gen.paper_w1_pair(400000, 0.75, 5), 300000)),
    ("skew", lambda: (gen.pair_uniform(30000, 500000, 6), 30000)),
]


@pytest.mark.parametrize("tiles", [1, 2, 3])
@pytest.mark.parametrize("fuse", [True, False])
def test_fused_keys(dev, env, tiles, fuse):
    env(tiles, fuse)
    for label, mk in INPUTS:
        data, la = mk()
        say("fused", fuse, "tiles", tiles, label)
        t = d(data, dev)
        im.inplace_merge(t, la)
        st = im.fetch_stats()
        got = h(t)
        want = oracle.merge(data, la)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, "%s: %d mismatches, first at %d" % (label, bad.size, bad[0])
        if not fuse:
            assert st["fused_nodes"] == 0
        elif label.startswith("balanced"):
            assert st["fused_nodes"] > 0, st


@pytest.mark.parametrize("fuse", [True, False])
def test_fused_int64_and_kv(dev, env, fuse):
    env(2, fuse)
    data = gen.pair_uniform(260000, 260000, 7, dtype=np.int64)
    t = d(data, dev)
    im.inplace_merge(t, 260000)
    assert np.array_equal(h(t), oracle.merge(data, 260000))
    keys, vals = gen.pair_kv(240000, 240000, 8, key_hi=2 ** 40)
    for vdt in (np.uint32, np.uint64):
        k32 = keys.astype(np.int64) if vdt == np.uint64 else (keys % 2 ** 31).astype(np.int32)
        for q in (slice(0, 240000), slice(240000, None)):
            k32[q].sort()
        v = vals.astype(vdt)
        tk, tv = d(k32, dev), d(v, dev)
        im.inplace_merge_kv(tk, tv, 240000)
        st = im.fetch_stats()
        wk, wv = oracle.merge_kv(k32, v, 240000)
        assert np.array_equal(h(tk), wk) and np.array_equal(h(tv), wv), vdt
        if k32.dtype == np.int64 and vdt == np.uint64:
            assert st["fused_nodes"] == 0          # 16-byte elements are not fused


@pytest.mark.parametrize("fuse", [True, False])
def test_fused_batched(dev, env, fuse):
    env(1, fuse)
    data, off = gen.batch(60, 9, lo_exp=10.0, hi_exp=17.0)
    t = d(data, dev)
    im.batched_inplace_merge(t, d(off, dev))
    got = h(t)
    for q in range(60):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        assert np.array_equal(got[o0:o2], oracle.merge(data[o0:o2], int(o1 - o0))), q
