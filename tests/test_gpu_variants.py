"""The paper's alternative methods on the GPU, against the CPU oracle.

* FindMedian (Sec. 3.3, Alg. 1) on the device: the recursive division without
  data movement (im_divide) gives exactly the oracle's pair sizes, for both
  FindMedian and the exact middle co-rank, on the paper's W1 generator and on
  uniform and tie-heavy runs;
* the full merge with FindMedian splits and/or circular-shifting exchanges
  equals the stable merge (keys) element by element;
* circular shifting alone (im_rotate_cs) equals the definition of the
  exchange for lengths with one long cycle, many short cycles and segments;
* the out-of-place merge and the buffered merge equal the stable merge.
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
def leaf_tiles(monkeypatch):
    def setter(v):
        monkeypatch.setenv("IM_LEAF_TILES", str(v))
    return setter


def _inputs():
    yield "w1 1/4", gen.paper_w1_pair(40000, 0.25, 1), 10000
    yield "w1 1/2", gen.paper_w1_pair(40000, 0.5, 2), 20000
    yield "w1 3/4", gen.paper_w1_pair(40001, 0.75, 3), 30000
    yield "uniform", gen.pair_uniform(23457, 31001, 4), 23457
    yield "dup", gen.pair_uniform(30000, 30000, 5, hi=7), 30000
    yield "skew", gen.pair_uniform(50, 60000, 6), 50


@pytest.mark.parametrize("method", [im.SPLIT_CORANK, im.SPLIT_FINDMEDIAN])
def test_divide_matches_oracle(dev, method):
    name = "corank" if method == im.SPLIT_CORANK else "findmedian"
    for label, data, la in _inputs():
        for depth in (0, 1, 4, 9):
            say("divide", name, label, depth)
            got = h(im.divide(d(data, dev), la, depth, method))
            want = oracle.divide(data[:la], data[la:], depth, name)
            assert np.array_equal(got, want), (label, depth)


def test_divide_w1_full_depth(dev):
    # the paper's imbalance study shape: 2^18 elements, T up to 2^12 pairs
    data = gen.paper_w1_pair(2 ** 18, 0.5, 11)
    la = 2 ** 17
    for method, name in ((im.SPLIT_FINDMEDIAN, "findmedian"), (im.SPLIT_CORANK, "corank")):
        got = h(im.divide(d(data, dev), la, 12, method))
        want = oracle.divide(data[:la], data[la:], 12, name)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("split", [im.SPLIT_CORANK, im.SPLIT_FINDMEDIAN])
@pytest.mark.parametrize("rot", [im.ROTATE_SWAP_REV, im.ROTATE_CS])
@pytest.mark.parametrize("tiles", [1, 3])
def test_variant_merges(dev, leaf_tiles, split, rot, tiles):
    leaf_tiles(tiles)
    for label, data, la in _inputs():
        say("variant split", split, "rot", rot, "tiles", tiles, label)
        t = d(data, dev)
        im.inplace_merge_variant(t, la, split, rot)
        st = im.fetch_stats()
        got = h(t)
        want = oracle.merge(data, la)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, "%s: %d mismatches" % (label, bad.size)
        assert st["split_fallbacks"] >= 0
        assert st["levels_used"] >= 1


@pytest.mark.parametrize("dt", [np.int32, np.uint64])
def test_variant_int_types(dev, leaf_tiles, dt):
    leaf_tiles(2)
    data = gen.pair_uniform(70001, 65432, 12, dtype=dt)
    for split in (im.SPLIT_CORANK, im.SPLIT_FINDMEDIAN):
        for rot in (im.ROTATE_SWAP_REV, im.ROTATE_CS):
            t = d(data, dev)
            im.inplace_merge_variant(t, 70001, split, rot)
            assert np.array_equal(h(t), oracle.merge(data, 70001)), (split, rot)


# (lx, ly): one cycle (gcd 1) cut into many segments; many 2-cycles (block
# swap shape); gcd 64 with long cycles; tiny; gcd between
CS_CASES = [(1, 100000), (100000, 1), (50000, 50000), (64 * 1001, 64 * 777), (3, 5),
            (1, 1), (12345, 67890), (255, 257), (256 * 3, 256 * 5 + 1)]


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_rotate_cs_matches_definition(dev, dt):
    for lx, ly in CS_CASES:
        x = np.arange(lx + ly, dtype=dt) * 3 + 1
        say("rotate_cs", lx, ly)
        t = d(x, dev)
        im.rotate_cs(t, lx)
        want = oracle.rotate(x.astype(np.int64), lx).astype(dt)
        assert np.array_equal(h(t), want), (lx, ly)


# linear shifting: one long run of 1-element swaps, equal parts (a single
# block swap), runs of many swaps longer than a segment in both directions,
# tiny and coprime shapes, chains of exactly one segment
LS_CASES = CS_CASES + [(7, 300001), (300001, 7), (256, 256 * 257), (256 * 257 + 5, 256),
                       (1000, 1000 * 600 + 999), (2, 3), (0, 5), (5, 0)]


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_rotate_ls_matches_definition_and_counts(dev, dt):
    for lx, ly in LS_CASES:
        x = np.arange(lx + ly, dtype=dt) * 3 + 1
        say("rotate_ls", lx, ly)
        t = d(x, dev)
        _, swaps = im.rotate_ls(t, lx)
        want = oracle.rotate(x.astype(np.int64), lx).astype(dt)
        assert np.array_equal(h(t), want), (lx, ly)
        # the paper's swap count, as the oracle's linear shifting performs it
        _, want_swaps = oracle.rotate_ls(x.astype(np.int64), lx)
        assert swaps == want_swaps, (lx, ly, swaps, want_swaps)


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.int64, np.uint64])
def test_out_of_place_and_buffered(dev, dt):
    for la, lb, seed in [(1, 1, 1), (17920, 17921, 2), (100003, 77777, 3), (5, 300000, 4),
                         (250000, 0, 5)]:
        data = gen.pair_uniform(la, lb, seed, dtype=dt)
        want = oracle.merge(data, la)
        src = d(data, dev)
        out = im.merge_out_of_place(src, la)
        assert np.array_equal(h(out), want), (la, lb)
        assert np.array_equal(h(src), data)               # input untouched
        im.inplace_merge_buffered(src, la)
        assert np.array_equal(h(src), want), (la, lb)
