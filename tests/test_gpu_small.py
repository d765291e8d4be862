"""The one-launch path for a small single pair (at most a quarter of the
resident tiles): every workgroup finds its tile's co-ranks and readers from
the keys and merges one tile.  Parity with the oracle on ragged sizes up to
the path's bound and one past it (the division path), on the edge shapes
(in order, reversed, equal keys, one-element runs, ties), keys of every type
and key+payload; the same results with the path turned off (IM_SMALL=0);
the statistics of the one launch."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2005_12648_amd as im

pytestmark = pytest.mark.gpu

TILE32 = 512 * 33        # configuration-0 tiles: 512 threads x 33 (int32) or 17 (int64) items
TILE64 = 512 * 17


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def d(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _bound_tiles():
    # resident workgroups of the leaf merge's configuration 0 (two per CU)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return 2 * cus // 4


def merge_both_ways(data, la, dev, monkeypatch, label):
    want = oracle.merge(data, la)
    got = {}
    for small in ("1", "0"):
        monkeypatch.setenv("IM_SMALL", small)
        t = d(data, dev)
        im.inplace_merge(t, la)
        st = im.fetch_stats()
        got[small] = (t.cpu().numpy(), st)
        bad = np.flatnonzero(got[small][0] != want)
        assert bad.size == 0, "%s (IM_SMALL=%s): %d mismatches, first at %d" % (
            label, small, bad.size, bad[0])
    monkeypatch.delenv("IM_SMALL")
    return got["1"][1]


def test_small_path_sizes(dev, monkeypatch):
    b = _bound_tiles()
    for n in [2, 3, 17, TILE32 - 1, TILE32, TILE32 + 1, 7 * TILE32 + 3, b * TILE32,
              b * TILE32 + 1]:
        rng = np.random.default_rng(n)
        la = int(rng.integers(1, n))
        data = gen.pair_uniform(la, n - la, 300 + n % 1000)
        say("small path", n, la)
        st = merge_both_ways(data, la, dev, monkeypatch, "n=%d" % n)
        if n <= b * TILE32:
            assert st["leaves"] == 1 and st["tiles"] == (n + TILE32 - 1) // TILE32
            assert st["leaf_elems"] == n and st["rotations"] == 0


@pytest.mark.parametrize("shape", ["in_order", "reversed", "equal", "one_a", "one_b", "ties",
                                   "skew"])
def test_small_path_shapes(dev, monkeypatch, shape):
    n = 5 * TILE32 + 11
    rng = np.random.default_rng(7)
    if shape == "in_order":
        data, la = np.arange(n, dtype=np.int32), n // 3
    elif shape == "reversed":
        data, la = np.concatenate([np.arange(n // 2, n), np.arange(0, n // 2)]).astype(np.int32), n - n // 2
    elif shape == "equal":
        data, la = np.full(n, 5, dtype=np.int32), n // 2
    elif shape == "one_a":
        data = np.concatenate([[n // 2], np.arange(n - 1)]).astype(np.int32)
        la = 1
    elif shape == "one_b":
        data = np.concatenate([np.arange(n - 1), [n // 3]]).astype(np.int32)
        la = n - 1
    elif shape == "ties":
        data, la = gen.pair_dup(n // 2, n - n // 2, 8), n // 2
    else:
        data, la = gen.pair_uniform(n // 20, n - n // 20, 9), n // 20
    merge_both_ways(data, la, dev, monkeypatch, shape)


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.int64, np.uint64])
def test_small_path_key_types(dev, monkeypatch, dt):
    info = np.iinfo(dt)
    tile = TILE32 if np.dtype(dt).itemsize == 4 else TILE64
    n = 9 * tile + 5
    rng = np.random.default_rng(11)
    a = np.sort(rng.integers(info.min, info.max, n // 2, dtype=dt, endpoint=True))
    b = np.sort(rng.integers(info.min, info.max, n - n // 2, dtype=dt, endpoint=True))
    a[0], b[-1] = info.min, info.max
    merge_both_ways(np.concatenate([a, b]), a.size, dev, monkeypatch, dt.__name__)


def test_small_path_key_payload(dev, monkeypatch):
    (k, v), la = gen.make("c3", scale=10)            # int64 keys in [0, 4096), uint32 payload
    want_k, want_v = oracle.merge_kv(k, v, la)
    for small in ("1", "0"):
        monkeypatch.setenv("IM_SMALL", small)
        kt, vt = d(k, dev), d(v, dev)
        im.inplace_merge_kv(kt, vt, la)
        torch.cuda.synchronize()
        assert np.array_equal(kt.cpu().numpy(), want_k), small
        assert np.array_equal(vt.cpu().numpy(), want_v), small
