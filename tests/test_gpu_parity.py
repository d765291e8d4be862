"""Parity of the HIP path with the CPU oracle (element by element, bit exact).

Every call goes through the C ABI (ctypes binding) into the HIP kernels; the
expected values come only from ``oracle/``.  Sizes span several workgroup
tiles with ragged tails; the environment hook IM_LEAF_TILES shrinks the leaf
capacity so that small inputs exercise the division levels, the block swaps,
the three-reversal exchanges and multi-tile leaves with their barrier.
"""
import os
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2005_12648_amd as im

pytestmark = pytest.mark.gpu

TILE32 = 512 * 35     # leaf-merge tile of 4-byte keys
TILE64 = 512 * 17     # leaf-merge tile of 8-byte keys


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def d(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def h(t):
    return t.cpu().numpy()


def check_merge(data, la, dev, label=""):
    say("merge", label, data.dtype, data.size, la)
    t = d(data, dev)
    im.inplace_merge(t, la)
    torch.cuda.synchronize()
    want = oracle.merge(data, la)
    got = h(t)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, "%s: %d mismatches, first at %d" % (label, bad.size, bad[0])


@pytest.fixture
def leaf_tiles(monkeypatch):
    def setter(v):
        if v is None:
            monkeypatch.delenv("IM_LEAF_TILES", raising=False)
        else:
            monkeypatch.setenv("IM_LEAF_TILES", str(v))
    return setter


# ---------------------------------------------------------------- co-rank
def test_corank_every_diagonal_c1(dev):
    data, la = gen.make("c1")
    a, b = data[:la], data[la:]
    ks = np.arange(data.size + 1, dtype=np.int64)
    got = h(im.corank(d(data, dev), la, d(ks, dev)))
    assert np.array_equal(got, oracle.corank(a, b, ks))


@pytest.mark.parametrize("kind", ["dup", "skew", "w1", "tiny_keys"])
def test_corank_special_inputs(dev, kind):
    if kind == "dup":
        data, la = gen.pair_dup(5000, 7000, 3), 5000
    elif kind == "skew":
        data, la = gen.pair_uniform(37, 20000, 4), 37
    elif kind == "w1":
        data, la = gen.paper_w1_pair(30000, 0.25, 5), 7500
    else:
        data, la = gen.pair_uniform(3000, 3000, 6, hi=2), 3000
    ks = np.arange(data.size + 1, dtype=np.int64)
    got = h(im.corank(d(data, dev), la, d(ks, dev)))
    assert np.array_equal(got, oracle.corank(data[:la], data[la:], ks))


# --------------------------------------------------------------- rotation
ROT_CASES = [(1, 1), (1, 99999), (99999, 1), (4096, 4096), (4097, 4095), (12345, 67890),
             (2 ** 20, 2 ** 20 + 3), (3, 2 ** 17), (8191, 8193), (0, 10), (10, 0)]


@pytest.mark.parametrize("lx,ly", ROT_CASES)
@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_rotate(dev, lx, ly, dt):
    x = (np.arange(lx + ly, dtype=np.int64) * 7 + 3).astype(dt)
    t = d(x, dev)
    im.rotate(t, lx)
    want = oracle.rotate(x.astype(np.int64), lx).astype(dt)
    assert np.array_equal(h(t), want)


# ----------------------------------------------------------------- merge
def test_merge_c1_full(dev):
    data, la = gen.make("c1")
    check_merge(data, la, dev, "c1")


EDGE = [
    ("a_empty", np.arange(10, dtype=np.int32), 0),
    ("b_empty", np.arange(10, dtype=np.int32), 10),
    ("ordered", np.arange(100000, dtype=np.int32), 50000),
    ("inverted_equal", np.concatenate([np.arange(5000, 10000), np.arange(5000)]).astype(np.int32), 5000),
    ("inverted_unequal", np.concatenate([np.arange(777, 20000), np.arange(777)]).astype(np.int32), 20000 - 777),
    ("all_equal", np.full(50001, 9, dtype=np.int32), 20000),
    ("one_one", np.array([5, 3], dtype=np.int32), 1),
    ("one_many", np.concatenate([[10 ** 6], np.arange(30000)]).astype(np.int32), 1),
    ("many_one", np.concatenate([np.arange(30000), [-5]]).astype(np.int32), 30000),
    ("boundary_tie", np.concatenate([np.full(9000, 7), np.full(9000, 7)]).astype(np.int32), 9000),
]


@pytest.mark.parametrize("name,data,la", EDGE, ids=[e[0] for e in EDGE])
def test_merge_edge_cases(dev, name, data, la):
    check_merge(data, la, dev, name)


@pytest.mark.parametrize("n", [2, 3, 100, TILE32 - 1, TILE32, TILE32 + 1, 3 * TILE32 + 17,
                               10 * TILE32 + 5, 123457])
def test_merge_ragged_sizes(dev, n):
    rng = np.random.default_rng(n)
    la = int(rng.integers(1, n))
    data = gen.pair_uniform(la, n - la, n)
    check_merge(data, la, dev, "ragged")


@pytest.mark.parametrize("tiles", [1, 2, 5])
@pytest.mark.parametrize("case", ["balanced", "skew", "dup", "w1"])
def test_merge_division_levels(dev, leaf_tiles, tiles, case):
    """Small leaf capacity -> several division levels, swaps and reversals."""
    leaf_tiles(tiles)
    n = 400_000 + 123
    if case == "balanced":
        data, la = gen.pair_uniform(n // 2, n - n // 2, 21), n // 2
    elif case == "skew":
        data, la = gen.pair_uniform(n // 16, n - n // 16, 22), n // 16
    elif case == "dup":
        data, la = gen.pair_dup(n // 2, n - n // 2, 23), n // 2
    else:
        data, la = gen.paper_w1_pair(n, 0.75, 24), int(n * 0.75)
    check_merge(data, la, dev, case)
    st = im.fetch_stats()
    say(st)
    if case in ("balanced", "skew") and tiles <= 2:
        # leaf span is zero: only the size bound makes leaves
        assert st["levels_used"] >= 3
        assert st["rotations"] > 0


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.int64, np.uint64])
def test_merge_dtypes_extremes(dev, leaf_tiles, dt):
    leaf_tiles(2)
    info = np.iinfo(dt)
    rng = np.random.default_rng(1)
    n = 70001
    a = np.sort(rng.integers(info.min, info.max, size=n // 3, dtype=dt, endpoint=True))
    b = np.sort(rng.integers(info.min, info.max, size=n - n // 3, dtype=dt, endpoint=True))
    a[0], a[-1], b[0], b[-1] = info.min, info.max, info.min, info.max
    check_merge(np.concatenate([a, b]), a.size, dev, str(dt))


# --------------------------------------------------------- key + payload
@pytest.mark.parametrize("kd,vd", [(np.int64, np.uint32), (np.int32, np.uint32),
                                   (np.int32, np.uint64), (np.int64, np.uint64),
                                   (np.uint64, np.int32)])
@pytest.mark.parametrize("tiles", [None, 1, 3])
def test_merge_kv(dev, leaf_tiles, kd, vd, tiles):
    leaf_tiles(tiles)
    la, lb = 150_001, 99_998
    keys = gen.pair_uniform(la, lb, 31, hi=4096, dtype=np.int64).astype(kd)
    vals = np.arange(la + lb).astype(vd)
    tk, tv = d(keys, dev), d(vals, dev)
    im.inplace_merge_kv(tk, tv, la)
    torch.cuda.synchronize()
    wk, wv = oracle.merge_kv(keys, vals, la)
    assert np.array_equal(h(tk), wk)
    assert np.array_equal(h(tv), wv)


# --------------------------------------------------------------- batched
@pytest.mark.parametrize("tiles", [None, 1])
def test_batched(dev, leaf_tiles, tiles):
    leaf_tiles(tiles)
    data, off = gen.batch(300, 41, lo_exp=0.0, hi_exp=15.5)
    # a few degenerate instances: empty A, empty B, empty both
    off = off.copy()
    t, to = d(data, dev), d(off, dev)
    im.batched_inplace_merge(t, to, max_instance=int(np.max(off[2::2] - off[:-1:2])))
    torch.cuda.synchronize()
    got = h(t)
    for q in range(300):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        want = oracle.merge(data[o0:o2], int(o1 - o0))
        assert np.array_equal(got[o0:o2], want), q


def test_batched_degenerate_instances(dev, leaf_tiles):
    leaf_tiles(1)
    rng = np.random.default_rng(9)
    sizes = [(0, 0), (0, 5), (5, 0), (1, 1), (30000, 0), (20000, 20001), (3, 40000), (0, 0)]
    parts, off = [], [0]
    for la, lb in sizes:
        a = np.sort(rng.integers(0, 100, la)).astype(np.int32)
        b = np.sort(rng.integers(0, 100, lb)).astype(np.int32)
        parts += [a, b]
        off += [off[-1] + la, off[-1] + la + lb]
    data = np.concatenate(parts)
    off = np.array(off, dtype=np.int64)
    t = d(data, dev)
    im.batched_inplace_merge(t, d(off, dev))
    torch.cuda.synchronize()
    got = h(t)
    for q in range(len(sizes)):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        assert np.array_equal(got[o0:o2], oracle.merge(data[o0:o2], int(o1 - o0))), q


def test_batched_kv(dev, leaf_tiles):
    leaf_tiles(1)
    data, off = gen.batch(64, 43, lo_exp=3.0, hi_exp=15.0)
    keys = (data % 100).astype(np.int64)
    for q in range(64):
        keys[off[2 * q]:off[2 * q + 1]].sort()
        keys[off[2 * q + 1]:off[2 * q + 2]].sort()
    vals = np.arange(keys.size, dtype=np.uint32)
    tk, tv = d(keys, dev), d(vals, dev)
    im.batched_inplace_merge_kv(tk, tv, d(off, dev))
    torch.cuda.synchronize()
    gk, gv = h(tk), h(tv)
    for q in range(64):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        wk, wv = oracle.merge_kv(keys[o0:o2], vals[o0:o2], int(o1 - o0))
        assert np.array_equal(gk[o0:o2], wk) and np.array_equal(gv[o0:o2], wv), q


# ------------------------------------------------------------ merge sort
# sizes around the tile sort's tiles (16384 4-byte or 8192 8-byte keys)
@pytest.mark.parametrize("n", [1, 2, 8191, 8192, 8193, 16383, 16384, 16385, 100003,
                               3 * 16384 + 5, 2 ** 20 + 37])
@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_merge_sort(dev, n, dt):
    x = gen.unsorted(n, 77 + n).astype(dt)
    t = d(x, dev)
    im.inplace_merge_sort(t)
    torch.cuda.synchronize()
    assert np.array_equal(h(t), oracle.sort_keys(x))


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.int64, np.uint64])
def test_merge_sort_extreme_keys(dev, dt):
    # the type's maximum is also the tile sort's end-of-run sentinel: keys
    # equal to it, to the minimum and heavy duplicates must come out right
    info = np.iinfo(dt)
    r = np.random.default_rng(91)
    for n in (5000, 16384 + 3, 70001):
        pick = r.integers(0, 6, size=n)
        x = r.integers(0, 4, size=n).astype(dt)
        x[pick == 0] = info.max
        x[pick == 1] = info.min
        t = torch.from_numpy(x).to(dev)
        im.inplace_merge_sort(t)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), oracle.sort_keys(x)), (dt.__name__, n)


def test_merge_sort_forced_levels(dev, leaf_tiles):
    leaf_tiles(1)
    x = gen.unsorted(3 * 2 ** 18 + 11, 78)
    t = d(x, dev)
    im.inplace_merge_sort(t)
    torch.cuda.synchronize()
    assert np.array_equal(h(t), oracle.sort_keys(x))


# ---------------------------------------------------------- checked mode
def test_checked_mode_and_faults(dev, monkeypatch):
    x = np.concatenate([np.arange(100), np.arange(50)[::-1]]).astype(np.int32)  # B unsorted
    t = d(x, dev)
    monkeypatch.setenv("IM_CHECK", "1")
    with pytest.raises(im.IMError) as e:
        im.inplace_merge(t, 100)
    assert e.value.code == -5
    ok = gen.pair_uniform(1000, 1000, 3)
    t2 = d(ok, dev)
    im.inplace_merge(t2, 1000)          # checked and sorted: passes
    assert np.array_equal(h(t2), oracle.merge(ok, 1000))
    monkeypatch.delenv("IM_CHECK")
    monkeypatch.setenv("IM_FAULT", "alloc")
    with pytest.raises(im.IMError) as e:
        im.inplace_merge(d(ok, dev), 1000)
    assert e.value.code == -4
    monkeypatch.setenv("IM_FAULT", "launch")
    with pytest.raises(im.IMError) as e:
        im.inplace_merge(d(ok, dev), 1000)
    assert e.value.code == -3
    monkeypatch.delenv("IM_FAULT")
    t3 = d(ok, dev)
    im.inplace_merge(t3, 1000)
    assert np.array_equal(h(t3), oracle.merge(ok, 1000))


def test_user_workspace(dev):
    data = gen.pair_uniform(60000, 70000, 5)
    need = im.workspace_bytes(data.size, 1, torch.int32)
    assert need > 0
    buf = torch.empty(need, dtype=torch.uint8, device=dev)
    im.set_workspace(buf)
    try:
        check_merge(data, 60000, dev, "user ws")
        assert need > 4096
        small = torch.empty(4096, dtype=torch.uint8, device=dev)
        im.set_workspace(small)
        with pytest.raises(im.IMError) as e:
            im.inplace_merge(d(data, dev), 60000)
        assert e.value.code == -4
    finally:
        im.set_workspace(None)


def test_repeat_runs_identical(dev):
    data, la = gen.make("c2", scale=6)
    outs = []
    for _ in range(3):
        t = d(data, dev)
        im.inplace_merge(t, la)
        outs.append(h(t))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    assert np.array_equal(outs[0], oracle.merge(data, la))


@pytest.mark.parametrize("la,lb", [(3000, 3_000_000), (3_000_000, 3000),
                                   (1_000_000, 5_000_000), (5_000_000, 1_000_000)])
def test_merge_leaf_beyond_grid(dev, la, lb):
    """Leaves with more tiles than resident workgroups: the smaller part bounds
    how far elements travel, and the tile order follows it."""
    data = gen.pair_uniform(la, lb, la + 7 * lb)
    check_merge(data, la, dev, "big leaf")
    st = im.fetch_stats()
    say(st)
    assert st["leaves"] >= 1


@pytest.mark.parametrize("la,lb", [(20_000, 400_000), (400_000, 20_000), (50_000, 60_000)])
def test_merge_leaf_span_hook(dev, leaf_tiles, la, lb):
    leaf_tiles(8)        # leaf capacity 8 tiles, span 6 tiles
    data = gen.pair_uniform(la, lb, la + lb)
    check_merge(data, la, dev, "span hook")
