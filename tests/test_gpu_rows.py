"""Wide rows (the elements of the paper's Sec. 4 test cases: a key in the
first word, then a payload) merged in place on the GPU, against the CPU
oracle's stable row merge, row by row and word by word.

* row widths that select each chunk width of the rows leaf merge (16, 8 and
  4 bytes) and rows from one key word to 64 KiB, with ragged last tiles;
* all four key types, ties, skewed sizes, already ordered and inverted runs;
* small leaf capacities (IM_LEAF_TILES) so the division runs several
  levels, with the fused two-level exchange on and off (IM_FUSE=0), and a
  small grid (IM_LEAF_GRID) so tiles wait for their readers.
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2005_12648_amd as im

pytestmark = pytest.mark.gpu

TDT = {np.int32: torch.int32, np.uint32: torch.uint32, np.int64: torch.int64,
       np.uint64: torch.uint64}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def d(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def h(t):
    return t.cpu().numpy()


@pytest.fixture
def env(monkeypatch):
    def setter(tiles=None, fuse=True, grid=None):
        for k, v in (("IM_LEAF_TILES", tiles), ("IM_LEAF_GRID", grid)):
            if v is None:
                monkeypatch.delenv(k, raising=False)
            else:
                monkeypatch.setenv(k, str(v))
        if fuse:
            monkeypatch.delenv("IM_FUSE", raising=False)
        else:
            monkeypatch.setenv("IM_FUSE", "0")
    return setter


def run(rows, la, dev):
    t = d(rows, dev)
    im.inplace_merge_rows(t, la)
    st = im.fetch_stats()
    got = h(t)
    want = oracle.merge_rows(rows, la)
    bad = np.flatnonzero(np.any(got != want, axis=1))
    return bad, st


# (row bytes, rows in A, rows in B): chunk 16 / 8 / 4 bytes, ragged tiles;
# 16-byte rows of up to 16 KiB take the three-deep kind, 32 and 64 KiB ones
# the two-deep kind with larger tiles
SHAPES = [(4, 70001, 65537), (8, 40000, 50003), (12, 30001, 29999), (16, 25000, 27001),
          (20, 20011, 19999), (64, 9001, 12007), (100, 5003, 4001), (256, 3001, 2999),
          (1000, 1201, 999), (4096, 301, 277), (16384, 77, 91), (32768, 31, 29),
          # the largest row of a three-deep tile (56 KiB) and the next 16-byte
          # multiple, which takes the two-deep kind
          (57344, 9, 11), (57360, 10, 9),
          (65536, 23, 19),
          # the paper's largest element (key + 16384 ints); 8-byte multiples
          # above 32 KiB; above 64 KiB in 4-byte chunks
          (65540, 23, 19), (32776, 40, 33), (81920, 17, 21)]


@pytest.mark.parametrize("row_bytes,la,lb", SHAPES)
def test_rows_shapes(dev, env, row_bytes, la, lb):
    env(tiles=2)
    rows = gen.rows_pair(la, lb, row_bytes // 4, 100 + row_bytes)
    say("rows", row_bytes, la, lb)
    bad, st = run(rows, la, dev)
    assert bad.size == 0, "%d rows differ, first %d" % (bad.size, bad[0])
    # (with one-row tiles and a two-tile leaf capacity every node ends in an
    # early exit or a whole exchange, and no leaf is left to merge)
    assert st["leaf_elems"] + st["rotated_elems"] > 0


@pytest.mark.parametrize("shift_words", [1, 2])
@pytest.mark.parametrize("row_bytes,la,lb", [(48, 20011, 19999), (64, 9001, 12007),
                                             (1024, 1201, 999)])
def test_rows_unaligned_base(dev, env, shift_words, row_bytes, la, lb):
    # rows whose base lies 4 or 8 bytes past a 16-byte boundary move in the
    # widest chunk the address allows (the 4- and 8-byte row kinds), with
    # several division levels; nothing before the base is written
    env(tiles=3)
    rows = gen.rows_pair(la, lb, row_bytes // 4, 500 + row_bytes + shift_words)
    n, words = rows.shape
    buf = torch.zeros(n * words + shift_words, dtype=torch.int32, device=dev)
    t = buf[shift_words:].view(n, words)
    assert t.data_ptr() % 16 == 4 * shift_words
    t.copy_(d(rows, dev))
    say("rows unaligned", row_bytes, la, lb, shift_words)
    im.inplace_merge_rows(t, la)
    bad = np.flatnonzero(np.any(h(t) != oracle.merge_rows(rows, la), axis=1))
    assert bad.size == 0, "%d rows differ, first %d" % (bad.size, bad[0])
    assert np.all(h(buf[:shift_words]) == 0)


def test_rows_too_wide_refused(dev):
    rows = np.zeros((4, 81924 // 4), dtype=np.int32)
    t = d(rows, dev)
    with pytest.raises(im.IMError) as e:
        im.inplace_merge_rows(t, 2)
    assert e.value.code == im.ERR_INVALID_ARG


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.int64, np.uint64])
def test_rows_key_types_and_ties(dev, env, dt):
    env(tiles=3)
    for la, lb, hi, words in [(20000, 23001, 2 ** 31, 16), (15000, 15000, 7, 8),
                              (300, 40000, 2 ** 31, 4), (40000, 300, 1000, 32)]:
        keys = gen.pair_uniform(la, lb, 7 + la, hi=hi, dtype=dt)
        rows = gen.rows_pair(la, lb, words, 9 + lb, dtype=dt, keys=keys)
        say("rows", dt.__name__, la, lb, hi, words)
        t = torch.from_numpy(rows).to(dev)
        assert t.dtype == TDT[dt]
        im.inplace_merge_rows(t, la)
        want = oracle.merge_rows(rows, la)
        assert np.array_equal(h(t), want), (la, lb, hi)


@pytest.mark.parametrize("tiles", [1, 2, 5])
@pytest.mark.parametrize("fuse", [True, False])
def test_rows_division_levels(dev, env, tiles, fuse):
    env(tiles=tiles, fuse=fuse)
    for row_bytes, la, lb, seed in [(64, 60000, 60000, 1), (48, 50001, 70003, 2),
                                    (512, 8000, 9000, 3)]:
        rows = gen.rows_pair(la, lb, row_bytes // 4, seed)
        say("levels", tiles, fuse, row_bytes, la, lb)
        bad, st = run(rows, la, dev)
        assert bad.size == 0, "%d rows differ" % bad.size
        assert st["levels_used"] >= 2
        if not fuse:
            assert st["fused_nodes"] == 0


def test_rows_small_grid_waits(dev, env):
    # a grid of 3 workgroups: every tile of a leaf waits for its readers
    env(tiles=None, grid=3)
    for row_bytes, la, lb in [(64, 20000, 21001), (1024, 1500, 1400), (12, 40001, 39999)]:
        rows = gen.rows_pair(la, lb, row_bytes // 4, 31 + la)
        say("grid 3", row_bytes, la, lb)
        bad, _ = run(rows, la, dev)
        assert bad.size == 0


def test_rows_special_cases(dev, env):
    env(tiles=2)
    w = 16
    # already ordered, inverted (a single exchange B|A), all keys equal
    a = gen.rows_pair(5000, 0, w, 41)
    b = gen.rows_pair(4000, 0, w, 42)
    b[:, 0] += a[-1, 0]
    ordered = np.concatenate([a, b])
    inverted = np.concatenate([b, a])
    same = gen.rows_pair(6000, 7000, w, 43)
    same[:, 0] = 5
    for label, rows, la in [("ordered", ordered, 5000), ("inverted", inverted, 4000),
                            ("equal", same, 6000)]:
        say("special", label)
        bad, _ = run(rows, la, dev)
        assert bad.size == 0, label
    assert np.array_equal(oracle.merge_rows(same, 6000), same)
    # one side empty: nothing happens
    t = d(ordered, dev)
    im.inplace_merge_rows(t, 0)
    im.inplace_merge_rows(t, t.shape[0])
    assert np.array_equal(h(t), ordered)


def test_rows_paper_generator(dev, env):
    # the paper's W1 keys (Sec. 4) with 1 KiB elements, split at 1/4, 1/2, 3/4
    env()
    for frac, seed in ((0.25, 51), (0.5, 52), (0.75, 53)):
        n = 24000
        keys = gen.paper_w1_pair(n, frac, seed)
        la = int(n * frac)
        rows = gen.rows_pair(la, n - la, 256, seed, keys=keys)
        say("w1 rows", frac)
        bad, _ = run(rows, la, dev)
        assert bad.size == 0


def test_rows_checked_mode_and_workspace(dev, env, monkeypatch):
    env(tiles=2)
    # checked mode reads the keys a row apart: an unsorted B is refused and
    # nothing is merged; sorted runs pass
    rows = gen.rows_pair(3000, 2000, 16, 61)
    bad = rows.copy()
    bad[3000:, 0] = bad[3000:, 0][::-1].copy()
    monkeypatch.setenv("IM_CHECK", "1")
    t = d(bad, dev)
    with pytest.raises(im.IMError) as e:
        im.inplace_merge_rows(t, 3000)
    assert e.value.code == -5
    bad_run, _ = run(rows, 3000, dev)
    assert bad_run.size == 0
    monkeypatch.delenv("IM_CHECK")
    # a caller workspace sized by the rows query works; a 4 KiB one is refused
    need = im.rows_workspace_bytes(rows.shape[0], 64, torch.int32)
    assert need > 4096
    buf = torch.empty(need, dtype=torch.uint8, device=dev)
    im.set_workspace(buf)
    try:
        bad_ws, _ = run(rows, 3000, dev)
        assert bad_ws.size == 0
        small = torch.empty(4096, dtype=torch.uint8, device=dev)
        im.set_workspace(small)
        with pytest.raises(im.IMError) as e:
            im.inplace_merge_rows(d(rows, dev), 3000)
        assert e.value.code == -4
    finally:
        im.set_workspace(None)
