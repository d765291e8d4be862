"""Seeded random sweep of the HIP path against the CPU oracle.

Each case draws the run lengths (log-uniform up to 2^20, empty runs
included), the key type and range (full range or heavy ties), the form
(keys, key+payload, rows, batched), the leaf configuration, a leaf
capacity of a few tiles (several division levels), a small leaf grid
(workgroups that wait for readers handed out by the slot counter) and
the fused two-level exchange on or off.  Every output is compared with
the oracle element by element.
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2005_12648_amd as im

pytestmark = pytest.mark.gpu

KEYS = [np.int32, np.uint32, np.int64, np.uint64]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture
def knobs(monkeypatch):
    def setter(tiles, grid, fuse, cfg):
        for k, v in (("IM_LEAF_TILES", tiles), ("IM_LEAF_GRID", grid)):
            if v is None:
                monkeypatch.delenv(k, raising=False)
            else:
                monkeypatch.setenv(k, str(v))
        if fuse:
            monkeypatch.delenv("IM_FUSE", raising=False)
        else:
            monkeypatch.setenv("IM_FUSE", "0")
        im.set_config(cfg)
    yield setter
    im.set_config(-1)


def lengths(r):
    def one():
        return 0 if r.random() < 0.05 else int(round(2.0 ** r.uniform(0, 20)))
    return one(), one()


@pytest.mark.parametrize("case", range(1000))
def test_random_case(dev, knobs, case):
    r = np.random.default_rng(20051264 + case)
    tiles = [None, 2, 3, 7][r.integers(4)]
    grid = [None, None, 2, 5][r.integers(4)]
    fuse = bool(r.integers(2))
    cfg = int(r.integers(-1, 4))
    knobs(tiles, grid, fuse, cfg)
    kd = KEYS[r.integers(4)]
    wide = 2 ** 31 if np.dtype(kd).itemsize == 4 else 2 ** 62
    hi = wide if r.random() < 0.6 else int(r.integers(2, 64))
    form = ["keys", "kv", "rows", "batched"][case % 4]
    seed = 7000 + case
    if form == "keys":
        la, lb = lengths(r)
        x = gen.pair_uniform(la, lb, seed, hi=hi, dtype=kd)
        say("case", case, form, kd.__name__, la, lb, hi, tiles, grid, fuse, cfg)
        t = torch.from_numpy(x).to(dev)
        im.inplace_merge(t, la)
        assert np.array_equal(t.cpu().numpy(), oracle.merge(x, la))
    elif form == "kv":
        la, lb = lengths(r)
        vd = [np.uint32, np.uint64][r.integers(2)]
        k = gen.pair_uniform(la, lb, seed, hi=hi, dtype=kd)
        v = np.arange(la + lb, dtype=vd)
        say("case", case, form, kd.__name__, vd.__name__, la, lb, hi, tiles, grid, fuse, cfg)
        tk, tv = torch.from_numpy(k).to(dev), torch.from_numpy(v).to(dev)
        im.inplace_merge_kv(tk, tv, la)
        wk, wv = oracle.merge_kv(k, v, la)
        assert np.array_equal(tk.cpu().numpy(), wk) and np.array_equal(tv.cpu().numpy(), wv)
    elif form == "rows":
        words = [1, 3, 4, 16, 64, 257][r.integers(6)]
        la, lb = [int(v) // words + (1 if v else 0) for v in lengths(r)]
        keys = gen.pair_uniform(la, lb, seed, hi=hi, dtype=kd)
        x = gen.rows_pair(la, lb, words, seed + 1, dtype=kd, keys=keys)
        say("case", case, form, kd.__name__, x.shape, la, lb, hi, tiles, grid, fuse)
        t = torch.from_numpy(x).to(dev)
        im.inplace_merge_rows(t, la)
        assert np.array_equal(t.cpu().numpy(), oracle.merge_rows(x, la))
    else:
        n_inst = int(r.integers(1, 300))
        runs = [int(round(2.0 ** r.uniform(0, 14))) if r.random() > 0.05 else 0
                for _ in range(2 * n_inst)]
        runs[0] = max(runs[0], 1)
        off = np.concatenate([[0], np.cumsum(runs)]).astype(np.int64)
        x = np.concatenate([gen.sorted_uniform(m, 0, hi, seed + q, kd) for q, m in enumerate(runs)])
        say("case", case, form, kd.__name__, n_inst, int(off[-1]), hi, tiles, grid, fuse, cfg)
        t = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        im.batched_inplace_merge(t, torch.from_numpy(off).to(dev))
        got = t.cpu().numpy()
        for q in range(n_inst):
            o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
            assert np.array_equal(got[o0:o2], oracle.merge(x[o0:o2], int(o1 - o0))), q
