"""The allocation-free entry point inplace_merge_noalloc, through the C ABI,
against inplace_merge on the same inputs (bit exact): two calls in a row on
one device, the second on a smaller input, with forced division levels so
that every workspace region (nodes, exchanges, leaves, tiles, flags) is used;
int32 and int64 keys; and a merge too large for the static array refused
before any work (the data pointer is never touched)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import gen
import paper_2005_12648_amd as im

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(t, la):
    lib = im.load()
    code = {torch.int32: 0, torch.uint32: 1, torch.int64: 2, torch.uint64: 3}[t.dtype]
    rc = lib.inplace_merge_noalloc(ctypes.c_void_p(t.data_ptr()), la, t.numel() - la, code,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise im.IMError(rc, lib.inplace_merge_last_error().decode())


@pytest.mark.parametrize("tiles", [None, 3])
@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_noalloc_matches_inplace_merge(dev, monkeypatch, tiles, dt):
    if tiles:
        monkeypatch.setenv("IM_LEAF_TILES", str(tiles))
    for n, la, seed, hi in [(3_000_001, 1_300_000, 91, 2 ** 31), (200_003, 150_000, 92, 50)]:
        data = gen.pair_uniform(la, n - la, seed, hi=hi, dtype=dt)
        say("noalloc", dt.__name__, tiles, n, la)
        a = torch.from_numpy(data).to(dev)
        b = a.clone()
        im.inplace_merge(a, la)
        _noalloc(b, la)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (n, la)
        assert bool((b[1:] >= b[:-1]).all())


def test_noalloc_refuses_what_does_not_fit(dev):
    lib = im.load()
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: refused on the host
    rc = lib.inplace_merge_noalloc(fake, 2 ** 35, 2 ** 35, 0, None)
    assert rc == im.ERR_WORKSPACE
    assert "static scratch" in lib.inplace_merge_last_error().decode()
    # and the entry point still works afterwards
    data = gen.pair_uniform(70_000, 70_001, 93)
    t = torch.from_numpy(data).to(dev)
    u = t.clone()
    _noalloc(t, 70_000)
    im.inplace_merge(u, 70_000)
    torch.cuda.synchronize()
    assert torch.equal(t, u)
