"""The boundary's own forms and guarantees, through the C ABI:

* the offsets-only batched forms (the total is read back from the offsets)
  against the oracle, keys and key+payload;
* inplace_merge_last_stats against inplace_merge_fetch_stats;
* a caller workspace of inplace_merge_workspace_bytes(N, dtype) bytes serves a
  single merge and an in-place merge sort of N;
* two merge sorts enqueued on two streams at once, each against np.sort (the
  sort passes' offsets live in the ordered workspace);
* a merge enqueued on a capturing stream is refused with IM_ERR_INVALID_ARG;
* the device-side error word stays clear on good inputs.
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


def _batch(rng, n, hi, dtype):
    parts, off = [], [0]
    for q in range(n):
        la, lb = (int(x) for x in rng.integers(0, 3000, size=2))
        if q % 7 == 0:
            la = 0
        a = np.sort(rng.integers(0, hi, la)).astype(dtype)
        b = np.sort(rng.integers(0, hi, lb)).astype(dtype)
        parts += [a, b]
        off += [off[-1] + la, off[-1] + la + lb]
    return np.concatenate(parts), np.array(off, dtype=np.int64)


@pytest.mark.parametrize("dtype", [np.int32, np.uint64])
def test_offsets_only_batched_forms(dev, dtype):
    rng = np.random.default_rng(81)
    data, off = _batch(rng, 37, 200, dtype)
    say("offsets-only batch", dtype.__name__, data.size)
    want = data.copy()
    for q in range((off.size - 1) // 2):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        want[o0:o2] = oracle.merge(data[o0:o2], int(o1 - o0))
    # a buffer longer than the offsets' total: the tail stays untouched
    tail = np.arange(100, dtype=dtype)
    t = d(np.concatenate([data, tail]), dev)
    im.batched_inplace_merge(t, d(off, dev), sized=False)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    assert np.array_equal(got[:data.size], want)
    assert np.array_equal(got[data.size:], tail)
    # key + payload (payload = position)
    vals = np.arange(data.size, dtype=np.uint32)
    kt, vt = d(data, dev), d(vals, dev)
    im.batched_inplace_merge_kv(kt, vt, d(off, dev), sized=False)
    torch.cuda.synchronize()
    wk, wv = data.copy(), vals.copy()
    for q in range((off.size - 1) // 2):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        wk[o0:o2], wv[o0:o2] = oracle.merge_kv(data[o0:o2], vals[o0:o2], int(o1 - o0))
    assert np.array_equal(kt.cpu().numpy(), wk)
    assert np.array_equal(vt.cpu().numpy(), wv)


def test_last_stats_matches_fetch_stats(dev):
    data, la = gen.make("c1")
    t = d(data, dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        im.inplace_merge(t, la)
    a = im.last_stats()            # synchronises the stream the merge ran on
    b = im.fetch_stats(stream=s)
    assert a == b
    assert a["leaf_elems"] == data.size and a["leaves"] >= 1
    assert np.array_equal(t.cpu().numpy(), oracle.merge(data, la))


def test_workspace_bytes_single_form_serves_merge_and_sort(dev):
    n = 300_001
    rng = np.random.default_rng(82)
    need = im.workspace_bytes(n, 1, torch.int32)
    say("caller workspace", need, "bytes")
    assert 0 < need < 64 << 20
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    try:
        im.set_workspace(ws)
        la = 120_000
        data = np.concatenate([np.sort(rng.integers(0, 1 << 31, la)),
                               np.sort(rng.integers(0, 1 << 31, n - la))]).astype(np.int32)
        t = d(data, dev)
        im.inplace_merge(t, la)
        u = rng.integers(-(1 << 31), 1 << 31, n).astype(np.int32)
        tu = d(u, dev)
        im.inplace_merge_sort(tu)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), oracle.merge(data, la))
        assert np.array_equal(tu.cpu().numpy(), np.sort(u))
    finally:
        torch.cuda.synchronize()
        im.set_workspace(None)


def test_two_stream_sorts(dev):
    rng = np.random.default_rng(83)
    xs = [rng.integers(0, 1 << 31, n).astype(np.int32) for n in (1_500_007, 700_001)]
    ts = [d(x, dev) for x in xs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    say("two sorts on two streams")
    for rep in range(3):
        for x, t in zip(xs, ts):
            t.copy_(d(x, dev))
        torch.cuda.synchronize()
        for t, s in zip(ts, streams):
            with torch.cuda.stream(s):
                im.inplace_merge_sort(t)
        torch.cuda.synchronize()
        for x, t in zip(xs, ts):
            assert np.array_equal(t.cpu().numpy(), np.sort(x)), rep


def test_capture_is_refused(dev):
    data, la = gen.make("c1")
    t = d(data, dev)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    code = None
    with torch.cuda.graph(g):
        try:
            im.inplace_merge(t, la)
        except im.IMError as e:
            code = e.code
    assert code == im.ERR_INVALID_ARG
    torch.cuda.synchronize()
    # nothing ran: the input is untouched, and an eager merge still works
    assert np.array_equal(t.cpu().numpy(), data)
    im.inplace_merge(t, la)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.merge(data, la))


def test_device_status_clear_after_merges(dev):
    data, la = gen.make("c1")
    t = d(data, dev)
    im.inplace_merge(t, la)
    torch.cuda.synchronize()
    assert im.device_status() == 0
