"""Full-size parity: the workloads of the benchmark at their full sizes, run
through the C ABI in the launch configuration bench.py times, compared with
the CPU oracle element by element (the oracle finishes each in seconds):
c2 (plain, skewed, duplicate-heavy), c3 key+payload, the c4 batch and sort,
c5 plain and learned, and 1 GiB of rows of 64 B, 4 KiB and 64 KiB."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
import paper_2005_12648_amd as im

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_and_compare(data, la, dev, label):
    say("full-size", label, data.dtype, data.size, la)
    t = torch.from_numpy(data).to(dev)
    im.inplace_merge(t, la)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    del t
    want = oracle.merge(data, la)
    bad = int(np.count_nonzero(got != want))
    assert bad == 0, "%s: %d mismatches" % (label, bad)


@pytest.mark.parametrize("name", ["c2", "c2_skew", "c2_dup"])
def test_c2_full(dev, name):
    data, la = gen.make(name)
    run_and_compare(data, la, dev, name)


def test_c3_kv_full(dev):
    (keys, vals), la = gen.make("c3")
    say("full-size c3", keys.size)
    tk = torch.from_numpy(keys).to(dev)
    tv = torch.from_numpy(vals).to(dev)
    im.inplace_merge_kv(tk, tv, la)
    torch.cuda.synchronize()
    wk, wv = oracle.merge_kv(keys, vals, la)
    assert np.array_equal(tk.cpu().numpy(), wk)
    assert np.array_equal(tv.cpu().numpy(), wv)


def test_c4_batch_full(dev):
    data, off = gen.make("c4_batch")
    say("full-size c4 batch", data.size)
    t = torch.from_numpy(data).to(dev)
    max_inst = int(np.max(off[2::2] - off[0:-1:2]))
    im.batched_inplace_merge(t, torch.from_numpy(off).to(dev), max_instance=max_inst)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    for q in range(len(off) // 2):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        assert np.array_equal(got[o0:o2], oracle.merge(data[o0:o2], int(o1 - o0))), q


def test_c4_sort_full(dev):
    x = gen.make("c4_sort")
    say("full-size c4 sort", x.size)
    t = torch.from_numpy(x).to(dev)
    im.inplace_merge_sort(t)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.sort_keys(x))


def test_c5_plain_and_learned_full(dev):
    data, la = gen.make("c5")
    say("full-size c5", data.size)
    want = oracle.merge(data, la)
    t = torch.from_numpy(data).to(dev)
    model = im.MergeModel(seed=5).train(t, la, samples=8192, steps=20000, lr=1e-2)
    im.inplace_merge(t, la)
    torch.cuda.synchronize()
    assert int(np.count_nonzero(t.cpu().numpy() != want)) == 0
    t.copy_(torch.from_numpy(data).to(dev))
    model.merge(t, la)
    torch.cuda.synchronize()
    assert int(np.count_nonzero(t.cpu().numpy() != want)) == 0


@pytest.mark.parametrize("row_bytes", [64, 4096, 65536])
def test_rows_full(dev, row_bytes):
    # the rows form of the benchmark: 1 GiB of rows, L_A = L_B
    n = 2 ** 30 // row_bytes
    la = n // 2
    rows = gen.rows_pair(la, n - la, row_bytes // 4, 12648 + 60 + row_bytes.bit_length())
    say("full-size rows", row_bytes, n)
    t = torch.from_numpy(rows).to(dev)
    im.inplace_merge_rows(t, la)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    del t
    want = oracle.merge_rows(rows, la)
    bad = int(np.count_nonzero(np.any(got != want, axis=1)))
    assert bad == 0, "rows %d: %d mismatched rows" % (row_bytes, bad)
