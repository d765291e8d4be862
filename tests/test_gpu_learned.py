"""Learned split (1->32->1 ReLU network): GPU kernels against the fp64 oracle,
and exactness of the corrected co-ranks.

* forward pass and MSE gradient of the device kernels vs oracle.MLP64
  (fp32 on the device: rtol 1e-4 / atol 1e-6 for gradients, 1e-5 for outputs);
* co-ranks found from a prediction equal the oracle's for every diagonal,
  whatever the parameters (trained, untrained, NaN);
* merges through the learned path equal the oracle bit for bit;
* the trained network needs fewer probes per diagonal than plain binary
  search on the mixture workload (what the network buys).
Trained weights themselves are not compared ("parity unpinned").
"""
import math
import os
import sys
import tempfile

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


def random_params(seed):
    r = np.random.default_rng(seed)
    th = r.normal(0, 0.7, im.MLP_PARAMS)
    return th.astype(np.float32)


def test_forward_parity(dev):
    th = random_params(1)
    m = im.MergeModel(params=th)
    x = np.random.default_rng(2).uniform(0, 1, 10000).astype(np.float32)
    y = m.forward(d(x, dev)).cpu().numpy().astype(np.float64)
    ref = oracle.MLP64(32).forward(th.astype(np.float64), x.astype(np.float64))
    assert np.allclose(y, ref, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("M", [1, 63, 5000, 100003])
def test_gradient_parity(dev, M):
    th = random_params(3 + M)
    m = im.MergeModel(params=th)
    r = np.random.default_rng(M)
    x = r.uniform(0, 1, M).astype(np.float32)
    t = r.uniform(0, 1, M).astype(np.float32)
    g, loss = m.grad(d(x, dev), d(t, dev))
    ref = oracle.MLP64(32)
    th64 = th.astype(np.float64)
    gref = ref.grad(th64, x.astype(np.float64), t.astype(np.float64))
    lref = ref.loss(th64, x.astype(np.float64), t.astype(np.float64))
    assert np.allclose(g.cpu().numpy(), gref, rtol=1e-4, atol=1e-6)
    assert math.isclose(float(loss.item()), lref, rel_tol=1e-4, abs_tol=1e-7)


@pytest.fixture(scope="module")
def mixture(dev):
    data, la = gen.make("c5", scale=8)          # 2^20 + 2^20 of the mixture workload
    t = d(data, dev)
    model = im.MergeModel(seed=7).train(t, la, samples=4096, steps=1500, lr=3e-3)
    return data, la, t, model


def test_learned_corank_exact_and_cheaper(dev, mixture):
    data, la, t, model = mixture
    n = data.size
    ks = np.unique(np.concatenate([np.linspace(0, n, 50001).astype(np.int64),
                                   [0, 1, 2, n - 2, n - 1, n, la, la + 1]]))
    want = oracle.corank(data[:la], data[la:], ks)
    got_l, probes_l = model.corank(t, la, d(ks, dev))
    got_p, probes_p = im.corank(t, la, d(ks, dev), probes=True)
    assert np.array_equal(got_l.cpu().numpy(), want)
    assert np.array_equal(got_p.cpu().numpy(), want)
    ml = float(probes_l.double().mean())
    mp = float(probes_p.double().mean())
    say("probes per diagonal: learned %.2f, plain %.2f" % (ml, mp))
    assert ml < mp


@pytest.mark.parametrize("params", ["zeros", "nan", "huge"])
def test_bad_model_still_exact(dev, mixture, params):
    data, la, t, _ = mixture
    th = np.zeros(im.MLP_PARAMS, np.float32)
    if params == "nan":
        th[:] = np.nan
    elif params == "huge":
        th[:] = 1e30
    m = im.MergeModel(params=th)
    ks = np.linspace(0, data.size, 20001).astype(np.int64)
    got, _ = m.corank(t, la, d(ks, dev))
    assert np.array_equal(got.cpu().numpy(), oracle.corank(data[:la], data[la:], ks))


@pytest.mark.parametrize("tiles", [None, 1])
def test_learned_merge_matches_oracle(dev, mixture, monkeypatch, tiles):
    data, la, _, model = mixture
    if tiles:
        monkeypatch.setenv("IM_LEAF_TILES", str(tiles))
    t = d(data, dev)
    model.merge(t, la)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.merge(data, la))


def test_save_load_roundtrip(dev, mixture):
    data, la, t, model = mixture
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "m.bin")
        model.save(path)
        m2 = im.MergeModel.load_file(path)
    assert np.array_equal(model.params().numpy(), m2.params().numpy())
    ks = np.linspace(0, data.size, 4097).astype(np.int64)
    a, pa = model.corank(t, la, d(ks, dev))
    b, pb = m2.corank(t, la, d(ks, dev))
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert np.array_equal(pa.cpu().numpy(), pb.cpu().numpy())   # same error scale


def test_training_reduces_loss(dev, mixture):
    data, la, t, model = mixture
    n = data.size
    ks = np.linspace(0, n, 2049).astype(np.int64)
    x = (ks / n).astype(np.float32)
    tgt = (oracle.corank(data[:la], data[la:], ks) / la).astype(np.float32)
    _, l_trained = model.grad(d(x, dev), d(tgt, dev))
    _, l_init = im.MergeModel(seed=7).grad(d(x, dev), d(tgt, dev))
    say("loss: init %.3e trained %.3e" % (l_init.item(), l_trained.item()))
    assert l_trained.item() < 0.1 * l_init.item()
