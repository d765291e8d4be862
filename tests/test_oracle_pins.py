"""Pins of the CPU oracle against what the paper and mathematics fix.

No GPU.  The oracle (``oracle/``) is checked against:
  * brute force: the stable sort of A++B by (key, source A<B, index), every
    (L_A, L_B) <= 6 with keys in {0, 1, 2} -- the definition of the problem
    (Sec. 1) under the stable reading;
  * hand-worked fixtures under tests/golden/ (merge with ties; the linear
    shifting trace and the circular shifting cycle of Sec. 3.4);
  * the counts the paper proves: circular shifting uses gcd(L_A, L_B) cycles
    and moves every element exactly once (Sec. 3.4 proof, Sec. 3.5); linear
    shifting swaps exactly L_A elements when L_A = L_B (Sec. 3.5) and
    L_X + L_Y - gcd in general;
  * invariants: sorted output, same multiset, identity on already ordered
    input, B|A on inverted input (the early exits of Alg. 1 and Alg. 2/3);
  * co-rank properties: i(0) = 0, i(N) = L_A, steps of 0 or 1;
  * the network's gradients against central finite differences, and the
    first Adam step against its closed form;
  * the merge-sort result against a bottom-up merge sort built from the
    oracle's own merge.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def brute_merge(a, b):
    tagged = [(int(x), 0, i) for i, x in enumerate(a)] + [(int(x), 1, i) for i, x in enumerate(b)]
    return sorted(tagged)


def test_exhaustive_small_stable():
    # every pair of sorted runs of length <= 6 over keys {0,1,2}
    runs = {0: [()]}
    for L in range(1, 7):
        runs[L] = [c for c in itertools.combinations_with_replacement(range(3), L)]
    n_cases = 0
    for la in range(0, 7):
        for lb in range(0, 7):
            for a in runs[la]:
                for b in runs[lb]:
                    data = np.array(a + b, dtype=np.int32)
                    got = oracle.merge(data, la)
                    ref = brute_merge(a, b)
                    assert got.tolist() == [t[0] for t in ref]
                    # co-rank by definition from the brute-force tags
                    ks = np.arange(la + lb + 1)
                    want = [sum(1 for t in ref[:k] if t[1] == 0) for k in ks]
                    assert oracle.corank(np.array(a, np.int32), np.array(b, np.int32), ks).tolist() == want
                    n_cases += 1
    assert n_cases == 84 * 84   # multisets of size <= 6 over 3 keys: 84 per run


def test_kv_stability_brute():
    rng = np.random.default_rng(5)
    for _ in range(300):
        la, lb = rng.integers(0, 40, size=2)
        a = np.sort(rng.integers(0, 4, la)).astype(np.int64)
        b = np.sort(rng.integers(0, 4, lb)).astype(np.int64)
        keys = np.concatenate([a, b])
        vals = np.arange(la + lb, dtype=np.uint32)
        k, v = oracle.merge_kv(keys, vals, int(la))
        ref = brute_merge(a, b)
        assert k.tolist() == [t[0] for t in ref]
        assert v.tolist() == [t[2] + (0 if t[1] == 0 else int(la)) for t in ref]
        # payload = index  =>  (key, payload) strictly increasing
        pairs = list(zip(k.tolist(), v.tolist()))
        assert all(p < q for p, q in zip(pairs, pairs[1:]))


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.int64, np.uint64])
def test_random_against_library_sort(dt):
    rng = np.random.default_rng(7)
    for _ in range(50):
        la, lb = rng.integers(0, 3000, size=2)
        hi = int(rng.choice([3, 100, 2 ** 31 - 1]))
        a = np.sort(rng.integers(0, hi, la)).astype(dt)
        b = np.sort(rng.integers(0, hi, lb)).astype(dt)
        got = oracle.merge(np.concatenate([a, b]), int(la))
        assert np.array_equal(got, np.sort(np.concatenate([a, b]), kind="stable"))


def test_extreme_keys():
    for dt in (np.int32, np.int64, np.uint32, np.uint64):
        info = np.iinfo(dt)
        a = np.array([info.min, 0, info.max], dtype=dt)
        b = np.array([info.min, info.max, info.max], dtype=dt)
        got = oracle.merge(np.concatenate([a, b]), 3)
        assert got.tolist() == sorted(a.tolist() + b.tolist())


def test_early_exit_cases():
    a = np.arange(10, dtype=np.int32)
    b = np.arange(10, 20, dtype=np.int32)
    ab = np.concatenate([a, b])
    assert np.array_equal(oracle.merge(ab, 10), ab)                 # A[last] <= B[0]
    ba = np.concatenate([b, a])
    assert np.array_equal(oracle.merge(ba, 10), np.concatenate([a, b]))   # A[0] > B[last]
    eq = np.full(17, 4, dtype=np.int32)
    assert np.array_equal(oracle.merge(eq, 5), eq)                  # all equal: identity
    assert np.array_equal(oracle.merge(ab, 0), ab)
    assert np.array_equal(oracle.merge(ab, 20), ab)
    k, v = oracle.merge_kv(np.full(9, 3, np.int64), np.arange(9, dtype=np.uint32), 4)
    assert v.tolist() == list(range(9))


def _read(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *rest = line.split()
            out.setdefault(tag, []).append(rest)
    return out


def test_golden_merge_ties():
    g = _read("merge_ties.txt")
    a = np.array([int(x) for x in g["A"][0]], np.int64)
    b = np.array([int(x) for x in g["B"][0]], np.int64)
    keys = np.concatenate([a, b])
    vals = np.arange(len(keys), dtype=np.uint32)
    k, v = oracle.merge_kv(keys, vals, len(a))
    exp = [t.split(":") for t in g["C"][0]]
    assert k.tolist() == [int(t[0]) for t in exp]
    assert v.tolist() == [int(t[2]) + (0 if t[1] == "A" else len(a)) for t in exp]
    assert oracle.corank(a, b, range(len(keys) + 1)).tolist() == [int(x) for x in g["I"][0]]


def test_golden_ls_trace():
    g = _read("ls_trace.txt")
    start = np.array([int(x) for x in g["START"][0]])
    final = [int(x) for x in g["STEP"][-1]]
    res, swaps = oracle.rotate_ls(start, 2)
    assert res.tolist() == final
    assert swaps == int(g["SWAPS"][0][0])
    assert oracle.rotate(start, 2).tolist() == final


def test_golden_cs_cycle():
    g = _read("cs_cycle.txt")
    la, lb = int(g["LA"][0][0]), int(g["LB"][0][0])
    # the recurrence of the proof, written out
    seq, i = [], 0
    while True:
        seq.append(i)
        i = i + lb if i < la else i - la
        if i == 0:
            break
    assert seq == [int(x) for x in g["CYCLE"][0]]
    res, cycles, moves = oracle.rotate_cs(np.arange(la + lb), la)
    assert cycles == int(g["CYCLES"][0][0]) and moves == int(g["MOVES"][0][0])
    assert res.tolist() == list(range(la, la + lb)) + list(range(la))


def test_rotation_counts_exhaustive():
    for lx in range(0, 41):
        for ly in range(0, 41):
            x = np.arange(lx + ly) * 3 + 1
            want = np.concatenate([x[lx:], x[:lx]])
            assert np.array_equal(oracle.rotate(x, lx), want)
            r_ls, swaps = oracle.rotate_ls(x, lx)
            assert np.array_equal(r_ls, want)
            r_cs, cyc, mov = oracle.rotate_cs(x, lx)
            assert np.array_equal(r_cs, want)
            if lx and ly:
                g = math.gcd(lx, ly)
                assert swaps == lx + ly - g
                assert cyc == g                       # gcd cycles, not lcm
                assert mov == lx + ly                 # every element moved once
                if lx == ly:
                    assert swaps == lx                # exactly L_A swaps when equal
            else:
                assert swaps == 0 and cyc == 0 and mov == 0


def test_corank_properties_random():
    rng = np.random.default_rng(11)
    for _ in range(40):
        la, lb = rng.integers(0, 500, size=2)
        hi = int(rng.choice([2, 50, 10 ** 6]))
        a = np.sort(rng.integers(0, hi, la)).astype(np.int32)
        b = np.sort(rng.integers(0, hi, lb)).astype(np.int32)
        ks = np.arange(la + lb + 1)
        i = oracle.corank(a, b, ks)
        assert i[0] == 0 and i[-1] == la
        d = np.diff(i)
        assert set(np.unique(d).tolist()) <= {0, 1}
        # i(k) is the count of A among the first k of the brute-force merge
        ref = brute_merge(a, b)
        src = np.array([t[1] for t in ref])
        assert np.array_equal(i[1:], np.cumsum(src == 0))
        # any order of diagonals is accepted
        perm = rng.permutation(ks)
        assert np.array_equal(oracle.corank(a, b, perm), i[perm])


def test_mlp_gradient_finite_differences():
    m = oracle.MLP64(32)
    rng = np.random.default_rng(3)
    theta = rng.normal(0, 0.5, 97)
    x = rng.uniform(0, 1, 64)
    t = rng.uniform(0, 1, 64)
    g = m.grad(theta, x, t)
    h = 1e-6
    fd = np.empty_like(theta)
    for j in range(theta.size):
        e = np.zeros_like(theta)
        e[j] = h
        fd[j] = (m.loss(theta + e, x, t) - m.loss(theta - e, x, t)) / (2 * h)
    # kinks of ReLU are measure zero for random draws
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_mlp_forward_special_cases():
    m = oracle.MLP64(32)
    theta = np.zeros(97)
    theta[96] = 0.25
    assert np.allclose(m.forward(theta, [0.0, 0.5, 1.0]), 0.25)   # only b2
    theta = np.zeros(97)
    theta[0] = 2.0          # w1[0]
    theta[32] = -0.5        # b1[0]: hinge at x = 0.25
    theta[64] = 3.0         # w2[0]
    y = m.forward(theta, [0.0, 0.25, 1.0])
    assert np.allclose(y, [0.0, 0.0, 3.0 * (2.0 - 0.5)])


def test_adam_first_step_closed_form():
    # with zero moments, the bias-corrected first step is -lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.zeros(4)
    new, mo, ve = oracle.MLP64.adam_step(th, g, np.zeros(4), np.zeros(4), 1, lr=0.1)
    assert np.allclose(new, -0.1 * g / (np.abs(g) + 1e-8))
    assert np.allclose(mo, 0.1 * g) and np.allclose(ve, 0.001 * g * g)


# ------------------------------------------------------------- FindMedian
def _fm_cases():
    cases, cur = [], None
    for line in open(os.path.join(GOLD, "findmedian_trace.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "CASE":
            ib = f.index("B")
            cur = (np.array(f[2:ib], dtype=np.int64), np.array(f[ib + 1:], dtype=np.int64))
        elif f[0] == "RESULT":
            cases.append((cur[0], cur[1], (int(f[1]), int(f[2]))))
    return cases


def test_golden_findmedian_trace():
    cases = _fm_cases()
    assert len(cases) == 4
    for a, b, want in cases:
        assert oracle.find_median(a, b) == want


def _fm_valid(a, b, pa, pb):
    # Sec. 3.3: A0 <= B1 and B0 <= A1 (every element of the left halves is at
    # most every element of the right halves)
    if not (0 <= pa <= a.size and 0 <= pb <= b.size):
        return False
    if pa > 0 and pb < b.size and a[pa - 1] > b[pb]:
        return False
    if pb > 0 and pa < a.size and b[pb - 1] > a[pa]:
        return False
    return True


def test_findmedian_valid_exhaustive_small():
    # every pair of sorted runs of length <= 5 over keys {0, 1, 2, 3}
    runs = [np.array(c, dtype=np.int32) for n in range(6)
            for c in itertools.combinations_with_replacement(range(4), n)]
    for a in runs:
        for b in runs:
            pa, pb = oracle.find_median(a, b)
            assert _fm_valid(a, b, pa, pb), (a, b, pa, pb)


def test_findmedian_special_cases_and_interleaved():
    r = np.random.default_rng(5)
    for _ in range(200):
        la, lb = r.integers(1, 50, size=2)
        a = np.sort(r.integers(0, 100, la)).astype(np.int64)
        b = np.sort(r.integers(100, 200, lb)).astype(np.int64)
        assert oracle.find_median(a, b) == (la, 0)       # A before B
        assert oracle.find_median(b, a) == (0, la)       # B before A
    # equal-length perfectly interleaved runs: the split is exactly balanced
    for n in range(1, 200):
        a = np.arange(n, dtype=np.int64) * 2
        b = a + 1
        pa, pb = oracle.find_median(a, b)
        assert pa + pb == n and _fm_valid(a, b, pa, pb)


def test_divide_pairs_merge_to_sorted():
    # the pairs of either division, merged one by one and concatenated, give
    # the sorted input (keys); the co-rank division is balanced to one element
    r = np.random.default_rng(6)
    for trial in range(20):
        la, lb = r.integers(0, 3000, size=2)
        hi = 20 if trial % 2 else 2 ** 31
        a = np.sort(r.integers(0, hi, la)).astype(np.int32)
        b = np.sort(r.integers(0, hi, lb)).astype(np.int32)
        want = np.sort(np.concatenate([a, b]))
        for method in ("corank", "findmedian"):
            for depth in (1, 3, 5):
                sizes = oracle.divide(a, b, depth, method)
                assert sizes.shape == (2 ** depth, 2)
                assert sizes[:, 0].sum() == la and sizes[:, 1].sum() == lb
                ao = np.concatenate([[0], np.cumsum(sizes[:, 0])])
                bo = np.concatenate([[0], np.cumsum(sizes[:, 1])])
                parts = []
                for p in range(2 ** depth):
                    pa, pb = a[ao[p]:ao[p + 1]], b[bo[p]:bo[p + 1]]
                    parts.append(oracle.merge(np.concatenate([pa, pb]), pa.size))
                got = np.concatenate(parts) if parts else np.zeros(0, np.int32)
                assert np.array_equal(got, want), (method, depth)
                if method == "corank":
                    tot = sizes.sum(axis=1)
                    assert tot.max() - tot.min() <= 1


def test_merge_par_equals_merge():
    r = np.random.default_rng(7)
    for n, la in [(0, 0), (1, 1), (10, 3), (100001, 40000), (300000, 150000)]:
        d = r.integers(0, 1000, n).astype(np.int64)
        d[:la].sort()
        d[la:].sort()
        got, threads = oracle.merge_par(d, la)
        assert threads >= 1
        assert np.array_equal(got, oracle.merge(d, la))
    # cuts that fall inside runs of equal keys, and every B before every A:
    # each thread's own bisection must agree with the stable order
    for d, la in [(np.zeros(100003, np.int64), 50000),
                  (np.concatenate([np.arange(5000, 9000), np.arange(0, 5000)]).astype(np.int64), 4000)]:
        got, _ = oracle.merge_par(d, la)
        assert np.array_equal(got, oracle.merge(d, la))


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.int64, np.uint64])
def test_merge_rows_brute(dt):
    # wide elements (Sec. 4: the key is the first word of each element): the
    # stable merge of rows by their first column, by brute force; payload
    # words must travel with their key
    rng = np.random.default_rng(17)
    for _ in range(200):
        la, lb = (int(x) for x in rng.integers(0, 25, size=2))
        w = int(rng.integers(1, 6))
        a = np.sort(rng.integers(0, 5, la)).astype(dt)
        b = np.sort(rng.integers(0, 5, lb)).astype(dt)
        rows = rng.integers(0, 1000, size=(la + lb, w)).astype(dt)
        rows[:, 0] = np.concatenate([a, b])
        got = oracle.merge_rows(rows, la)
        ref = brute_merge(a, b)
        want = np.array([rows[t[2] + (0 if t[1] == 0 else la)] for t in ref],
                        dtype=dt).reshape(la + lb, w)
        assert np.array_equal(got, want)
    # the input is not modified; a single column is the plain merge
    x = np.array([[3], [7], [1], [9]], dtype=dt)
    assert np.array_equal(oracle.merge_rows(x, 2)[:, 0], oracle.merge(x[:, 0].copy(), 2))
    assert x[:, 0].tolist() == [3, 7, 1, 9]


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_sort_keys_equals_bottom_up_merges(dt):
    # the merge-sort driver's result (the sorted input) equals a bottom-up
    # merge sort built from the oracle's own stable merge: runs of width w
    # merged pairwise, the unpaired last run carried over, w doubling (the
    # passes of the library's sort, Q17), so each pins the other; also
    # sortedness and the same multiset
    rng = np.random.default_rng(23)
    for n in (0, 1, 2, 3, 7, 64, 1000, 4099):
        for hi in (4, 2 ** 31):
            x = rng.integers(0, hi, n).astype(dt)
            y = x.copy()
            w = 1
            while w < n:
                for o in range(0, n, 2 * w):
                    e = min(o + 2 * w, n)
                    if o + w < e:
                        y[o:e] = oracle.merge(y[o:e].copy(), w)
                w *= 2
            s = oracle.sort_keys(x)
            assert np.array_equal(s, y), (n, hi)
            assert np.all(s[1:] >= s[:-1])
            assert sorted(s.tolist()) == sorted(x.tolist())
