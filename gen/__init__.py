"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds none of the merge's arithmetic: only random draws and sorting of each run
(numpy, host memory).  Both the HIP path and the CPU oracle consume these
arrays; neither produces them.

Workloads (sizes and distributions of the target configurations):
  * ``uniform``   -- int32 runs, each drawn uniform in [0, 2^31) and sorted
                     (2^16 + 2^16; 2^27 + 2^27; skewed 2^23 + (2^27 - 2^23)).
  * ``dup``       -- int32 keys uniform in [0, 1024): heavy ties.
  * ``kv``        -- int64 keys uniform in [0, 4096), uint32 payload = index in
                     the concatenated A|B after each run is sorted.
  * ``batch``     -- n instances, L_A and L_B each round(2^U), U ~ U[6, 20],
                     int32 uniform keys, packed, int64 offsets[2n+1].
  * ``unsorted``  -- int32 uniform, unsorted (merge-sort input).
  * ``learned``   -- int64, A = floor(lognormal(mu=20, sigma=2)), B = a
                     16-component Gaussian mixture (equal weights, means
                     uniform in [0, 2^40), sigma 2^30), both clipped at 0,
                     sorted.
  * ``paper_w1``  -- the paper's own generator (Sec. 4, test cases):
                     a[0] = 0, a[i] = a[i-1] + 5 * rand01(); int32 by floor.
  * ``rows``      -- wide elements (Sec. 4 test cases: elements of several
                     bytes compared on their first word): an (n, w) array whose
                     column 0 holds each run's sorted keys (uniform in [0, hi),
                     or the W1 walk) and whose other words are uniform payload.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 12648


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def sorted_uniform(n: int, lo: int, hi: int, seed: int, dtype=np.int32) -> np.ndarray:
    r = _rng(seed)
    x = r.integers(lo, hi, size=n, dtype=np.int64).astype(dtype)
    x.sort(kind="stable")
    return x


def pair_uniform(la: int, lb: int, seed: int, hi: int = 2 ** 31, dtype=np.int32) -> np.ndarray:
    """A|B: two independent sorted runs uniform in [0, hi)."""
    a = sorted_uniform(la, 0, hi, seed, dtype)
    b = sorted_uniform(lb, 0, hi, seed + 1_000_003, dtype)
    return np.concatenate([a, b])


def pair_dup(la: int, lb: int, seed: int) -> np.ndarray:
    return pair_uniform(la, lb, seed, hi=1024)


def pair_kv(la: int, lb: int, seed: int, key_hi: int = 4096):
    keys = pair_uniform(la, lb, seed, hi=key_hi, dtype=np.int64)
    vals = np.arange(la + lb, dtype=np.uint32)
    return keys, vals


def batch(n_inst: int, seed: int, lo_exp: float = 6.0, hi_exp: float = 20.0,
          dtype=np.int32):
    """Packed instances and offsets[2n+1] (host arrays)."""
    r = _rng(seed)
    la = np.rint(2.0 ** r.uniform(lo_exp, hi_exp, size=n_inst)).astype(np.int64)
    lb = np.rint(2.0 ** r.uniform(lo_exp, hi_exp, size=n_inst)).astype(np.int64)
    off = np.zeros(2 * n_inst + 1, dtype=np.int64)
    off[1::2] = la
    off[2::2] = lb
    off = np.cumsum(off)
    total = int(off[-1])
    data = r.integers(0, 2 ** 31, size=total, dtype=np.int64).astype(dtype)
    for q in range(n_inst):
        data[off[2 * q]:off[2 * q + 1]].sort()
        data[off[2 * q + 1]:off[2 * q + 2]].sort()
    return data, off


def unsorted(n: int, seed: int, dtype=np.int32) -> np.ndarray:
    return _rng(seed).integers(0, 2 ** 31, size=n, dtype=np.int64).astype(dtype)


def pair_learned(la: int, lb: int, seed: int) -> np.ndarray:
    r = _rng(seed)
    a = np.floor(np.clip(r.lognormal(mean=20.0, sigma=2.0, size=la), 0, 2.0 ** 62)).astype(np.int64)
    means = r.uniform(0.0, 2.0 ** 40, size=16)
    comp = r.integers(0, 16, size=lb)
    b = r.normal(loc=means[comp], scale=2.0 ** 30)
    b = np.floor(np.clip(b, 0, 2.0 ** 62)).astype(np.int64)
    a.sort()
    b.sort()
    return np.concatenate([a, b])


def paper_w1(n: int, seed: int) -> np.ndarray:
    """Sec. 4 generator: running sum of 5 * U[0,1) increments, floored to int32."""
    r = _rng(seed)
    inc = r.random(n) * 5.0
    inc[0] = 0.0
    return np.floor(np.cumsum(inc)).astype(np.int32)


def paper_w1_pair(n: int, split: float, seed: int) -> np.ndarray:
    la = int(n * split)
    a = paper_w1(la, seed)
    b = paper_w1(n - la, seed + 7)
    return np.concatenate([a, b])


# Named configurations (sizes of the target workloads).
CONFIGS = {
    "c1": dict(kind="uniform", la=2 ** 16, lb=2 ** 16, seed=SEED_BASE + 10),
    "c2": dict(kind="uniform", la=2 ** 27, lb=2 ** 27, seed=SEED_BASE + 20),
    "c2_skew": dict(kind="uniform", la=2 ** 23, lb=2 ** 27 - 2 ** 23, seed=SEED_BASE + 21),
    "c2_dup": dict(kind="dup", la=2 ** 27, lb=2 ** 27, seed=SEED_BASE + 22),
    "c3": dict(kind="kv", la=2 ** 26, lb=2 ** 26, seed=SEED_BASE + 30),
    "c4_batch": dict(kind="batch", n=4096, seed=SEED_BASE + 40),
    "c4_sort": dict(kind="unsorted", n=2 ** 28, seed=SEED_BASE + 41),
    "c5": dict(kind="learned", la=2 ** 28, lb=2 ** 28, seed=SEED_BASE + 50),
}


def make(name: str, scale: int = 0):
    """Inputs of a named configuration; ``scale`` > 0 divides every length by
    2**scale (same distributions, smaller sizes) for quick tests."""
    c = dict(CONFIGS[name])
    kind = c.pop("kind")
    d = 2 ** scale
    if kind == "uniform":
        return pair_uniform(max(c["la"] // d, 1), max(c["lb"] // d, 1), c["seed"]), max(c["la"] // d, 1)
    if kind == "dup":
        return pair_dup(max(c["la"] // d, 1), max(c["lb"] // d, 1), c["seed"]), max(c["la"] // d, 1)
    if kind == "kv":
        la, lb = max(c["la"] // d, 1), max(c["lb"] // d, 1)
        k, v = pair_kv(la, lb, c["seed"])
        return (k, v), la
    if kind == "batch":
        hi = 20.0 - scale
        return batch(max(c["n"] // d, 1), c["seed"], 6.0, max(hi, 6.5))
    if kind == "unsorted":
        return unsorted(max(c["n"] // d, 1), c["seed"])
    if kind == "learned":
        la, lb = max(c["la"] // d, 1), max(c["lb"] // d, 1)
        return pair_learned(la, lb, c["seed"]), la
    raise KeyError(name)


# --------------------------------------------------------------------------
# Device-side generators (same distributions, drawn with torch's seeded
# generator on the GPU so full-size benchmark inputs take milliseconds).
# Values differ from the numpy draws above; both are seeded and synthetic.
# --------------------------------------------------------------------------
def rows_pair(la: int, lb: int, words: int, seed: int, hi: int = 2 ** 31, dtype=np.int32,
              keys: np.ndarray | None = None) -> np.ndarray:
    """(la+lb, words) rows: column 0 = sorted keys of A then of B (uniform in
    [0, hi), or the given A|B keys), other columns uniform payload."""
    if keys is None:
        keys = pair_uniform(la, lb, seed, hi=hi, dtype=dtype)
    r = _rng(seed + 7)
    rows = r.integers(0, 2 ** 31, size=(la + lb, words), dtype=np.int64).astype(dtype)
    rows[:, 0] = keys.astype(dtype)
    return rows


def torch_rows_pair(la: int, lb: int, words: int, seed: int, device, dtype=None):
    """Device form of rows_pair (keys uniform in [0, 2^31))."""
    import torch
    dtype = dtype or torch.int32
    g = _tgen(seed + 7, device)
    rows = torch.randint(0, 2 ** 31, (la + lb, words), generator=g, device=device,
                         dtype=torch.int64).to(dtype)
    rows[:, 0] = torch_pair_uniform(la, lb, seed, device, dtype=dtype)
    return rows


def _tgen(seed: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def torch_sorted_uniform(n: int, hi: int, seed: int, device, dtype=None):
    import torch
    dtype = dtype or torch.int32
    g = _tgen(seed, device)
    x = torch.randint(0, hi, (n,), generator=g, device=device, dtype=torch.int64)
    return torch.sort(x.to(dtype)).values


def torch_pair_uniform(la: int, lb: int, seed: int, device, hi: int = 2 ** 31, dtype=None):
    import torch
    a = torch_sorted_uniform(la, hi, seed, device, dtype)
    b = torch_sorted_uniform(lb, hi, seed + 1_000_003, device, dtype)
    return torch.cat([a, b])


def torch_unsorted(n: int, seed: int, device, dtype=None):
    import torch
    g = _tgen(seed, device)
    return torch.randint(0, 2 ** 31, (n,), generator=g, device=device,
                         dtype=torch.int64).to(dtype or torch.int32)


def torch_batch(n_inst: int, seed: int, device, lo_exp: float = 6.0, hi_exp: float = 20.0):
    """Packed int32 instances (each run sorted) and int64 offsets[2n+1], on device."""
    import torch
    r = _rng(seed)
    la = np.rint(2.0 ** r.uniform(lo_exp, hi_exp, size=n_inst)).astype(np.int64)
    lb = np.rint(2.0 ** r.uniform(lo_exp, hi_exp, size=n_inst)).astype(np.int64)
    off = np.zeros(2 * n_inst + 1, dtype=np.int64)
    off[1::2] = la
    off[2::2] = lb
    off = np.cumsum(off)
    total = int(off[-1])
    g = _tgen(seed + 1, device)
    vals = torch.randint(0, 2 ** 31, (total,), generator=g, device=device, dtype=torch.int64)
    # sort every run at once: run index in the high bits, value in the low 31
    run_len = torch.from_numpy(np.diff(off)).to(device)
    run_id = torch.repeat_interleave(torch.arange(2 * n_inst, device=device), run_len)
    key = torch.sort((run_id << 31) | vals).values
    data = (key & (2 ** 31 - 1)).to(torch.int32)
    return data, torch.from_numpy(off).to(device), off


def torch_pair_learned(la: int, lb: int, seed: int, device):
    import torch
    g = _tgen(seed, device)
    a = torch.empty(la, dtype=torch.float64, device=device).log_normal_(20.0, 2.0, generator=g)
    r = _rng(seed)
    means = torch.from_numpy(r.uniform(0.0, 2.0 ** 40, size=16)).to(device)
    comp = torch.randint(0, 16, (lb,), generator=g, device=device)
    b = torch.normal(means[comp], 2.0 ** 30, generator=g)
    a = torch.floor(torch.clamp(a, 0, 2.0 ** 62)).to(torch.int64)
    b = torch.floor(torch.clamp(b, 0, 2.0 ** 62)).to(torch.int64)
    return torch.cat([torch.sort(a).values, torch.sort(b).values])
