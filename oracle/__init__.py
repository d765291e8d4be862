"""CPU oracle for the parallel in-place merge of Bramas & Bramas (arXiv 2005.12648).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2005_12648_amd/`` and never imports it.

Contents and the passage each one follows:

* :func:`merge`, :func:`merge_kv` -- the problem statement (Sec. 1): two sorted
  runs A|B become one sorted run.  Stable reading: ties take A first (the
  per-pair ``std::inplace_merge`` of Alg. 2/3 is stable).  Plain two-finger
  merge in C (``oracle.c``), out of place, copied back.
* :func:`merge_rows` -- the same stable merge for wide elements (Sec. 4 test
  cases: elements of several bytes compared on their first bytes): the rows
  are ordered by the key in their first column, ties take A, and each row
  moves whole.  The order comes from :func:`merge_kv` on (key, row index).
* :func:`corank` -- number of A elements among the first k merged outputs: the
  "optimal" split of Sec. 3.1 for an arbitrary output rank, by walking the merge.
* :func:`rotate`, :func:`rotate_ls`, :func:`rotate_cs` -- the partition exchange
  X|Y -> Y|X of Sec. 3.4: the definition, linear shifting with its swap counter
  and circular shifting with its cycle/move counters (Sec. 3.4 proof, Sec. 3.5).
* :func:`sort_keys` -- the merge-sort driver's result is the sorted input; the
  library sort is the definition.
* :func:`find_median` -- FindMedian, Alg. 1 (Sec. 3.3), step by step, with the
  reading of its garbled loop stated in ``oracle.c``.
* :func:`divide` -- the recursive division of Sec. 3 (as Alg. 3 recurses on
  A0|B0 and A1|B1) down to 2^depth pairs, with FindMedian or the exact co-rank
  at the middle rank as the split; returns the pair sizes.  No data moves: the
  pairs are ranges of the original A and B.
* :func:`merge_par` -- the stable merge on all host cores (timing only).
* :class:`MLP64` -- fp64 forward pass, MSE loss, closed-form gradients and one
  Adam step of the 1->32->1 ReLU network used to predict co-ranks.  The paper
  has no learned component: input x = k/N, target t = i(k)/L_A, mean squared
  error and Adam are this project's own choices.

Parity status: merge, co-rank and rotation are pinned by brute force and by the
paper's proven counts (tests/test_oracle_pins.py).  The MLP gradients are pinned
by central finite differences; trained weights are "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no HIP headers involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        vp = ctypes.c_void_p
        for t in ("i32", "u32", "i64", "u64"):
            f = getattr(lib, "orc_merge_" + t)
            f.argtypes = [vp, i64, i64]
            f.restype = ctypes.c_int
            f = getattr(lib, "orc_merge_kv_" + t)
            f.argtypes = [vp, vp, i64, i64, i64]
            f.restype = ctypes.c_int
            f = getattr(lib, "orc_corank_" + t)
            f.argtypes = [vp, i64, vp, i64, vp, i64, vp]
            f.restype = None
            f = getattr(lib, "orc_find_median_" + t)
            f.argtypes = [vp, i64, vp, i64, vp, vp]
            f.restype = None
            f = getattr(lib, "orc_merge_par_" + t)
            f.argtypes = [vp, i64, i64]
            f.restype = ctypes.c_int
        lib.orc_rotate_def.argtypes = [vp, i64, i64]
        lib.orc_rotate_def.restype = ctypes.c_int
        lib.orc_rotate_ls.argtypes = [vp, i64, i64]
        lib.orc_rotate_ls.restype = i64
        lib.orc_rotate_cs.argtypes = [vp, i64, i64, vp, vp]
        lib.orc_rotate_cs.restype = ctypes.c_int
        _lib = lib
    return _lib


_SUFFIX = {np.dtype(np.int32): "i32", np.dtype(np.uint32): "u32",
           np.dtype(np.int64): "i64", np.dtype(np.uint64): "u64"}


def _suffix(arr: np.ndarray) -> str:
    try:
        return _SUFFIX[arr.dtype]
    except KeyError:
        raise TypeError("oracle: unsupported key dtype %s" % arr.dtype) from None


def merge(data: np.ndarray, la: int) -> np.ndarray:
    """Stable merge of the sorted runs data[:la] and data[la:] (ties take A).

    Returns a new array; ``data`` is not modified."""
    out = np.ascontiguousarray(data).copy()
    n = out.shape[0]
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    rc = getattr(_load(), "orc_merge_" + _suffix(out))(out.ctypes.data, la, n - la)
    if rc != 0:
        raise MemoryError("oracle merge: allocation failed")
    return out


def merge_kv(keys: np.ndarray, vals: np.ndarray, la: int):
    """Stable key+payload merge: keys decide, payloads follow, ties take A."""
    k = np.ascontiguousarray(keys).copy()
    v = np.ascontiguousarray(vals).copy()
    n = k.shape[0]
    if v.shape[0] != n or not 0 <= la <= n:
        raise ValueError("shape mismatch")
    rc = getattr(_load(), "orc_merge_kv_" + _suffix(k))(
        k.ctypes.data, v.ctypes.data, v.dtype.itemsize, la, n - la)
    if rc != 0:
        raise MemoryError("oracle merge_kv: allocation failed")
    return k, v


def merge_rows(rows: np.ndarray, la: int) -> np.ndarray:
    """Stable merge of the rows of a 2-D array: rows[:la] and rows[la:] are
    ascending by column 0; ties take A; rows move whole (Sec. 4 elements)."""
    r = np.ascontiguousarray(rows)
    if r.ndim != 2 or not 0 <= la <= r.shape[0]:
        raise ValueError("shape mismatch")
    idx = np.arange(r.shape[0], dtype=np.uint64)
    _, order = merge_kv(r[:, 0].copy(), idx, la)
    return r[order.astype(np.int64)]


def corank(a: np.ndarray, b: np.ndarray, ks) -> np.ndarray:
    """i(k) for each k in ``ks``: how many A elements are among the first k
    outputs of the stable merge of a and b.  Any order of ks is accepted."""
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    if a.dtype != b.dtype:
        raise TypeError("a and b must share a dtype")
    ks = np.asarray(ks, dtype=np.int64)
    order = np.argsort(ks, kind="stable")
    sk = np.ascontiguousarray(ks[order])
    if sk.size and (sk[0] < 0 or sk[-1] > a.size + b.size):
        raise ValueError("diagonal out of range")
    res = np.empty(sk.size, dtype=np.int64)
    getattr(_load(), "orc_corank_" + _suffix(a))(
        a.ctypes.data, a.size, b.ctypes.data, b.size, sk.ctypes.data, sk.size, res.ctypes.data)
    out = np.empty_like(res)
    out[order] = res
    return out


def rotate(x: np.ndarray, lx: int) -> np.ndarray:
    """Definition of the partition exchange: X|Y -> Y|X (int64 buffer)."""
    d = np.ascontiguousarray(x, dtype=np.int64).copy()
    _load().orc_rotate_def(d.ctypes.data, lx, d.size - lx)
    return d


def rotate_ls(x: np.ndarray, lx: int):
    """Linear shifting (Sec. 3.4).  Returns (result, element swaps)."""
    d = np.ascontiguousarray(x, dtype=np.int64).copy()
    swaps = _load().orc_rotate_ls(d.ctypes.data, lx, d.size - lx)
    return d, int(swaps)


def rotate_cs(x: np.ndarray, lx: int):
    """Circular shifting (Sec. 3.4).  Returns (result, cycles, moves)."""
    d = np.ascontiguousarray(x, dtype=np.int64).copy()
    cyc = ctypes.c_int64(0)
    mov = ctypes.c_int64(0)
    _load().orc_rotate_cs(d.ctypes.data, lx, d.size - lx, ctypes.byref(cyc), ctypes.byref(mov))
    return d, int(cyc.value), int(mov.value)


def merge_par(data: np.ndarray, la: int):
    """merge() computed by all host cores; returns (result, threads used)."""
    out = np.ascontiguousarray(data).copy()
    n = out.shape[0]
    if not 0 <= la <= n:
        raise ValueError("la out of range")
    rc = getattr(_load(), "orc_merge_par_" + _suffix(out))(out.ctypes.data, la, n - la)
    if rc < 0:
        raise MemoryError("oracle merge_par: allocation failed")
    return out, int(rc)


def find_median(a: np.ndarray, b: np.ndarray):
    """FindMedian (Alg. 1) of the sorted runs a and b: returns (p_A, p_B)."""
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    if a.dtype != b.dtype:
        raise TypeError("a and b must share a dtype")
    pa = ctypes.c_int64(0)
    pb = ctypes.c_int64(0)
    getattr(_load(), "orc_find_median_" + _suffix(a))(
        a.ctypes.data, a.size, b.ctypes.data, b.size, ctypes.byref(pa), ctypes.byref(pb))
    return int(pa.value), int(pb.value)


def divide(a: np.ndarray, b: np.ndarray, depth: int, method: str = "corank"):
    """Split (a, b) recursively into 2**depth pairs (A_p, B_p), in order.

    method "corank": the exact split at the middle rank floor((|A|+|B|)/2)
    (ties take A); "findmedian": Alg. 1.  Returns an int64 array of shape
    (2**depth, 2) holding (|A_p|, |B_p|)."""
    if method not in ("corank", "findmedian"):
        raise ValueError("method")
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    nodes = [(0, a.size, 0, b.size)]            # (a_off, la, b_off, lb)
    for _ in range(depth):
        nxt = []
        for ao, la, bo, lb in nodes:
            sa, sb = a[ao:ao + la], b[bo:bo + lb]
            if method == "corank":
                k = (la + lb) // 2
                i = int(corank(sa, sb, [k])[0]) if la + lb > 0 else 0
                j = k - i
            else:
                i, j = find_median(sa, sb) if la + lb > 0 else (0, 0)
            nxt.append((ao, i, bo, j))
            nxt.append((ao + i, la - i, bo + j, lb - j))
        nodes = nxt
    return np.array([(la, lb) for _, la, _, lb in nodes], dtype=np.int64)


def sort_keys(x: np.ndarray) -> np.ndarray:
    """Result of the in-place merge sort driver: the sorted input."""
    return np.sort(np.asarray(x), kind="stable")


# --------------------------------------------------------------------------
# fp64 reference of the 1 -> H -> 1 ReLU network that predicts co-ranks.
# Parameter vector layout (shared by convention with the device kernels, not
# by code): [w1 (H), b1 (H), w2 (H), b2 (1)].
# --------------------------------------------------------------------------
class MLP64:
    """y(x) = sum_h w2[h] * relu(w1[h] * x + b1[h]) + b2, loss = mean((y - t)^2)."""

    def __init__(self, hidden: int = 32):
        self.H = hidden

    def unpack(self, theta):
        H = self.H
        th = np.asarray(theta, dtype=np.float64)
        if th.size != 3 * H + 1:
            raise ValueError("expected %d parameters" % (3 * H + 1))
        return th[:H], th[H:2 * H], th[2 * H:3 * H], th[3 * H]

    def forward(self, theta, x):
        w1, b1, w2, b2 = self.unpack(theta)
        x = np.asarray(x, dtype=np.float64)
        z = np.outer(x, w1) + b1            # (M, H) pre-activation
        h = np.maximum(z, 0.0)              # ReLU
        return h @ w2 + b2

    def loss(self, theta, x, t):
        y = self.forward(theta, x)
        r = y - np.asarray(t, dtype=np.float64)
        return float(np.mean(r * r))

    def grad(self, theta, x, t):
        """Closed-form gradient of the mean squared error."""
        w1, b1, w2, b2 = self.unpack(theta)
        x = np.asarray(x, dtype=np.float64)
        t = np.asarray(t, dtype=np.float64)
        m = x.size
        z = np.outer(x, w1) + b1
        h = np.maximum(z, 0.0)
        y = h @ w2 + b2
        dy = 2.0 * (y - t) / m              # d loss / d y
        g_w2 = h.T @ dy
        g_b2 = dy.sum()
        dz = np.outer(dy, w2) * (z > 0.0)   # ReLU derivative (0 at z == 0)
        g_w1 = dz.T @ x
        g_b1 = dz.sum(axis=0)
        return np.concatenate([g_w1, g_b1, g_w2, [g_b2]])

    @staticmethod
    def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam update (Kingma & Ba, Alg. 1); ``step`` counts from 1."""
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** step)
        vhat = v / (1.0 - beta2 ** step)
        return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
