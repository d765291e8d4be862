#!/usr/bin/env python3
"""Benchmark of the MI355X in-place merge (one GPU).

A step is one whole in-place merge -- division levels, tile co-ranks and the
leaf merge -- of int32 runs L_A = L_B = 2^27 (uniform in [0, 2^31), each run
sorted), the input already resident in HBM.  The merge works in place, so the
K timed steps run on K separate copies of the input prepared before the timed
region; nothing is restored inside it.

Printed on stdout: ONE JSON line with the headline (Gelem/s), the roofline of
the dominant kernel (per-stage HIP events recorded on the merge's stream over
the timed region), the CPU oracle timed on this host's cores, and the other
forms side by side (batched merge of 4096 instances vs 4096 plain calls,
in-place merge sort of 2^28 int32, learned split vs plain on int64 2^28+2^28,
key+payload, skewed and duplicate-heavy variants, the paper's FindMedian and
circular shifting, out-of-place comparators, and rows of 64 B to 64 KiB).  Every GPU result is
compared with the CPU oracle; mismatch counts are part of the line.
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
SEED = 12648


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def src_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# Sources whose change makes a committed counter summary stale: the kernel,
# the shared declarations, and the files that decide its launches and
# descriptors (plan, launch sequence, split kernel).
KERNEL_SOURCES = {
    "leafmerge": ["paper_2005_12648_amd/csrc/im_leaf.hip", "paper_2005_12648_amd/csrc/im_common.h",
                  "paper_2005_12648_amd/csrc/im_capi.hip", "paper_2005_12648_amd/csrc/im_split.hip"],
    "rotate": ["paper_2005_12648_amd/csrc/im_rotate.hip", "paper_2005_12648_amd/csrc/im_common.h",
               "paper_2005_12648_amd/csrc/im_capi.hip", "paper_2005_12648_amd/csrc/im_split.hip"],
    "split": ["paper_2005_12648_amd/csrc/im_split.hip", "paper_2005_12648_amd/csrc/im_search.h"],
    "tilerank": ["paper_2005_12648_amd/csrc/im_split.hip", "paper_2005_12648_amd/csrc/im_search.h"],
    # (leaf planning has no kernel of its own: leaves get their tiles where
    # the split kernel emits them)
    "plan": ["paper_2005_12648_amd/csrc/im_split.hip"],
}


def traffic_from_profile(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != src_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("hbm_bytes_per_launch")


def measured_hbm(ms: float):
    """HBM bytes of one headline merge as rocprofv3 counted them (FETCH_SIZE +
    WRITE_SIZE of the exchange and leaf-merge kernels, scaled by a plain copy
    of known size), over the merge time; None unless both counter summaries
    match the current kernel sources.  The split and co-rank kernels are left
    out (latency-bound searches, a few MB)."""
    total = 0.0
    for kernel in ("rotate", "leafmerge"):
        path = os.path.join(ROOT, "profiles", "traffic_%s_c2.json" % kernel)
        per = traffic_from_profile(kernel, "c2")
        if per is None:
            return None
        with open(path) as f:
            rec = json.load(f)
        total += rec["hbm_read_bytes_per_run"] + rec["hbm_write_bytes_per_run"]
    gbs = total / ms / 1e6
    return {"bytes_per_merge": int(total), "gb_s": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_elem": round(total / 2 ** 28, 2),
            "source": "profiles/traffic_rotate_c2.json + profiles/traffic_leafmerge_c2.json"}


class Timer:
    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def cpu_oracle_time(fn, budget_s: float):
    """Run the oracle until budget_s of wall time is spent (at least once)."""
    times, out = [], None
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        out = fn()
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start >= budget_s:
            break
    return out, float(np.median(times)), len(times)


def mismatches(got_t, want_np):
    got = got_t.cpu().numpy()
    return int(np.count_nonzero(got != want_np))


def timed_merges(torch, im, pristine, la, steps, warmup, fn=None, profile=False):
    """K merges on K prepared copies; returns (ms per step, stage profile, buffers)."""
    fn = fn or (lambda b: im.inplace_merge(b, la))
    bufs = [torch.empty_like(pristine) for _ in range(steps)]
    for _ in range(warmup):
        bufs[0].copy_(pristine)
        fn(bufs[0])
    for b in bufs:
        b.copy_(pristine)
    torch.cuda.synchronize()
    if profile:
        im.profile_read()          # drop anything recorded before
        im.profile(True)
    with Timer(torch) as t:
        for k in range(steps):
            fn(bufs[k])
    prof = None
    if profile:
        prof = im.profile_read()
        im.profile(False)
    return t.ms / steps, prof, bufs


def roofline(prof, stats, esize, steps, workload):
    """Dominant kernel by total time; algorithmic bytes per launch / avg launch time."""
    per_call = {
        # every leaf element is read once and written once
        "leafmerge": 2.0 * stats["leaf_elems"] * esize,
        # block swap: read + write each exchanged element once; three
        # reversals: twice
        "rotate": 2.0 * esize * (stats["rotated_elems"] + stats["reversed_elems"]),
        # two key loads per probe
        "split": 2.0 * esize * stats["search_probes"],
        "tilerank": 0.0,
        "plan": 0.0,
    }
    stage_ms = {k: v[0] for k, v in prof.items()}
    dom = max(stage_ms, key=lambda k: stage_ms[k])
    ms, launches = prof[dom]
    launches = max(int(launches), 1)
    avg_launch_ms = ms / launches
    bytes_per_launch = per_call[dom] * steps / launches
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(dom, workload)
    return {
        "kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic, "avg_launch_ms": round(avg_launch_ms, 5),
        "launches_per_step": launches / steps,
        "algorithmic_bytes_per_launch": bytes_per_launch,
        "stage_ms_per_step": {k: round(v / steps, 5) for k, v in stage_ms.items()},
    }


def bench_headline(torch, im, oracle, gen, dev, args):
    la = lb = 2 ** 27
    n = la + lb
    log("c2: generating int32 2^27 + 2^27 on the device")
    pristine = gen.torch_pair_uniform(la, lb, SEED + 20, dev)
    # leaf configuration chosen by the autotuner (outside the timed region)
    off1 = torch.tensor([0, la, n], dtype=torch.int64, device=dev)
    tune_ms = []
    if not args.no_tune:
        chosen, tune_ms = im.autotune(pristine, off1, reps=3)
        log("c2: autotune ms per config", ["%.3f" % m for m in tune_ms], "chosen", chosen)
    # the timed steps carry no stage events; a second pass with per-stage
    # events (which add small gaps between launches) feeds the roofline
    ms, _, bufs = timed_merges(torch, im, pristine, la, args.steps, args.warmup)
    log("c2: %.3f ms/step, %.1f Gelem/s" % (ms, n / ms / 1e6))
    ms_prof, prof, pbufs = timed_merges(torch, im, pristine, la, args.steps, 0, profile=True)
    stats = im.fetch_stats()
    del pbufs
    log("c2: profiled pass %.3f ms/step" % ms_prof)
    res = {"ms": ms, "prof": prof, "stats": stats, "n": n,
           "tune_ms": [round(m, 4) for m in tune_ms]}
    cpu = None
    if not args.no_cpu:
        host = pristine.cpu().numpy()
        half = args.cpu_seconds / 2
        log("c2: CPU oracle, single thread then all host cores, %.0f s each" % half)
        want, med_s, reps = cpu_oracle_time(lambda: oracle.merge(host, la), half)
        par_out = {}

        def run_par():
            r, th = oracle.merge_par(host, la)
            par_out["threads"] = th
            return r
        want_p, med_p, reps_p = cpu_oracle_time(run_par, half)
        cpu = {"value": round(n / med_p / 1e9, 4), "unit": "Gelem/s",
               "cores": par_out["threads"], "kind": "oracle",
               "sample": "full workload (int32 2^27+2^27), %d repetitions, median; the "
                         "oracle's all-cores stable merge (OpenMP: cuts at equal output "
                         "ranks, each thread bisects its own cut's co-rank and merges its "
                         "piece into a fresh buffer, parallel copy back; -O3)" % reps_p,
               "speedup_over_single_thread": round(med_s / med_p, 2),
               "single_thread_value": round(n / med_s / 1e9, 4),
               "single_thread_sample": "%d repetitions, median; two-finger merge into a "
                                       "fresh buffer + copy back" % reps,
               "host_cores_available": os.cpu_count()}
        if not np.array_equal(want, want_p):
            raise SystemExit("oracle all-cores merge differs from the single-thread merge")
        res["mismatch"] = mismatches(bufs[0], want) + mismatches(bufs[-1], want)
        log("c2: mismatches vs oracle:", res["mismatch"])
    res["cpu"] = cpu
    del bufs
    torch.cuda.empty_cache()
    return res


def bench_variant(torch, im, oracle, gen, dev, name, steps):
    """The small C1 merge, skewed / duplicate-heavy int32 and the key+payload form."""
    if name == "c3_kv":
        la = lb = 2 ** 26
        keys = gen.torch_pair_uniform(la, lb, SEED + 30, dev, hi=4096, dtype=torch.int64)
        vals = torch.arange(la + lb, dtype=torch.int32, device=dev).to(torch.uint32)
        kb = [keys.clone() for _ in range(steps)]
        vb = [vals.clone() for _ in range(steps)]
        with Timer(torch) as t:
            for k in range(steps):
                im.inplace_merge_kv(kb[k], vb[k], la)
        wk, wv = oracle.merge_kv(keys.cpu().numpy(), vals.cpu().numpy(), la)
        bad = mismatches(kb[0], wk) + mismatches(vb[0], wv)
        n = la + lb
        ms = t.ms / steps
        return {"workload": "int64 keys in [0,4096) + uint32 payload, 2^26+2^26",
                "gelem_s": round(n / ms / 1e6, 2), "ms": round(ms, 4), "mismatches": bad,
                "effective_gb_s": round(2 * 12 * n / ms / 1e6, 1)}
    if name == "c1":
        la, lb, hi, seed = 2 ** 16, 2 ** 16, 2 ** 31, SEED + 10
    elif name == "c2_skew":
        la, lb, hi, seed = 2 ** 23, 2 ** 27 - 2 ** 23, 2 ** 31, SEED + 21
    else:
        la, lb, hi, seed = 2 ** 27, 2 ** 27, 1024, SEED + 22
    pristine = gen.torch_pair_uniform(la, lb, seed, dev, hi=hi)
    # the small merge is launch-bound: time more of them
    ms, _, bufs = timed_merges(torch, im, pristine, la, 50 if name == "c1" else steps, 1)
    want = oracle.merge(pristine.cpu().numpy(), la)
    bad = mismatches(bufs[0], want)
    n = la + lb
    out = {"workload": "int32 %d+%d keys in [0,%d)" % (la, lb, hi), "gelem_s": round(n / ms / 1e6, 2),
           "ms": round(ms, 4), "mismatches": bad}
    if name == "c1":
        # the same merges through the division path (one-launch path off)
        os.environ["IM_SMALL"] = "0"
        try:
            ms_d, _, bufs_d = timed_merges(torch, im, pristine, la, 50, 1)
        finally:
            del os.environ["IM_SMALL"]
        out["one_launch_path"] = True
        out["division_path_ms"] = round(ms_d, 4)
        out["mismatches_division_path"] = mismatches(bufs_d[0], want)
    return out


def event_timed(torch, pristine, buf, fn, reps):
    """Median ms of fn() over reps runs, each on a fresh copy of pristine in buf
    (copies outside the timed events)."""
    ts = []
    for _ in range(reps):
        buf.copy_(pristine)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def bench_graph_single(torch, im, oracle, gen, dev, reps):
    """The headline merge captured once as a one-instance graph and replayed
    on fresh copies of its input, against the eager call on the same copies
    (events around each call, copies outside)."""
    la = lb = 2 ** 27
    log("c2 graph: generating int32 2^27 + 2^27 on the device")
    pristine = gen.torch_pair_uniform(la, lb, SEED + 20, dev)
    buf = torch.empty_like(pristine)
    off = torch.tensor([0, la, la + lb], dtype=torch.int64, device=dev)
    want = oracle.merge(pristine.cpu().numpy(), la)
    eager_ms = event_timed(torch, pristine, buf, lambda: im.inplace_merge(buf, la), reps)
    bad_eager = mismatches(buf, want)
    g = im.MergeGraph(buf, off)
    try:
        graph_ms = event_timed(torch, pristine, buf, g.launch, reps)
    finally:
        g.close()
    bad_graph = mismatches(buf, want)
    n = la + lb
    return {"workload": "int32 2^27+2^27 (the headline input), one-instance captured graph",
            "graph_ms": round(graph_ms, 4), "graph_gelem_s": round(n / graph_ms / 1e6, 2),
            "eager_ms": round(eager_ms, 4), "eager_gelem_s": round(n / eager_ms / 1e6, 2),
            "mismatches_graph": bad_graph, "mismatches_eager": bad_eager,
            "timing": "median of %d calls, HIP events around each call" % reps}


def bench_batched(torch, im, oracle, gen, dev, steps):
    log("c4: generating 4096 instances")
    data, off_d, off = gen.torch_batch(4096, SEED + 40, dev)
    total = int(off[-1])
    max_inst = int(np.max(off[2::2] - off[0:-1:2]))
    # autotuner: every leaf configuration timed on a copy, winner remembered
    chosen, tune_ms = im.autotune(data, off_d, max_instance=max_inst, reps=3)
    log("c4: autotune ms per config", ["%.3f" % m for m in tune_ms], "chosen", chosen)
    fn = lambda b: im.batched_inplace_merge(b, off_d, max_instance=max_inst)
    ms_b, _, bufs = timed_merges(torch, im, data, 0, steps, 1, fn=fn)
    used_cfg = im.fetch_stats()["leaf_config"]
    # the same merge recorded once in a HIP graph, replayed on fresh copies
    gbuf = data.clone()
    graph = im.MergeGraph(gbuf, off_d, max_instance=max_inst)
    coop = graph.cooperative
    event_timed(torch, data, gbuf, graph.launch, 1)                 # warm
    ms_g = event_timed(torch, data, gbuf, graph.launch, max(steps, 3))
    ebuf = data.clone()
    ms_e = event_timed(torch, data, ebuf, lambda: fn(ebuf), max(steps, 3))
    graph.launch()
    torch.cuda.synchronize()
    got_g = gbuf.cpu().numpy()
    graph.close()
    del gbuf, ebuf
    # the same 4096 instances as separate plain calls on one stream
    loop_buf = data.clone()

    def plain_loop(b):
        for q in range(4096):
            o0, o1, o2 = int(off[2 * q]), int(off[2 * q + 1]), int(off[2 * q + 2])
            im.inplace_merge(b[o0:o2], o1 - o0)
    plain_loop(data.clone())        # warm
    with Timer(torch) as t:
        plain_loop(loop_buf)
    ms_p = t.ms
    host = data.cpu().numpy()
    got_b = bufs[0].cpu().numpy()
    got_p = loop_buf.cpu().numpy()
    bad_b = bad_p = bad_g = 0
    for q in range(4096):
        o0, o1, o2 = off[2 * q], off[2 * q + 1], off[2 * q + 2]
        want = oracle.merge(host[o0:o2], int(o1 - o0))
        bad_b += int(np.count_nonzero(got_b[o0:o2] != want))
        bad_p += int(np.count_nonzero(got_p[o0:o2] != want))
        bad_g += int(np.count_nonzero(got_g[o0:o2] != want))
    log("c4: batched %.3f ms, graph %.3f ms (eager per-call %.3f), plain loop %.3f ms"
        % (ms_b, ms_g, ms_e, ms_p))
    return {"workload": "4096 instances, L_A, L_B ~ round(2^U[6,20]) int32, %d elements" % total,
            "batched_gelem_s": round(total / ms_b / 1e6, 2), "batched_ms": round(ms_b, 4),
            "leaf_config": used_cfg, "autotune_ms_per_config": [round(m, 4) for m in tune_ms],
            "graph_ms": round(ms_g, 4), "graph_gelem_s": round(total / ms_g / 1e6, 2),
            "eager_single_call_ms": round(ms_e, 4), "graph_leaf_node_cooperative": coop,
            "plain_loop_gelem_s": round(total / ms_p / 1e6, 2), "plain_loop_ms": round(ms_p, 3),
            "speedup_vs_plain_loop": round(ms_p / ms_b, 2),
            "mismatches_batched": bad_b, "mismatches_graph": bad_g,
            "mismatches_plain_loop": bad_p}


def bench_sort(torch, im, oracle, gen, dev):
    n = 2 ** 28
    log("c4: merge sort of 2^28 int32")
    x = gen.torch_unsorted(n, SEED + 41, dev)
    ms, _, bufs = timed_merges(torch, im, x, 0, 2, 1, fn=lambda b: im.inplace_merge_sort(b))
    want = oracle.sort_keys(x.cpu().numpy())
    bad = mismatches(bufs[0], want)
    return {"workload": "in-place merge sort, 2^28 int32 uniform", "gelem_s": round(n / ms / 1e6, 3),
            "ms": round(ms, 3), "mismatches": bad}


def bench_learned(torch, im, oracle, gen, dev, steps):
    la = lb = 2 ** 28
    n = la + lb
    log("c5: generating int64 lognormal | 16-component mixture, 2^28 + 2^28")
    pristine = gen.torch_pair_learned(la, lb, SEED + 50, dev)
    model = im.MergeModel(seed=SEED)
    t0 = time.perf_counter()
    model.train(pristine, la, samples=8192, steps=20000, lr=1e-2)
    train_s = time.perf_counter() - t0
    k = min(steps, 4)
    fn_l = lambda b: model.merge(b, la)
    fn_p = lambda b: im.inplace_merge(b, la)
    # both forms warmed up, then timed in alternation (median of rounds), so
    # neither is favoured by running first after training
    buf = torch.empty_like(pristine)
    for fn in (fn_l, fn_p):
        buf.copy_(pristine)
        fn(buf)
    torch.cuda.synchronize()
    rounds_l, rounds_p = [], []
    for _ in range(5):
        rounds_l.append(timed_merges(torch, im, pristine, la, k, 0, fn=fn_l)[0])
        rounds_p.append(timed_merges(torch, im, pristine, la, k, 0, fn=fn_p)[0])
    ms_l = sorted(rounds_l)[2]
    ms_p = sorted(rounds_p)[2]
    del buf
    _, prof_l, bufs = timed_merges(torch, im, pristine, la, k, 0, fn=fn_l, profile=True)
    st_l = im.fetch_stats()
    want = oracle.merge(pristine.cpu().numpy(), la)
    bad_l = mismatches(bufs[0], want)
    del bufs
    _, prof_p, bufs = timed_merges(torch, im, pristine, la, k, 0, fn=fn_p, profile=True)
    st_p = im.fetch_stats()
    bad_p = mismatches(bufs[0], want)
    del bufs
    # probes per diagonal on the tile diagonals of this workload
    ks = torch.linspace(0, n, 65537, device=dev).to(torch.int64)
    _, probes_l = model.corank(pristine, la, ks)
    _, probes_p = im.corank(pristine, la, ks, probes=True)
    log("c5: learned %.3f ms, plain %.3f ms" % (ms_l, ms_p))
    search_ms = lambda p: (p["split"][0] + p["tilerank"][0]) / k
    return {"workload": "int64, A lognormal(20,2), B 16-comp. mixture, 2^28+2^28",
            "learned_gelem_s": round(n / ms_l / 1e6, 2), "plain_gelem_s": round(n / ms_p / 1e6, 2),
            "learned_ms": round(ms_l, 4), "plain_ms": round(ms_p, 4),
            "search_ms_learned": round(search_ms(prof_l), 4),
            "search_ms_plain": round(search_ms(prof_p), 4),
            "probes_per_search_learned": round(st_l["search_probes"] / max(st_l["searches"], 1), 2),
            "probes_per_search_plain": round(st_p["search_probes"] / max(st_p["searches"], 1), 2),
            "probes_per_diagonal_learned_65537": round(float(probes_l.double().mean()), 2),
            "probes_per_diagonal_plain_65537": round(float(probes_p.double().mean()), 2),
            "timing": "median of 5 alternating rounds of %d merges per form, after a warm-up "
                      "merge of each" % k,
            "rounds_ms_learned": [round(x, 4) for x in rounds_l],
            "rounds_ms_plain": [round(x, 4) for x in rounds_p],
            "train_s": round(train_s, 3), "mismatches_learned": bad_l, "mismatches_plain": bad_p}


def bench_findmedian(torch, im, gen, dev, steps):
    """FindMedian (Alg. 1) against the exact co-rank split: the paper's
    imbalance study on its W1 generator (largest pair with FindMedian over
    largest pair with exact middle splits, minus one), and the whole merge
    of the balanced int32 workload with either split."""
    study = {}
    for logs in (16, 20, 22):
        S = 2 ** logs
        for frac in (0.25, 0.5, 0.75):
            data = gen.paper_w1_pair(S, frac, SEED + 60 + logs)
            la = int(S * frac)
            t = torch.from_numpy(data).to(dev)
            a, b = data[:la], data[la:]
            row_pair, row_work = {}, {}
            for depth in range(1, 17):
                if 2 ** depth > S // 4:
                    break
                mx = {}
                for name, m in (("fm", im.SPLIT_FINDMEDIAN), ("ex", im.SPLIT_CORANK)):
                    sz = im.divide(t, la, depth, m).cpu().numpy()
                    ao = np.concatenate([[0], np.cumsum(sz[:, 0])])[:-1]
                    bo = np.concatenate([[0], np.cumsum(sz[:, 1])])[:-1]
                    tot = sz.sum(axis=1)
                    # a pair needs a merge when both parts are non-empty and
                    # its last A element exceeds its first B element
                    need = (sz[:, 0] > 0) & (sz[:, 1] > 0)
                    idx = np.flatnonzero(need)
                    need[idx] = a[ao[idx] + sz[idx, 0] - 1] > b[np.minimum(bo[idx], b.size - 1)]
                    mx[name] = (int(tot.max()), int((tot * need).max()))
                T = str(2 ** depth)
                row_pair[T] = round((mx["fm"][0] - mx["ex"][0]) / mx["ex"][0], 5)
                row_work[T] = (round((mx["fm"][1] - mx["ex"][1]) / mx["ex"][1], 5)
                               if mx["ex"][1] else None)
            key = "S=2^%d split=%.2f" % (logs, frac)
            study[key] = {"largest_pair": row_pair, "largest_pair_needing_a_merge": row_work}
    la = lb = 2 ** 27
    n = la + lb
    pristine = gen.torch_pair_uniform(la, lb, SEED + 20, dev)
    res = {}
    for name, split in (("corank", im.SPLIT_CORANK), ("findmedian", im.SPLIT_FINDMEDIAN)):
        ms, _, bufs = timed_merges(torch, im, pristine, la, steps, 1,
                                   fn=lambda b: im.inplace_merge_variant(b, la, split,
                                                                         im.ROTATE_SWAP_REV))
        st = im.fetch_stats()
        res[name] = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
                     "levels_used": st["levels_used"], "leaves": st["leaves"],
                     "split_fallbacks": st["split_fallbacks"]}
        del bufs
    same = True
    a = pristine.clone()
    b = pristine.clone()
    im.inplace_merge_variant(a, la, im.SPLIT_FINDMEDIAN, im.ROTATE_SWAP_REV)
    im.inplace_merge(b, la)
    same = bool(torch.equal(a, b))
    log("f2: findmedian merge %.3f ms, corank %.3f ms" % (res["findmedian"]["ms"],
                                                         res["corank"]["ms"]))
    return {"workload": "W1 generator (Sec. 4) at S=2^16..2^22, splits 1/4,1/2,3/4; merge of "
                        "int32 2^27+2^27",
            "imbalance_rel": study,
            "imbalance_note": "(max FindMedian - max exact co-rank) / max exact co-rank, over "
                              "the 2^depth pairs; 'largest_pair' counts every pair, "
                              "'largest_pair_needing_a_merge' only pairs with both parts "
                              "non-empty and out of order",
            "merge_c2": res, "findmedian_equals_corank_result": same}


def bench_exchanges(torch, im, oracle, gen, dev, steps):
    """Linear vs circular shifting (Sec. 3.4), alone and inside the merge, and
    the out-of-place comparators."""
    out = {}
    n = 2 ** 28
    x = torch.arange(n, dtype=torch.int32, device=dev)
    for label, lx in (("swap 2^27|2^27", n // 2), ("2^27+3|2^27-3", n // 2 + 3),
                      ("2^24|rest", 2 ** 24)):
        buf = x.clone()
        # the merge's exchange: one block swap when the parts are equal, else
        # three reversals; the paper's linear shifting step by step; circular
        # shifting
        ms_sr = event_timed(torch, x, buf, lambda: im.rotate(buf, lx), max(steps, 3))
        ms_ls = event_timed(torch, x, buf, lambda: im.rotate_ls(buf, lx, count=False),
                            max(steps, 3))
        ms_cs = event_timed(torch, x, buf, lambda: im.rotate_cs(buf, lx), max(steps, 3))
        buf.copy_(x)
        _, swaps = im.rotate_ls(buf, lx)
        ok = bool(torch.equal(buf[:n - lx], x[lx:]) and torch.equal(buf[n - lx:], x[:lx]))
        moved = 2 * 4 * n          # every element read and written once (definition)
        out[label] = {"swap_rev_ms": round(ms_sr, 4), "ls_ms": round(ms_ls, 4),
                      "cs_ms": round(ms_cs, 4),
                      "swap_rev_eff_gb_s": round(moved / ms_sr / 1e6, 1),
                      "ls_eff_gb_s": round(moved / ms_ls / 1e6, 1),
                      "cs_eff_gb_s": round(moved / ms_cs / 1e6, 1),
                      "ls_swaps": swaps, "ls_correct": ok}
        del buf
    del x
    torch.cuda.empty_cache()
    la = lb = 2 ** 27
    pristine = gen.torch_pair_uniform(la, lb, SEED + 20, dev)
    merges = {}
    for name, fn in (
            ("in_place_swap_rev", lambda b: im.inplace_merge(b, la)),
            ("in_place_cs", lambda b: im.inplace_merge_variant(b, la, im.SPLIT_CORANK,
                                                               im.ROTATE_CS)),
            ("buffered_alloc_merge_copy_free", lambda b: im.inplace_merge_buffered(b, la))):
        ms, _, bufs = timed_merges(torch, im, pristine, la, 3, 1, fn=fn)
        merges[name] = {"ms": round(ms, 4), "gelem_s": round((la + lb) / ms / 1e6, 2)}
        del bufs
    o = torch.empty_like(pristine)
    ms_oop = event_timed(torch, pristine, pristine.clone(),
                         lambda: im.merge_out_of_place(pristine, la, o), 3)
    merges["out_of_place_only"] = {"ms": round(ms_oop, 4),
                                   "gelem_s": round((la + lb) / ms_oop / 1e6, 2)}
    want = im.merge_out_of_place(pristine, la)
    chk = pristine.clone()
    im.inplace_merge_variant(chk, la, im.SPLIT_CORANK, im.ROTATE_CS)
    merges["cs_equals_out_of_place"] = bool(torch.equal(chk, want))
    log("f3: exchanges", out)
    log("f3: merges", merges)
    return {"workload": "int32 exchanges of 2^28 elements; merges of int32 2^27+2^27",
            "exchange": out, "merge_c2": merges}


def bench_rows(torch, im, oracle, gen, dev, steps):
    """f4: wide rows (Sec. 4 elements: key word + payload), 1 GiB per width,
    L_A = L_B, uniform keys; against a plain device copy of the same bytes
    (the floor of any method that moves every row once) and the oracle."""
    out = {}
    total = 2 ** 30
    for W in (64, 256, 1024, 4096, 16384, 65536, 65540):
        n = total // W
        la = n // 2
        log("f4: rows of %d bytes, %d + %d" % (W, la, n - la))
        pristine = gen.torch_rows_pair(la, n - la, W // 4, SEED + 60 + W.bit_length(), dev)
        buf = torch.empty_like(pristine)
        ms = event_timed(torch, pristine, buf, lambda: im.inplace_merge_rows(buf, la), steps)
        st = im.fetch_stats()
        copy_ms = event_timed(torch, pristine, buf, lambda: buf.copy_(pristine), steps)
        # stage split of one more merge (events on the merge's stream)
        buf.copy_(pristine)
        torch.cuda.synchronize()
        im.profile_read()
        im.profile(True)
        im.inplace_merge_rows(buf, la)
        torch.cuda.synchronize()
        prof = im.profile_read()
        im.profile(False)
        want = oracle.merge_rows(pristine.cpu().numpy(), la)
        got = buf.cpu().numpy()
        bad = int(np.count_nonzero(np.any(got != want, axis=1)))
        del got, want
        moved = 2 * W * (st["rotated_elems"] + st["leaf_elems"])     # read + write
        out["rows_%d_B" % W] = {
            "rows": n, "ms": round(ms, 4), "grows_s": round(n / ms / 1e6, 4),
            "effective_gb_s": round(2 * n * W / ms / 1e6, 1),
            "copy_ms": round(copy_ms, 4), "copy_gb_s": round(2 * n * W / copy_ms / 1e6, 1),
            "moved_bytes": moved, "moved_gb_s": round(moved / ms / 1e6, 1),
            "levels_used": st["levels_used"], "leaves": st["leaves"],
            "fused_nodes": st["fused_nodes"], "tile_rows": st["tile"],
            "leaf_grid": st["leaf_grid"],
            "stages_ms": {k: round(v[0], 4) for k, v in prof.items()},
            "mismatched_rows": bad}
        del pristine, buf
        torch.cuda.empty_cache()
    return {"workload": "rows of W bytes (int32 key + payload), floor(2^30/W) rows, "
                        "L_A = L_B (rounded down), keys uniform in [0,2^31); 65540 B is "
                        "the paper's largest element", "widths": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--forms", choices=["all", "none", "rows", "learned", "exchanges", "c1", "sort"],
                    default="all",
                    help="other workloads after the headline: all, none, or only the rows, "
                         "the learned-split, the exchange, the small (c1) or the merge-sort forms")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (profiling runs: default leaf configuration)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device 3 times (the known-size "
                         "reference that scales the HBM byte counters) and exit")
    ap.add_argument("--then-copy-probe", action="store_true",
                    help="after the benchmark line, the same three 1 GiB copies (one "
                         "counter run then holds the merge and its scale reference)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the merge is measured on one GPU (one MI355X); "
              "--gpus %d / WORLD_SIZE=%d is not supported" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_2005_12648_amd as im
    import oracle
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    im.load()
    dev = torch.device("cuda:0")
    def copy_probe():
        src = torch.ones(2 ** 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.copy_probe:
        copy_probe()
        print(json.dumps({"copy_probe_bytes_per_copy": 2 ** 30}), flush=True)
        return

    head = bench_headline(torch, im, oracle, gen, dev, args)
    n = head["n"]
    value = n / head["ms"] / 1e6
    roof = roofline(head["prof"], head["stats"], 4, args.steps, "c2")
    forms = {}
    if args.forms == "all":
        for name in ("c1", "c2_skew", "c2_dup", "c3_kv"):
            log("variant", name)
            forms[name] = bench_variant(torch, im, oracle, gen, dev, name, 3)
            torch.cuda.empty_cache()
        forms["c2_graph"] = bench_graph_single(torch, im, oracle, gen, dev, 7)
        torch.cuda.empty_cache()
        forms["c4_batched"] = bench_batched(torch, im, oracle, gen, dev, 3)
        torch.cuda.empty_cache()
        forms["c4_sort"] = bench_sort(torch, im, oracle, gen, dev)
        torch.cuda.empty_cache()
        forms["c5_learned"] = bench_learned(torch, im, oracle, gen, dev, args.steps)
        torch.cuda.empty_cache()
        forms["f2_findmedian"] = bench_findmedian(torch, im, gen, dev, 3)
        torch.cuda.empty_cache()
        forms["f3_exchange_and_out_of_place"] = bench_exchanges(torch, im, oracle, gen, dev, 3)
        torch.cuda.empty_cache()
        forms["f4_wide_rows"] = bench_rows(torch, im, oracle, gen, dev, 3)
    elif args.forms == "rows":
        forms["f4_wide_rows"] = bench_rows(torch, im, oracle, gen, dev, 3)
    elif args.forms == "learned":
        forms["c5_learned"] = bench_learned(torch, im, oracle, gen, dev, args.steps)
    elif args.forms == "c1":
        forms["c1"] = bench_variant(torch, im, oracle, gen, dev, "c1", 3)
    elif args.forms == "exchanges":
        forms["f3_exchange_and_out_of_place"] = bench_exchanges(torch, im, oracle, gen, dev, 3)
    elif args.forms == "sort":
        forms["c4_sort"] = bench_sort(torch, im, oracle, gen, dev)
    st = head["stats"]
    line = {
        "metric": "Gelem/s, in-place merge of int32 L_A=L_B=2^27",
        "value": round(value, 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded, generated on the device)",
        "config": {"workload": "c2: int32 in-place merge, L_A=L_B=2^27, runs uniform in [0,2^31) "
                               "each sorted", "elements": n,
                   "levels_used": st["levels_used"], "leaves": st["leaves"],
                   "leaf_capacity": st["leaf_capacity"], "tile": st["tile"],
                   "leaf_config": st["leaf_config"], "leaf_grid": st["leaf_grid"],
                   "autotune_ms_per_config": head["tune_ms"]},
        "effective_hbm_gb_s": round(2 * 4 * n / head["ms"] / 1e6, 1),
        "effective_hbm_frac": round(2 * 4 * n / head["ms"] / 1e6 / HBM_PEAK_GBS, 4),
        "measured_hbm": measured_hbm(head["ms"]),
        "mismatches": head.get("mismatch"),
        "roofline": roof,
        "cpu_baseline": head["cpu"],
        "forms": forms,
    }
    print(json.dumps(line), flush=True)
    if args.then_copy_probe:
        torch.cuda.empty_cache()
        copy_probe()
        log("copy probe: three device-to-device copies of 1 GiB")


if __name__ == "__main__":
    main()
