#!/usr/bin/env python3
"""Benchmark of the HSS hot path on one MI355X.

One step = one hss_partition (local sort of every segment, the splitter
rounds, the bucketed exchange) of N = 2^28 uniform uint64 keys in p = 1024
segments with eps = 0.02, inputs resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

The line carries the throughput, the roofline of the dominant kernel (its
algorithmic bytes per launch over its average launch time, HIP events on its
stream over the timed region), the rate of a plain streaming copy as the
achievable HBM reference, the Zipf-Morton payload workload at p = 4096 timed
the same way, and the CPU oracle on the same keys on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gkeys/s sort+partition, 2^28 u64 p=1024; % HBM peak; batched vs plain"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
WORKLOADS = {
    # name: (n, p, eps, data seed, hss seed, generator, payload)
    "uniform_u64_2^28_p1024": (1 << 28, 1024, 0.02, 2, 2, "uniform64", False),
    "zipf_morton_u64+payload_2^28_p4096": (1 << 28, 4096, 0.05, 3, 3, "zipf_morton", True),
    "uniform_u64_2^20_p16": (1 << 20, 16, 0.05, 1, 1, "uniform64", False),
}
# Measured HBM bytes per launch of each kernel family on the uniform 2^28,
# p=1024 partition: rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB per
# dispatch x 1024).  The factors are what the two counters read for a plain
# 2 GiB device copy: FETCH_SIZE 1 GiB (x 2), WRITE_SIZE 2 GiB (x 1).  The
# figures hold for the kernel sources with the hash below; after any change
# to them the traffic is reported as null until the counters are taken again.
TRAFFIC_WORKLOAD = "uniform_u64_2^28_p1024"
TRAFFIC_SRC_SHA = "e225b15e6edd7780"
TRAFFIC = {   # family: (fetch bytes, write bytes) per launch
    "radix_count": (2147719848, 71303168),
    "radix_scan": (134381585, 70254592),
    "radix_scatter": (2214747286, 2190616733),
    "exchange_copy": (2304444498, 2162073238),
    "small_sort": (2229693871, 2472052229),
}


def kernel_source_sha() -> str:
    """Hash of the sources of the measured kernel families (the radix passes,
    the small sort and the exchange, with the device helpers)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1803_01237_amd", "csrc")
    files = [os.path.join(csrc, f) for f in ("device.hpp", "exchange.hip", "radix.hip", "smallsort.hip")]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, fam):
    if workload != TRAFFIC_WORKLOAD or fam not in TRAFFIC or kernel_source_sha() != TRAFFIC_SRC_SHA:
        return None
    return sum(TRAFFIC[fam])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(keys, p, eps, hseed, payload, threads):
    """The oracle on the host cores: hss_partition of the whole workload (the
    same host keys as the GPU run), its per-segment and per-bucket work split
    over `threads` threads; then, for scale, the small configuration (2^20
    uniform keys, p = 16, eps = 0.05) on one thread."""
    import oracle
    import synth
    n = len(keys)
    vals = np.arange(n, dtype=np.uint64) if payload else None
    t0 = time.perf_counter()
    r = oracle.hss(keys, p, eps, hseed, vals=vals, mode="partition", trace_level=0, threads=threads)
    dt = time.perf_counter() - t0
    assert r.status == 0
    stages = {"local_sort": r.times[0], "rounds": r.times[1], "exchange": r.times[2]}
    del r, vals
    k1 = synth.make("uniform64", 1 << 20, 1)
    t1 = time.perf_counter()
    r1 = oracle.hss(k1, 16, 0.05, 1, mode="partition", trace_level=0, threads=1)
    d1 = time.perf_counter() - t1
    assert r1.status == 0
    return {"value": n / dt / 1e9, "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
            "sample": f"hss_partition of the whole workload ({n} keys, p={p}, eps={eps}) by the "
                      f"C++ oracle on {threads} host threads, {dt:.2f} s",
            "seconds": round(dt, 3),
            "stage_seconds": {k: round(v, 3) for k, v in stages.items()},
            "small_config": {"n": 1 << 20, "p": 16, "eps": 0.05, "threads": 1,
                             "seconds": round(d1, 3), "gkeys_per_s": round((1 << 20) / d1 / 1e9, 5)},
            "host": {"nproc": os.cpu_count(), "cpu": _cpu_model()}}


def copy_ceiling(nbytes=1 << 31, reps=10):
    """The achievable HBM rate: the library's 16-byte-per-lane streaming copy
    of `nbytes` over a few grid sizes, with and without non-temporal hints
    (best of each), beside torch's device copy; GB/s counts bytes read plus
    written."""
    import torch
    import paper_1803_01237_amd as hss
    src = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda:0")
    src.fill_(1)
    dst = torch.empty_like(src)

    def rate(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = 1e30
        for _ in range(reps):
            a.record()
            fn()
            b.record()
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        return 2 * nbytes / (best * 1e-3) / 1e9

    runs = {}
    for nt in (False, True):
        for wg in (1024, 2048, 4096, 8192, 16384):
            runs[f"wg{wg}{'_nt' if nt else ''}"] = round(rate(lambda: hss.stream_copy(dst, src, wg, nt)), 1)
    torch_rate = round(rate(lambda: dst.copy_(src)), 1)
    assert torch.equal(dst, src)
    best = max(runs, key=runs.get)
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "best": best, "GB_per_s": runs[best],
            "frac_of_peak": round(runs[best] / HBM_PEAK_GBS, 4), "runs": runs,
            "torch_copy_GB_per_s": torch_rate}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def batched_bench(steps, count):
    """The batched workload: `count` instances of uneven N and p (half u32,
    half u64 keys) partitioned by one hss_batch_partition, against the same
    instances as sequential hss_partition calls on one plan each."""
    import torch
    import paper_1803_01237_amd as hss
    import synth
    dev = torch.device("cuda:0")
    shapes = synth.batched_shapes(count)
    log(f"[bench] batched: {count} instances, {sum(s[0] for s in shapes)} keys")
    keys = []
    for sh in shapes:
        k = synth.batched_keys(sh)
        keys.append(torch.from_numpy(k.view(np.int64 if sh[3] == 8 else np.int32)).to(dev))
    seeds = [sh[5] for sh in shapes]
    kout = [torch.empty_like(k) for k in keys]
    offs = [torch.empty(sh[1] + 1, dtype=torch.int64, device=dev) for sh in shapes]
    total = sum(sh[0] for sh in shapes)
    with hss.BatchPlan([(sh[0], sh[1], sh[2], sh[3]) for sh in shapes], autotune=True) as bp:
        bp.partition(keys, seeds, keys_out=kout, offsets=offs)   # warmup, autotunes
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            bp.partition(keys, seeds, keys_out=kout, offsets=offs)
        torch.cuda.synchronize()
        b_ms = (time.perf_counter() - t0) * 1e3 / steps
        b_offs = [o.cpu().numpy() for o in offs]
        ws = bp.workspace_bytes
    plans = [hss.Plan(sh[0], sh[1], sh[2], key_bytes=sh[3]) for sh in shapes]
    try:
        for pl, k, sd, ko, of in zip(plans, keys, seeds, kout, offs):
            pl.partition(k, sd, keys_out=ko, offsets=of)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pl, k, sd, ko, of in zip(plans, keys, seeds, kout, offs):
            pl.partition(k, sd, keys_out=ko, offsets=of)
        torch.cuda.synchronize()
        p_ms = (time.perf_counter() - t0) * 1e3
        same = all(np.array_equal(a, o.cpu().numpy()) for a, o in zip(b_offs, offs))
    finally:
        for pl in plans:
            pl.close()
    return {"instances": count, "keys": total, "batched_ms": round(b_ms, 3),
            "batched_gkeys_per_s": round(total / (b_ms * 1e-3) / 1e9, 3),
            "plain_ms": round(p_ms, 3), "plain_gkeys_per_s": round(total / (p_ms * 1e-3) / 1e9, 3),
            "speedup": round(p_ms / b_ms, 2), "offsets_equal": bool(same),
            "workspace_gib": round(ws / 2**30, 2),
            "shape": "N log-uniform on [2^12, 2^22], p log-uniform on [8, 256], eps 0.05, "
                     "first half u32 keys, second half u64"}


SWEEP = ["UNIF", "SKEW1", "SKEW2", "SKEW3", "GAUSS", "ALLZEROS"]


def _timed(fn, steps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def options_bench(keys, n, p, eps, hseed, steps):
    """The plan options of the same kernels at the headline size: HSS with one
    round (k = 1, section 4.1), exact splitting (eps = p / N, tol = 0) and a
    fixed budget of 5 p and of p probes per round (section 6); then the
    rounds against p at eps = 2% (section 7.1) for the rate schedule, both
    budgets and the same budgets drawn as section 6's picks, on the first
    2^26 keys."""
    import torch
    import paper_1803_01237_amd as hss
    out = {}
    kout = torch.empty_like(keys)
    off = torch.empty(p + 1, dtype=torch.int64, device=keys.device)
    ideal = (np.arange(p + 1, dtype=object) * n) // p
    for name, e, k, c in [("one_round", eps, 1, 0), ("exact", p / n, 0, 0),
                          ("budget_5p", eps, 0, 5), ("budget_1p", eps, 0, 1)]:
        log(f"[bench] option {name}: eps={e} k_override={k} probes_per_round={c}")
        with hss.Plan(n, p, e, k_override=k, probes_per_round=c) as plan:
            ms = _timed(lambda: plan.partition(keys, hseed, keys_out=kout, offsets=off), steps)
            tr = plan.trace()
            tol, kk = plan.constants(1)[:2]
            o = off.cpu().numpy()
            dev = max(abs(int(o[i]) - int(ideal[i])) for i in range(p + 1))
            if dev > tol:
                raise RuntimeError(f"option {name}: splitter {dev} from its ideal rank, tol {tol}")
            out[name] = {"eps": e, "k": int(kk), "tol": int(tol), "ms_per_step": round(ms, 4),
                         "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3), "rounds": len(tr),
                         "probes_per_round": [r.m for r in tr], "max_splitter_deviation": dev}
    n2 = 1 << 26
    sub = keys[:n2]
    kout2 = torch.empty_like(sub)
    curve = {}
    for c, picks in ((0, False), (5, False), (1, False), (5, True), (1, True)):
        label = "schedule" if c == 0 else (f"picks_{c}p" if picks else f"budget_{c}p")
        curve[label] = {}
        for pp in (64, 256, 1024, 2048, 4096):
            off2 = torch.empty(pp + 1, dtype=torch.int64, device=keys.device)
            with hss.Plan(n2, pp, 0.02, probes_per_round=c, pick_sampler=picks) as plan:
                plan.partition(sub, hseed, keys_out=kout2, offsets=off2)
                tr = plan.trace()
                curve[label][str(pp)] = {"rounds": len(tr), "probes": sum(r.m for r in tr)}
    out["rounds_vs_p"] = {"n": n2, "eps": 0.02, "curves": curve}
    return out


def staged_bench(keys, n, hseed, steps, p=4096, r=64):
    """Section 5.3 at the headline size: single-stage HSS with p = 4096
    processors (eps = 2%) against two stages, r = sqrt(p) = 64 groups of 64
    (eps = 1% per stage, as in the paper's two-stage runs, so that the final
    imbalance stays within about 2%)."""
    import torch
    import paper_1803_01237_amd as hss
    kout = torch.empty_like(keys)
    off = torch.empty(p + 1, dtype=torch.int64, device=keys.device)
    grp = torch.empty(r + 1, dtype=torch.int64, device=keys.device)
    out = {"n": n, "p": p}
    log(f"[bench] single stage p={p}")
    with hss.Plan(n, p, 0.02, autotune=True) as plan:
        ms = _timed(lambda: plan.partition(keys, hseed, keys_out=kout, offsets=off), steps)
        tr = plan.trace()
        o = off.cpu().numpy().astype(np.int64)
        out["single"] = {"eps": 0.02, "ms_per_step": round(ms, 4),
                         "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3), "rounds": len(tr),
                         "probes": sum(x.m for x in tr), "max_bucket": int(np.diff(o).max())}
    log(f"[bench] two stages p={p} r={r}")
    with hss.StagedPlan(n, p, r, 0.01, 0.01, autotune=True) as plan:
        ms = _timed(lambda: plan.partition(keys, hseed, keys_out=kout, offsets=off, groups_out=grp),
                    steps)
        t1, ts, t2 = plan.times()
        o = off.cpu().numpy().astype(np.int64)
        g = grp.cpu().numpy().astype(np.int64)
        bound = int(n * 1.01 * 1.01 / p) + 2
        if int(np.diff(o).max()) > bound or o[0] != 0 or o[p] != n or g[r] != n:
            raise RuntimeError("two-stage balance check failed")
        out["two_stage"] = {"groups": r, "eps1": 0.01, "eps2": 0.01, "ms_per_step": round(ms, 4),
                            "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
                            "last_call_ms": {"stage1": round(t1 * 1e3, 3), "stage2_layout": round(ts * 1e3, 3),
                                             "stage2": round(t2 * 1e3, 3)},
                            "max_bucket": int(np.diff(o).max()), "max_group": int(np.diff(g).max()),
                            "workspace_gib": round(plan.workspace_bytes / 2**30, 2)}
        log(f"[bench] two-stage sort p={p} r={r}")
        ms = _timed(lambda: plan.sort(keys, hseed, keys_out=kout, offsets=off, groups_out=grp), steps)
        ku = kout[: 1 << 20].cpu().numpy().view(np.uint64)   # the first 2^20 keys in order
        if not np.all(ku[1:] >= ku[:-1]):
            raise RuntimeError("two-stage sort order check failed")
        out["two_stage_sort"] = {"ms_per_step": round(ms, 4), "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3)}
    return out


def sweep_bench(plan, keys, n, p, eps, hseed, steps):
    """The distributions of section 7.5 through the headline plan: one input
    buffer refilled per distribution, per-stage times from the HIP events."""
    import torch
    import synth
    kout = torch.empty_like(keys)
    off = torch.empty(p + 1, dtype=torch.int64, device=keys.device)
    tol = plan.constants(1)[0]
    ideal = (np.arange(p + 1, dtype=object) * n) // p
    out = {}
    for kind in SWEEP:
        log(f"[bench] sweep {kind}")
        keys.copy_(torch.from_numpy(synth.make(kind, n, 70).view(np.int64)))
        plan.partition(keys, hseed, keys_out=kout, offsets=off)
        torch.cuda.synchronize()
        plan.profile(True)
        plan.profile_reset()
        ms = _timed(lambda: plan.partition(keys, hseed, keys_out=kout, offsets=off), steps)
        prof = plan.profile_read()
        plan.profile(False)
        o = off.cpu().numpy()
        dev = max(abs(int(o[i]) - int(ideal[i])) for i in range(p + 1))
        if dev > tol:
            raise RuntimeError(f"sweep {kind}: splitter {dev} from its ideal rank, tol {tol}")
        st = {f: round(prof[f][0] / (steps + 1), 4) for f in prof if prof[f][1] > 0}
        tr = plan.trace()
        out[kind] = {"ms_per_step": round(ms, 4), "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
                     "rounds": len(tr), "probes": sum(r.m for r in tr), "stage_ms": st}
    return out


def served_bench(count, mults, check_every, wait_us=0):
    """The served workload: u64 requests with a payload arriving as a Poisson
    process, served by the library's request server; requests alternate
    between partition (even index) and sort (odd index).  The rate is set
    from the plain-path capacity (keys per second of one plan per request:
    create, partition or sort, release) times each multiplier.  Latency is
    completion minus the scheduled arrival; every check_every-th request is
    compared with its solo run.  With wait_us, one more run at 1.0 times
    the capacity lets a lone partition request wait that long for another
    to share its batch (latency for batching)."""
    import torch
    import paper_1803_01237_amd as hss
    import synth
    dev = torch.device("cuda:0")
    shapes = synth.served_shapes(count)
    total = sum(sh[0] for sh in shapes)
    mean_n = total / count

    def inputs(sh):
        return synth.device_keys(sh[0], sh[3], dev), torch.arange(sh[0], dtype=torch.int64, device=dev)

    def op_of(i):
        return "sort" if i % 2 else "partition"

    # plain-path capacity on the first requests
    cap_keys, cap_s = 0, 0.0
    for i, sh in enumerate(shapes[:min(48, count)]):
        keys, vals = inputs(sh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with hss.Plan(sh[0], sh[1], sh[2], payload=True) as pl:
            (pl.sort if op_of(i) == "sort" else pl.partition)(keys, sh[4], vals)
            torch.cuda.synchronize()
        cap_s += time.perf_counter() - t0
        cap_keys += sh[0]
    capacity = cap_keys / cap_s
    log(f"[bench] served: {count} requests, {total} keys; plain capacity {capacity / 1e9:.2f} Gkeys/s")
    runs = []
    window = 32
    inflight = 96
    for mult, wait in [(m, 0) for m in mults] + ([(1.0, wait_us)] if wait_us else []):
        rate = mult * capacity / mean_n                 # requests per second
        arrivals = np.cumsum(np.random.default_rng(5).exponential(1.0 / rate, count))
        lat, lag, kept = [], [], []
        with hss.Server(batch_wait_us=wait) as srv:
            t0 = srv.clock() + 0.05
            pending = {}
            t_last = 0.0

            def drain(block):
                nonlocal t_last
                for t in list(pending):
                    r = srv.wait(t) if block else srv.poll(t)
                    if r is None:
                        continue
                    i, arr = pending.pop(t)
                    lat.append(r.t_done - arr)
                    t_last = max(t_last, r.t_done)
                    if i % check_every == 0:
                        kept.append((i, r))

            for w0 in range(0, count, window):
                # inputs of the next window, made before their arrival times
                batch = [inputs(sh) for sh in shapes[w0:w0 + window]]
                torch.cuda.synchronize()
                for j, (keys, vals) in enumerate(batch):
                    i = w0 + j
                    sh = shapes[i]
                    arr = t0 + arrivals[i]
                    while srv.clock() < arr:
                        drain(False)
                    # a client with at most `inflight` requests outstanding:
                    # above the server's capacity the arrivals fall behind
                    while len(pending) >= inflight:
                        oldest = next(iter(pending))
                        r = srv.wait(oldest)
                        i0, a0 = pending.pop(oldest)
                        lat.append(r.t_done - a0)
                        t_last = max(t_last, r.t_done)
                        if i0 % check_every == 0:
                            kept.append((i0, r))
                    lag.append(max(0.0, srv.clock() - arr))
                    t = srv.submit(keys, sh[1], sh[2], sh[4], vals, sync=False, op=op_of(i))
                    pending[t] = (i, arr)
                del batch
            drain(True)
            st = srv.stats()
            mem = srv.memory()
        makespan = t_last - (t0 + arrivals[0])
        # each kept result against its solo run
        same = True
        for i, r in kept:
            sh = shapes[i]
            keys, vals = inputs(sh)
            with hss.Plan(sh[0], sh[1], sh[2], payload=True) as pl:
                ko, vo, off = (pl.sort if op_of(i) == "sort" else pl.partition)(keys, sh[4], vals)
                torch.cuda.synchronize()
                same = same and torch.equal(off, r.offsets) and torch.equal(ko, r.keys_out) \
                    and torch.equal(vo, r.vals_out)
        del kept
        lat_ms = np.array(lat) * 1e3
        runs.append({"rate_x_capacity": mult, "batch_wait_us": wait, "requests_per_s": round(rate, 1),
                     "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                     "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                     "throughput_gkeys_s": round(total / makespan / 1e9, 3),
                     "makespan_s": round(makespan, 3), "batches": st["batches"],
                     "mean_requests_per_batch": round(count / max(st["batches"], 1), 2),
                     "max_concurrent_batches": st["max_concurrent_batches"],
                     "max_admitted_gb": round(st["max_admitted_bytes"] / 1e9, 2),
                     "max_held_gb": round(mem["max_held_bytes"] / 1e9, 2),
                     "submit_lag_p99_ms": round(float(np.percentile(np.array(lag) * 1e3, 99)), 3),
                     "checked_against_solo": len(range(0, count, check_every)),
                     "all_equal": bool(same)})
        log(f"[bench] served x{mult} (wait {wait} us): p50 {runs[-1]['p50_ms']} ms, p99 {runs[-1]['p99_ms']} ms, "
            f"{runs[-1]['throughput_gkeys_s']} Gkeys/s, {st['batches']} batches")
    return {"requests": count, "keys": total, "plain_capacity_gkeys_s": round(capacity / 1e9, 3),
            "shape": "N = floor(2^U(14,26)) u64 keys + u64 payload, p = clamp(floor(e^U(ln 64, ln 2049)), "
                     "64, 2048), eps in {0.02, 0.05}, keys drawn on the device (torch generator per request), "
                     "Poisson arrivals; requests alternate partition and sort",
            "server": "2 workers (streams), 64 GiB HBM budget",
            "runs": runs}


def run_workload(name, keys, steps, warmup, op, sort_steps):
    """Time `steps` calls of the plan of workload `name` on `keys` (device)
    after `warmup` (the first warmup call runs the autotuner); returns the
    measurements and the plan (still open).  Per-stage times come from HIP
    events on the library's stream around every launch."""
    import torch
    import paper_1803_01237_amd as hss
    n, p, eps, dseed, hseed, kind, payload = WORKLOADS[name]
    dev = keys.device
    vals = torch.arange(n, dtype=torch.int64, device=dev) if payload else None
    kout = torch.empty_like(keys)
    vout = torch.empty_like(vals) if payload else None
    off = torch.empty(p + 1, dtype=torch.int64, device=dev)
    # the first warmup call runs the autotuner on this input (no warmup: no
    # autotuning, so that no timed step searches)
    plan = hss.Plan(n, p, eps, key_bytes=8, payload=payload, autotune=warmup > 0)
    log(f"[bench] {name}: workspace {plan.workspace_bytes / 2**30:.2f} GiB; warmup {warmup}")
    step = plan.partition if op == "partition" else plan.sort
    for _ in range(warmup):
        step(keys, hseed, vals, kout, vout, off)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_reset()
    log(f"[bench] {name}: timing {steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(keys, hseed, vals, kout, vout, off)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read()
    plan.profile(False)
    ms_step = (t1 - t0) * 1e3 / steps
    tr = plan.trace()
    # check the benched result: every splitter inside its target range
    tol = plan.constants(1)[0]
    o = off.cpu().numpy()
    ideal = (np.arange(p + 1, dtype=object) * n) // p
    bad = [i for i in range(1, p) if abs(int(o[i]) - int(ideal[i])) > tol]
    if bad or o[0] != 0 or o[p] != n:
        log(f"[bench] {name}: BALANCE CHECK FAILED at {bad[:5]}")
        sys.exit(1)
    # hss_sort for context (not the headline)
    sort_ms = None
    if sort_steps > 0:
        plan.sort(keys, hseed, vals, kout, vout, off)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(sort_steps):
            plan.sort(keys, hseed, vals, kout, vout, off)
        torch.cuda.synchronize()
        sort_ms = (time.perf_counter() - s0) * 1e3 / sort_steps
    # roofline of the dominant kernel family (largest share of the step)
    fam = max((f for f in prof if f != "rounds" and prof[f][1] > 0), key=lambda f: prof[f][0])
    f_ms, f_n, f_bytes = prof[fam]
    achieved = (f_bytes / f_n) / (f_ms / f_n * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": fam, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(name, fam), "traffic_unit": "bytes/launch",
            "avg_launch_ms": round(f_ms / f_n, 4),
            "bytes_per_launch": f_bytes // f_n}
    stages = {f: {"ms_per_step": round(prof[f][0] / steps, 4),
                  "launches_per_step": prof[f][1] // steps,
                  "GB_per_s": (round(prof[f][2] / (prof[f][0] * 1e-3) / 1e9, 1)
                               if prof[f][0] > 0 and prof[f][2] else None)}
              for f in prof}
    res = {"workload": name, "n": n, "p": p, "eps": eps, "payload": payload, "op": "hss_" + op,
           "ms_per_step": round(ms_step, 4), "gkeys_per_s": n / (ms_step * 1e-3) / 1e9,
           "stages": stages, "roofline": roof, "rounds": len(tr),
           "probes_per_round": [r.m for r in tr], "domain_per_round": [r.domain for r in tr],
           "knobs": plan.knobs(),
           "hss_sort_ms": None if sort_ms is None else round(sort_ms, 4),
           "hss_sort_gkeys_s": None if sort_ms is None else round(n / (sort_ms * 1e-3) / 1e9, 3)}
    del kout, vout, vals
    return res, plan


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform_u64_2^28_p1024", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="host threads of the CPU oracle baseline (0 to skip)")
    ap.add_argument("--skewed-steps", type=int, default=10,
                    help="steps of the Zipf-Morton payload workload at p = 4096 (0 to skip)")
    ap.add_argument("--no-copy-ceiling", dest="copy_ceiling", action="store_false",
                    help="skip the streaming-copy bandwidth reference")
    ap.add_argument("--sort-steps", type=int, default=3, help="hss_sort steps timed for context")
    ap.add_argument("--op", default="partition", choices=["partition", "sort"],
                    help="operation timed as the step (the headline is partition)")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="instances of the batched comparison (0 to skip)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--option-steps", type=int, default=3,
                    help="steps per plan option (one round, exact splitting); 0 to skip")
    ap.add_argument("--staged-steps", type=int, default=3,
                    help="single- vs two-stage partition at p = 4096 (0 to skip)")
    ap.add_argument("--sweep-steps", type=int, default=3,
                    help="steps per distribution of the sweep; 0 to skip")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="requests of the served workload (0 to skip)")
    ap.add_argument("--serve-rates", default="0.7,1.0,2.0",
                    help="arrival rates as multiples of the plain-path capacity")
    ap.add_argument("--serve-check-every", type=int, default=50)
    ap.add_argument("--serve-wait-us", type=int, default=2000,
                    help="one more served run at 1.0x with this batching wait (0 to skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device-to-device copy of 2 GiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        src = torch.empty(1 << 28, dtype=torch.int64, device="cuda:0")
        src.fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(10):
            dst.copy_(src)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / 10
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": src.numel() * 8,
                          "dispatches": 13, "copy_ms": round(ms, 4),
                          "copy_GB_per_s": round(2 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1)}),
              flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1803_01237_amd as hss
    import synth

    n, p, eps, dseed, hseed, kind, payload = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    log(f"[bench] generating {args.workload}: n={n} p={p} eps={eps}")
    keys_np = synth.make(kind, n, dseed)
    keys = torch.from_numpy(keys_np.view(np.int64)).to(dev)
    res, plan = run_workload(args.workload, keys, args.steps, args.warmup, args.op, args.sort_steps)
    ms_step, value, stages, roof = res["ms_per_step"], res["gkeys_per_s"], res["stages"], res["roofline"]
    kout = torch.empty_like(keys)
    off = torch.empty(p + 1, dtype=torch.int64, device=dev)
    vals = vout = None

    # both extra legs only at the headline workload; the options first, while
    # the input buffer still holds the headline keys
    headline = args.workload == "uniform_u64_2^28_p1024" and args.op == "partition"
    options = (options_bench(keys, n, p, eps, hseed, args.option_steps)
               if args.option_steps > 0 and headline else None)
    staged = (staged_bench(keys, n, hseed, args.staged_steps)
              if args.staged_steps > 0 and headline else None)
    sweep = (sweep_bench(plan, keys, n, p, eps, hseed, args.sweep_steps)
             if args.sweep_steps > 0 and headline else None)
    plan.close()
    del keys, kout, vout, vals
    torch.cuda.empty_cache()
    ceiling = copy_ceiling() if args.copy_ceiling else None
    # the Zipf-Morton configuration with a payload (p = 4096), timed the same way
    skewed = None
    if args.skewed_steps > 0 and headline:
        sname = "zipf_morton_u64+payload_2^28_p4096"
        sn, sp, seps, sdseed, shseed, skind, _ = WORKLOADS[sname]
        log(f"[bench] generating {sname}")
        sk = torch.from_numpy(synth.make(skind, sn, sdseed).view(np.int64)).to(dev)
        skewed, splan = run_workload(sname, sk, args.skewed_steps, min(args.warmup, 2), "partition", 0)
        splan.close()
        del sk
        torch.cuda.empty_cache()
    batched = batched_bench(args.batch_steps, args.batch_count) if args.batch_count > 0 else None
    served = (served_bench(args.serve_requests, [float(x) for x in args.serve_rates.split(",")],
                           args.serve_check_every, args.serve_wait_us) if args.serve_requests > 0 else None)

    cpu = None
    if args.cpu_threads > 0:
        threads = min(args.cpu_threads, os.cpu_count() or 1)
        log(f"[bench] CPU oracle on {threads} threads")
        cpu = cpu_baseline(keys_np, p, eps, hseed, payload, threads)
    del keys_np

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "p": p, "eps": eps,
                   "payload": payload, "op": "hss_" + args.op, "seed": hseed},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages": stages,
        "rounds": res["rounds"], "probes_per_round": res["probes_per_round"],
        "domain_per_round": res["domain_per_round"],
        "knobs": res["knobs"],
        "hss_sort_ms": res["hss_sort_ms"],
        "hss_sort_gkeys_s": res["hss_sort_gkeys_s"],
        "copy_ceiling": ceiling,
        "zipf_morton_p4096": skewed,
        "batched": batched,
        "served": served,
        "plan_options": options,
        "stages_p4096": staged,
        "distributions": sweep,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
