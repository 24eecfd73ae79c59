#!/usr/bin/env python
"""Decompressed GB/s of two-pass gzip decompression on one MI355X.

One step = one whole two-pass decompression of the workload's gzip member,
compressed input already in HBM, output left in HBM: block-start scan,
symbolic inflate, stitch, size scan, window propagation, translation.  The
default workload is 1 GiB of FASTQ-like text (100/150 bp reads) compressed as
one gzip member at level 6 and cut into 40 KiB compressed chunks (the
library's default).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
import zlib

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


CLOCK_GHZ = 2.4  # MI355X engine clock used for wave-cycle figures


def host_info():
    """CPU model and core counts of the host running the oracle."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0))}


def _pinned(core, fn):
    """fn() with the calling thread pinned to one core (sched_setaffinity of
    the thread, as taskset does for a process)."""
    old = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {core})
    try:
        return fn()
    finally:
        os.sched_setaffinity(0, old)


def cpu_baseline(comp: bytes, n_raw: int, crc_ref: int, workload: str):
    """The oracle's sequential gunzip (plain bit-serial RFC 1951/1952 inflate)
    of the benchmark's member, on one host core, in decompressed GB/s."""
    import oracle

    oracle.lib()
    core = max(os.sched_getaffinity(0))
    a = np.frombuffer(comp, dtype=np.uint8)

    def run():
        t0 = time.perf_counter()
        g = oracle.gunzip(a)
        return g, time.perf_counter() - t0

    g, dt = _pinned(core, run)
    ok = g.status == 0 and g.out.size == n_raw and (zlib.crc32(g.out) & 0xFFFFFFFF) == crc_ref
    del g
    h = host_info()
    return {
        "value": round(n_raw / dt / 1e9, 6),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the whole {workload} member ({n_raw} bytes, {len(comp)} compressed): the oracle's sequential "
                  f"gunzip on one host core (thread pinned to core {core}), {dt:.1f} s, "
                  f"{len(comp) / dt / 1e6:.1f} MB/s compressed, output equal to the source: {ok}",
        "seconds": round(dt, 3),
        "cpu_model": h["cpu_model"],
        "nproc": h["nproc"],
        "affinity_cores": h["affinity_cores"],
    }


def oracle_aggregate(comps, n_raw_total: int):
    """The oracle's gunzip over a set of files with one pinned thread per host
    core (at most 16), files taken from a shared queue; aggregate decompressed
    GB/s.  The oracle runs outside the interpreter lock."""
    import queue
    import threading

    import oracle

    oracle.lib()
    cores = sorted(os.sched_getaffinity(0))[:16]
    q = queue.Queue()
    for c in comps:
        q.put(np.frombuffer(c, dtype=np.uint8))
    bad = []

    def worker(core):
        def loop():
            while True:
                try:
                    a = q.get_nowait()
                except queue.Empty:
                    return
                g = oracle.gunzip(a)
                if g.status != 0:
                    bad.append(g.status)
        _pinned(core, loop)

    th = [threading.Thread(target=worker, args=(c,)) for c in cores]
    t0 = time.perf_counter()
    for t in th:
        t.start()
    for t in th:
        t.join()
    dt = time.perf_counter() - t0
    return {"GBps": round(n_raw_total / dt / 1e9, 4), "cores": len(cores), "seconds": round(dt, 3),
            "files": len(comps), "all_ok": not bad}


def copy_ceiling(dev, mib: int = 2048, reps: int = 5):
    """Device-to-device copy of `mib` MiB (read + write bytes / time): the
    HBM bandwidth a plain streaming kernel reaches on this GPU."""
    import statistics

    import torch

    n = mib << 18
    src = torch.ones(n, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(reps + 1):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = statistics.median(ms[1:])
    del src, dst
    return round(2 * 4 * n / t / 1e6, 1)


def path_bytes_per_out(ratio: float) -> float:
    """Algorithmic HBM bytes per decompressed byte of the whole path: the
    compressed input once, 16-bit symbols written and read, the output
    written (1/R + 5); the 96 KiB of windows per chunk come on top."""
    return 1.0 / ratio + 5.0


def fractions(gbps: float, ratio: float, copy_gbps):
    b = path_bytes_per_out(ratio)
    return {"hbm_frac": round(gbps * b / HBM_PEAK_GBS, 5),
            "copy_frac": round(gbps * b / copy_gbps, 5) if copy_gbps else None}


def timed_plan(gz, plan, out, steps: int, raw_dev=None):
    """Warm up once (output compared with raw_dev when given), then time
    `steps` launches; returns (seconds per step, last result, mean pass times)."""
    import torch

    stream = torch.cuda.current_stream()
    plan.launch(out, stream)
    r = plan.result()
    if r.status != 0:
        raise SystemExit(f"decompression failed: status {r.status}")
    if raw_dev is not None and not (r.out_len == raw_dev.numel() and torch.equal(out[: r.out_len], raw_dev)):
        raise SystemExit("output differs from the source text")
    passes = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.launch(out, stream)
        r = plan.result()
        if r.status != 0:
            raise SystemExit(f"decompression failed: status {r.status}")
        if plan.opts.timing:
            passes.append(plan.pass_times())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    avg = {k: sum(p[k] for p in passes) / len(passes) for k in passes[0]} if passes else {}
    return dt, r, avg


def large_leg(gz, name: str, steps: int, copy_gbps, chunk_sweep=()):
    """One of the large configurations (the level sweep's 4 GiB FASTQ-like
    members, the 2 GiB word stream): decompressed GB/s in the benchmark's
    launch configuration, HBM fractions, per-chunk placeholder fractions
    (Section IV-C's undetermined context, per chunk), the window
    propagation's time and bytes, and the block-start search's stage counts.
    Returns (result dict, raw, comp, segment bits)."""
    import torch

    t = time.perf_counter()
    raw, comp, seg = synth_workload(name)
    gen_s = time.perf_counter() - t
    dev = torch.device("cuda:0")
    d_comp = torch.frombuffer(bytearray(comp), dtype=torch.uint8).to(dev)
    d_raw = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
    out = torch.empty(len(raw), dtype=torch.uint8, device=dev)
    plan = gz.Plan(d_comp, 0, timing=1)
    dt, r, avg = timed_plan(gz, plan, out, steps, d_raw)
    ratio = len(raw) / len(comp)
    gbps = len(raw) / dt / 1e9
    tab = plan.chunk_table()
    st = plan.chunk_stats()
    ne = tab["start"] != np.uint64(gz.NONE)
    L = tab["len"][ne].astype(np.float64)
    ph = st["n_placeholders"][ne].astype(np.float64)
    frac = ph[1:] / np.maximum(L[1:], 1.0)  # chunk 0 has no unknown context
    n_acc = int(ne.sum())
    res = {
        "workload": name,
        "uncompressed_bytes": len(raw),
        "compressed_bytes": len(comp),
        "ratio": round(ratio, 4),
        "generate_s": round(gen_s, 1),
        "n_chunks": plan.n_chunks,
        "chunks_with_start": n_acc,
        "steps": steps,
        "ms_per_step": round(dt * 1e3, 3),
        "GBps": round(gbps, 3),
        **fractions(gbps, ratio, copy_gbps),
        "passes_ms": {k: round(v, 4) for k, v in avg.items()},
        "placeholder_frac": {
            "all_symbols": round(float(ph.sum() / max(L.sum(), 1.0)), 5),
            "chunk_mean": round(float(frac.mean()), 5) if frac.size else None,
            "chunk_p10": round(float(np.percentile(frac, 10)), 5) if frac.size else None,
            "chunk_p50": round(float(np.percentile(frac, 50)), 5) if frac.size else None,
            "chunk_p90": round(float(np.percentile(frac, 90)), 5) if frac.size else None,
            "chunk_max": round(float(frac.max()), 5) if frac.size else None,
        },
        "propagate": {"us": round(avg.get("propagate", 0.0) * 1e3, 1),
                      "algorithmic_bytes": n_acc * 3 * 32768,
                      "note": "per accepted chunk: 32768 16-bit tail symbols read, a 32 KiB window written"},
        "search": {k: int(st[k].sum()) for k in ("stage1", "stage2", "trial_rej", "confirm_rej")},
        "stats": {k: int(getattr(r, k)) for k in ("n_repairs", "n_retries", "n_extended", "n_syms",
                                                   "n_placeholders", "n_blocks")},
        "bit_exact": True,
    }
    for cb in chunk_sweep:
        p2 = gz.Plan(d_comp, 0, chunk_bytes=cb)
        dt2, r2, _ = timed_plan(gz, p2, out, 2, d_raw)
        res.setdefault("chunk_sweep", []).append({"chunk_bytes": cb, "n_chunks": p2.n_chunks,
                                                  "GBps": round(len(raw) / dt2 / 1e9, 3)})
        del p2
    del plan, d_raw, out, d_comp
    torch.cuda.empty_cache()
    return res, raw, comp, seg, tab, st


def synth_workload(name):
    import synth

    return synth.workload(name, index=True)


def false_positives(tab, st, n_repairs: int, gz):
    """Block-start candidates per chunk, from the device's own counts: the
    first bit passing the static checks (header and tables), whether the
    trial and confirmation blocks then rejected it (a false positive caught
    there), and accepted starts that the stitch check found off the block
    chain (false positives that got through, repaired).  The GPU tests check
    the accepted starts against the oracle's block map."""
    none = np.uint64(gz.NONE)
    sc = st["scan_cand"]
    has_sc = sc != none
    fd = tab["cand"]
    has_fd = fd != none
    return {"chunks": int(sc.size), "static_candidates": int(has_sc.sum()),
            "static_rejected_later": int((has_sc & (sc != fd)).sum()),
            "accepted": int(has_fd.sum()), "accepted_off_chain": int(n_repairs),
            "stage1_per_chunk_mean": round(float(st["stage1"].mean()), 3),
            "stage1_per_chunk_max": int(st["stage1"].max()),
            "stage2_per_chunk_mean": round(float(st["stage2"].mean()), 3),
            "trial_rej_per_chunk_max": int(st["trial_rej"].max()),
            "confirm_rej_per_chunk_max": int(st["confirm_rej"].max())}


def batched_vs_plain(n_files: int, reps: int, copy_gbps=None, keep_host=None):
    """Decompressed GB/s of n_files C1-like files (4 MiB FASTQ-like, gzip -6,
    seeds 1..n_files): back-to-back one-file launches on one stream (plain),
    one batched launch sequence (batched), and the batched sequence replayed
    from its HIP graph (graph).  Median over reps; inputs and outputs stay in
    HBM; every output is compared with its source text after the timing."""
    import statistics

    import torch

    import paper_1905_07224_amd as gz
    import synth

    dev = torch.device("cuda:0")
    raws, comps = [], []
    for k in range(1, n_files + 1):
        raw, comp = synth.make("fastq", 4 << 20, k, 6)
        raws.append(raw)
        comps.append(torch.frombuffer(bytearray(comp), dtype=torch.uint8).to(dev))
    total = sum(len(r) for r in raws)
    outs = [torch.empty(len(r), dtype=torch.uint8, device=dev) for r in raws]
    s = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        ms = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                e0.record(s)
                fn()
                e1.record(s)
            s.synchronize()
            ms.append(e0.elapsed_time(e1))
        return statistics.median(ms[1:])

    def exact():
        return all(torch.equal(o, torch.frombuffer(bytearray(r), dtype=torch.uint8).to(dev))
                   for o, r in zip(outs, raws))

    plans = [gz.Plan(c, 0) for c in comps]
    for p_ in plans:
        p_.workspace()

    def plain():
        for p_, o in zip(plans, outs):
            p_.launch(o, s)

    ms_plain = timed(plain)
    ok_plain = all(p_.result().status == 0 for p_ in plans) and exact()
    del plans
    bp = gz.BatchPlan(comps, 0, outs=outs)
    bp.workspace()
    ms_batch = timed(lambda: bp.launch(s))
    ok_batch = all(bp.result(i).status == 0 for i in range(n_files)) and exact()
    ms_graph = timed(lambda: bp.launch_graph(s))
    ok_graph = all(bp.result(i).status == 0 for i in range(n_files)) and exact()
    del bp
    # the autotuner's choice for the files' class (timed on the first file,
    # outside the timed region), applied to the whole batch
    choice = gz.autotune(comps[0])
    bt = gz.BatchPlan(comps, 0, outs=outs, tuned=1)
    bt.workspace()
    ms_tuned = timed(lambda: bt.launch(s))
    ok_tuned = all(bt.result(i).status == 0 for i in range(n_files)) and exact()
    del bt
    comp_total = sum(c.numel() for c in comps)
    ratio = total / comp_total
    if keep_host is not None:
        keep_host.append(("batched set: 32 FASTQ-like 4 MiB files", [c.cpu().numpy().tobytes() for c in comps], total))
    return {
        "files": n_files,
        "uncompressed_bytes": total,
        "compressed_bytes": comp_total,
        "plain_fractions": fractions(total / ms_plain / 1e6, ratio, copy_gbps),
        "batched_fractions": fractions(total / ms_batch / 1e6, ratio, copy_gbps),
        "graph_fractions": fractions(total / ms_graph / 1e6, ratio, copy_gbps),
        "reps": reps,
        "plain_GBps": round(total / ms_plain / 1e6, 4),
        "batched_GBps": round(total / ms_batch / 1e6, 4),
        "graph_GBps": round(total / ms_graph / 1e6, 4),
        "plain_ms": round(ms_plain, 3),
        "batched_ms": round(ms_batch, 3),
        "graph_ms": round(ms_graph, 3),
        "tuned_choice": choice,
        "tuned_GBps": round(total / ms_tuned / 1e6, 4),
        "bit_exact": bool(ok_plain and ok_batch and ok_graph and ok_tuned),
    }


C5_MIN, C5_MAX = 64 << 10, 2 << 30
C5_LOADS = (0.25, 0.5, 0.75, 0.9, 1.0, 1.2)


def c5_pool(n_files: int, seed: int = 5):
    """The job pool of the serving configuration: sizes log-uniform in
    [64 KiB, 2 GiB], FASTQ-like or word-stream text with equal odds, level
    drawn from {1, 6, 9}; file i is generated with seed 100 + i."""
    import synth

    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(C5_MIN), np.log(C5_MAX), n_files)).astype(np.int64)
    kinds = rng.choice(["fastq", "words"], n_files)
    levels = rng.choice([1, 6, 9], n_files)
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        raw, comp = synth.make(str(kinds[i]), int(sizes[i]), 100 + i, int(levels[i]), use_cache=False)
        return str(kinds[i]), int(levels[i]), raw, comp

    # largest first; zlib and the generators release the interpreter lock
    order = sorted(range(n_files), key=lambda i: -sizes[i])
    with ThreadPoolExecutor(max_workers=4) as ex:
        made = dict(zip(order, ex.map(one, order)))
    return [made[i] for i in range(n_files)]


def serving_c5(n_jobs: int, n_files: int, budget_gib: int, copy_gbps, loads=C5_LOADS, keep_host=None):
    """The serving loop under Poisson arrivals on the C5 pool.  Each job
    decompresses one pool file (drawn uniformly) into its own output buffer.
    Capacity is measured closed loop (every job submitted at once); then for
    each offered load, jobs arrive at load x capacity / mean job size.
    Latency = completion seen by the poll - scheduled arrival; GB/s = all
    bytes / (last completion - first arrival).  Every output is compared with
    its source after each run.  Before the runs the pool itself is decoded
    plain (one file after another on one stream), batched (one launch
    sequence); the compressed files are kept for the oracle's aggregate in
    the CPU leg."""
    import statistics

    import torch

    import paper_1905_07224_amd as gz

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    pool = c5_pool(n_files)
    gen_s = time.perf_counter() - t
    raws = [torch.frombuffer(bytearray(r), dtype=torch.uint8).to(dev) for _, _, r, _ in pool]
    comps = [torch.frombuffer(bytearray(c), dtype=torch.uint8).to(dev) for _, _, _, c in pool]
    host_comps = [c for _, _, _, c in pool]
    pool_raw = sum(len(r) for _, _, r, _ in pool)
    pool_comp = sum(len(c) for c in host_comps)
    for k in range(len(pool)):
        pool[k] = pool[k][:2]
    log(f"C5 pool: {n_files} files, {pool_raw / 2**30:.2f} GiB raw, {pool_comp / 2**30:.2f} GiB compressed, "
        f"generated in {gen_s:.1f} s")
    ratio = pool_raw / pool_comp

    # the pool decoded plain and batched
    outs = [torch.empty(r.numel(), dtype=torch.uint8, device=dev) for r in raws]
    s = torch.cuda.Stream()

    def timed(fn, reps=2):
        ms = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                e0.record(s)
                fn()
                e1.record(s)
            s.synchronize()
            ms.append(e0.elapsed_time(e1))
        return statistics.median(ms[1:])

    plans = [gz.Plan(c, 0) for c in comps]
    ws_plain = max(p_.info.ws_bytes for p_ in plans)
    shared = torch.empty(ws_plain + 256, dtype=torch.uint8, device=dev)

    def plain():
        for p_, o in zip(plans, outs):
            p_.launch(o, s, workspace=shared)

    ms_plain = timed(plain)
    # the plans share one workspace, which holds a plan's status until the
    # next plan runs: the last plan's status, and every output, are checked
    ok_plain = plans[-1].result().status == 0 and all(torch.equal(o, r) for o, r in zip(outs, raws))
    del plans, shared
    torch.cuda.empty_cache()
    bp = gz.BatchPlan(comps, 0, outs=outs)
    bp.workspace()
    ms_batch = timed(lambda: bp.launch(s))
    ok_batch = all(bp.result(i).status == 0 for i in range(n_files)) and all(
        torch.equal(o, r) for o, r in zip(outs, raws))
    batch_ws = bp.info.ws_bytes
    del bp, outs
    torch.cuda.empty_cache()
    log("C5 pool decoded plain and batched")
    if keep_host is not None:
        keep_host.append(("serving pool: 32 files, 64 KiB .. 2 GiB", host_comps, pool_raw))
    del host_comps
    pool_sets = {
        "files": n_files, "uncompressed_bytes": pool_raw, "compressed_bytes": pool_comp,
        "kinds_levels": [f"{k}/L{lv}/{r.numel()}" for (k, lv), r in zip(pool, raws)],
        "plain_GBps": round(pool_raw / ms_plain / 1e6, 3), "batched_GBps": round(pool_raw / ms_batch / 1e6, 3),
        "plain_fractions": fractions(pool_raw / ms_plain / 1e6, ratio, copy_gbps),
        "batched_fractions": fractions(pool_raw / ms_batch / 1e6, ratio, copy_gbps),
        "batched_ws_GiB": round(batch_ws / 2**30, 2), "generate_s": round(gen_s, 1),
        "bit_exact": bool(ok_plain and ok_batch),
    }
    log(f"C5 pool sets: {pool_sets}")

    rng = np.random.default_rng(7)
    pick = rng.integers(0, n_files, n_jobs)
    nbytes = np.array([raws[k].numel() for k in pick], dtype=np.int64)
    offs = np.concatenate(([0], np.cumsum(nbytes)))
    big = torch.empty(int(offs[-1]), dtype=torch.uint8, device=dev)
    outs = [big[int(offs[j]):int(offs[j + 1])] for j in range(n_jobs)]
    budget = budget_gib << 30
    mean_job = float(nbytes.mean())

    def run(arrivals):
        srv = gz.Server(budget_bytes=budget, max_inflight=4, max_batch=64)
        t0 = srv.stats()["now"]
        sched = [t0 + a for a in arrivals]
        done, nxt = {}, 0
        while len(done) < n_jobs:
            now = srv.stats()["now"]
            while nxt < n_jobs and sched[nxt] <= now:
                srv.submit(comps[pick[nxt]], outs[nxt], nxt)
                nxt += 1
            for d in srv.poll():
                done[d["tag"]] = d
            if nxt == n_jobs and len(done) < n_jobs:
                time.sleep(0.0002)
            if srv.stats()["now"] - t0 > 150:
                raise SystemExit("serving run did not finish within 150 s")
        info = srv.stats()
        srv.close()
        lat = np.array([done[k]["t_end"] - sched[k] for k in range(n_jobs)]) * 1e3
        span = max(d["t_end"] for d in done.values()) - sched[0]
        ok = all(done[k]["status"] == 0 and done[k]["out_len"] == nbytes[k] for k in range(n_jobs))
        ok = ok and all(torch.equal(outs[k], raws[pick[k]]) for k in range(n_jobs))
        big.zero_()
        gbps = float(nbytes.sum()) / span / 1e9
        return {
            "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "GBps": round(gbps, 3), **fractions(gbps, ratio, copy_gbps), "span_s": round(span, 3),
            "batches": int(info["batches"]), "mem_waited": int(info["mem_waited"]),
            "resident_peak_GiB": round(info["resident_peak"] / 2**30, 2),
            "arena_peak_GiB": round(info["arena_peak"] / 2**30, 2), "bit_exact": bool(ok),
        }

    closed = run([0.0] * n_jobs)
    capacity = closed["GBps"] * 1e9
    log(f"C5 closed loop: {closed}")
    points = []
    for load in loads:
        rate = load * capacity / mean_job
        arr = np.cumsum(rng.exponential(1.0 / rate, n_jobs))
        arr -= arr[0]
        res = run(list(arr))
        res = {"offered_load": load, "arrival_rate_per_s": round(rate, 3), **res}
        log(f"C5 load {load}: {res}")
        points.append(res)
    del big, outs, raws, comps
    torch.cuda.empty_cache()
    return {
        "jobs_per_point": n_jobs,
        "pool": pool_sets,
        "job_sizes": "log-uniform 64 KiB .. 2 GiB over the pool's files, each job drawn uniformly from the pool",
        "mean_job_bytes": int(mean_job),
        "total_bytes_per_point": int(nbytes.sum()),
        "budget_GiB": budget_gib,
        "closed_loop": closed,
        "capacity_GBps": round(capacity / 1e9, 3),
        "load_points": points,
        "bit_exact": bool(closed["bit_exact"] and all(p_["bit_exact"] for p_ in points)),
    }


def streaming(gz, d_comp, seg_bytes: int, n_raw: int, crc_ref: int, whole_bytes: int):
    """The member decoded in segments of seg_bytes compressed bytes (gz_stream_*),
    one output buffer and one workspace reused by every segment; timed over
    the whole member after one untimed pass."""
    import torch

    best = None
    for rep in range(2):
        s = gz.Stream(d_comp, seg_bytes)
        info = s.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        total, n = 0, 0
        for part in s:
            total += part.numel()
            n += 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        crc = s.last["crc32"]
        s.close()
        if total != n_raw or crc != crc_ref:
            raise SystemExit("streamed output differs from the source text (length or CRC-32)")
        if rep == 1:
            best = dt
    return {
        "segment_bytes": seg_bytes,
        "segments": n,
        "GBps": round(n_raw / best / 1e9, 3),
        "device_bytes": info["ws_bytes"] + info["out_bytes"],
        "whole_member_device_bytes": whole_bytes,
        "crc_checked": True,
    }


def bgzf_leg(gz, mib: int):
    """A BGZF-style file (64 KiB members) decoded as one batch of members
    (gz_plan_bgzf + gz_decompress_batch), timed after one untimed run."""
    import ctypes as C

    import torch

    import synth

    raw = synth.fastq_like(mib << 20, 2, read_lens=(100, 150))
    comp = synth.bgzf(raw, 6)
    d = torch.frombuffer(bytearray(comp), dtype=torch.uint8).cuda()
    out = torch.empty(len(raw), dtype=torch.uint8, device="cuda")
    L = gz.lib()
    hbuf = (C.c_uint8 * len(comp)).from_buffer_copy(comp)
    n_out, n_mem = C.c_uint64(), C.c_uint32()
    h = C.c_void_p()
    gz._check(L.gz_plan_bgzf(C.byref(h), C.c_void_p(d.data_ptr()), hbuf, d.numel(), C.c_void_p(out.data_ptr()),
                             out.numel(), C.byref(gz._opts()), C.byref(n_out), C.byref(n_mem)))
    try:
        info = gz.Info()
        gz._check(L.gz_plan_info(h, C.byref(info)))
        ws = torch.empty(info.ws_bytes, dtype=torch.uint8, device="cuda")
        st = torch.cuda.current_stream()
        best = None
        for rep in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gz._check(L.gz_decompress_batch(h, C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(st.cuda_stream)))
            for f in range(n_mem.value):
                r = gz.Result()
                gz._check(L.gz_result_get(h, f, C.byref(r)))
                if r.status != 0:
                    raise SystemExit(f"BGZF member {f} failed: status {r.status}")
            dt = time.perf_counter() - t0
            if rep and (best is None or dt < best):
                best = dt
        exact = bool(torch.equal(out, torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()))
        if not exact:
            raise SystemExit("BGZF output differs from the source text")
    finally:
        L.gz_plan_destroy(h)
    return {"uncompressed_bytes": len(raw), "compressed_bytes": len(comp), "members": n_mem.value,
            "GBps": round(len(raw) / best / 1e9, 3), "ms": round(best * 1e3, 3), "bit_exact": True}


def pair_batched(gz, files, copy_gbps):
    """The two level-sweep members together: back-to-back one-file launches
    on one stream (plain, one shared workspace) against one batched launch
    sequence; outputs compared with the sources."""
    import statistics

    import torch

    dev = torch.device("cuda:0")
    raws = [torch.frombuffer(bytearray(r), dtype=torch.uint8).to(dev) for r, _ in files]
    comps = [torch.frombuffer(bytearray(c), dtype=torch.uint8).to(dev) for _, c in files]
    outs = [torch.empty_like(r) for r in raws]
    total = sum(r.numel() for r in raws)
    ratio = total / sum(c.numel() for c in comps)
    s = torch.cuda.Stream()

    def timed(fn, reps=2):
        ms = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                e0.record(s)
                fn()
                e1.record(s)
            s.synchronize()
            ms.append(e0.elapsed_time(e1))
        return statistics.median(ms[1:])

    plans = [gz.Plan(c, 0) for c in comps]
    shared = torch.empty(max(p_.info.ws_bytes for p_ in plans), dtype=torch.uint8, device=dev)

    def plain():
        for p_, o in zip(plans, outs):
            p_.launch(o, s, workspace=shared)

    ms_plain = timed(plain)
    ok = plans[-1].result().status == 0 and all(torch.equal(o, r) for o, r in zip(outs, raws))
    del plans, shared
    torch.cuda.empty_cache()
    for o in outs:
        o.zero_()
    bp = gz.BatchPlan(comps, 0, outs=outs)
    bp.workspace()
    ms_batch = timed(lambda: bp.launch(s))
    ok = ok and all(bp.result(i).status == 0 for i in range(len(files))) and all(
        torch.equal(o, r) for o, r in zip(outs, raws))
    del bp, outs, raws, comps
    torch.cuda.empty_cache()
    g_p, g_b = total / ms_plain / 1e6, total / ms_batch / 1e6
    return {"files": len(files), "uncompressed_bytes": total, "plain_GBps": round(g_p, 3),
            "batched_GBps": round(g_b, 3), "plain_fractions": fractions(g_p, ratio, copy_gbps),
            "batched_fractions": fractions(g_b, ratio, copy_gbps), "bit_exact": bool(ok)}


def binary_leg(gz, mib: int, steps: int, copy_gbps):
    """Binary input (counters, random walks, noisy floats, random stretches
    stored): decompressed GB/s with the binary option (block starts searched
    without the ASCII test), default chunking."""
    import torch

    import synth

    t = time.perf_counter()
    raw = synth.binary_records(mib << 20, 11)
    comp = synth.gzip_member(raw, 6)
    gen_s = time.perf_counter() - t
    dev = torch.device("cuda:0")
    d_comp = torch.frombuffer(bytearray(comp), dtype=torch.uint8).to(dev)
    d_raw = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
    out = torch.empty(len(raw), dtype=torch.uint8, device=dev)
    plan = gz.Plan(d_comp, 0, binary=1, timing=1)
    dt, r, avg = timed_plan(gz, plan, out, steps, d_raw)
    tab = plan.chunk_table()
    n_acc = int((tab["start"] != np.uint64(gz.NONE)).sum())
    gbps = len(raw) / dt / 1e9
    res = {"uncompressed_bytes": len(raw), "compressed_bytes": len(comp), "level": 6, "generate_s": round(gen_s, 1),
           "n_chunks": plan.n_chunks, "chunks_with_start": n_acc, "GBps": round(gbps, 3),
           **fractions(gbps, len(raw) / len(comp), copy_gbps), "n_repairs": int(r.n_repairs),
           "n_retries": int(r.n_retries), "bit_exact": True}
    del plan, d_raw, out, d_comp
    torch.cuda.empty_cache()
    return res


def recorded_traffic(kernel: str, workload: str, chunk_bytes: int, window: int):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when that summary was taken on other kernel sources or
    another configuration."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"hbm_k_inflate_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if " = " in line and not line.startswith(("|", " ")):
            k, v = line.strip().split(" = ", 1)
            kv[k] = v
    h = hashlib.sha256()
    for f in ("gz_kernels.hip", "gz_device.h", "gz_internal.h"):
        with open(os.path.join(ROOT, "paper_1905_07224_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    same = (kv.get("source_sha256") == h.hexdigest() and kv.get("kernel", "").endswith(kernel)
            and kv.get("workload") == workload and kv.get("chunk_bytes") == str(chunk_bytes)
            and kv.get("window_syms") == str(window))
    return int(kv["traffic_bytes"]) if same else None


LEGS = ("c2_1mib", "c3", "c4", "stream", "binary", "bgzf", "batched", "serving", "cpu")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fastq_1GiB_L6")
    ap.add_argument("--chunk-bytes", type=int, default=0, help="compressed bytes per chunk (0: library default)")
    ap.add_argument("--waves-per-chunk", type=int, default=1)
    ap.add_argument("--window", type=int, default=0, help="LDS history ring per decoding wave (0: library default)")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="legs beside the timed plain run: " + ",".join(LEGS) + " (empty: none)")
    ap.add_argument("--large-steps", type=int, default=3, help="timed steps of the level-sweep and word legs")
    ap.add_argument("--batch-files", type=int, default=32, help="files of the batched-vs-plain set")
    ap.add_argument("--serve-jobs", type=int, default=500, help="jobs per load point of the serving runs")
    ap.add_argument("--serve-files", type=int, default=32, help="files of the serving pool")
    ap.add_argument("--serve-budget-gib", type=int, default=64, help="HBM budget of the jobs in flight")
    ap.add_argument("--stream-mib", type=int, default=256, help="streaming leg: compressed MiB per segment")
    ap.add_argument("--bgzf-mib", type=int, default=256, help="BGZF leg: MiB of FASTQ-like text in 64 KiB members")
    ap.add_argument("--binary-mib", type=int, default=512, help="binary leg: MiB of binary records")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after warmup, one device-to-device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: runs on one GPU only; the chunk chain is not sharded over several GPUs",
              file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x)
    unknown = legs - set(LEGS)
    if unknown:
        raise SystemExit(f"unknown legs: {sorted(unknown)}")

    import torch

    import paper_1905_07224_amd as gz
    import synth

    t = time.perf_counter()
    log(f"workload {args.workload}: generating / loading")
    raw, comp = synth.workload(args.workload)
    log(f"input ready: {len(raw)} bytes raw, {len(comp)} compressed (ratio {len(raw) / len(comp):.3f}) "
        f"in {time.perf_counter() - t:.1f} s")
    crc_ref = zlib.crc32(raw) & 0xFFFFFFFF
    ratio = len(raw) / len(comp)

    dev = torch.device("cuda:0")
    d_comp = torch.frombuffer(bytearray(comp), dtype=torch.uint8).to(dev)
    out = torch.empty(len(raw), dtype=torch.uint8, device=dev)
    window = args.window or gz.DEFAULT_WINDOW
    # chunk_bytes 0: the library's default (40 KiB)
    plan = gz.Plan(d_comp, 0, chunk_bytes=args.chunk_bytes, waves_per_chunk=args.waves_per_chunk,
                   window_syms=window, timing=1)
    n_chunks = plan.n_chunks
    chunk_bytes = (plan.info.payload_end - plan.info.payload_start + n_chunks - 1) // n_chunks
    log(f"plan: {n_chunks} chunks, workspace {plan.info.ws_bytes / 2**30:.2f} GiB")
    stream = torch.cuda.current_stream()

    # warmup, with a byte-exact check of the output against the source text
    for w in range(max(1, args.warmup)):
        plan.launch(out, stream)
        r = plan.result()
        if r.status != 0:
            raise SystemExit(f"decompression failed: status {r.status}")
        if w == 0:
            ref = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
            exact = bool(torch.equal(out[: r.out_len], ref)) and r.out_len == len(raw)
            del ref
            log(f"warmup: status {r.status}, byte-exact {exact}, passes {plan.pass_times()}")
            if not exact:
                raise SystemExit("output differs from the source text")

    if args.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings scale
        # the counters of the decompression kernels to bytes
        n = args.calib_copy_mib << 18
        src = torch.ones(n, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {n * 4} bytes read and written")
        del src, dst

    # timed steps
    passes = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch(out, stream)
        r = plan.result()  # waits for the stream
        if r.status != 0:
            raise SystemExit(f"decompression failed: status {r.status}")
        passes.append(plan.pass_times())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = plan.result().as_dict()
    ms_step = dt / args.steps * 1e3
    value = len(raw) * args.steps / dt / 1e9
    log(f"timed: {args.steps} steps, {ms_step:.2f} ms/step, {value:.2f} GB/s decompressed")

    # output check after the timed steps: length and CRC-32 against the trailer
    crc_out = zlib.crc32(out.cpu().numpy().tobytes()) & 0xFFFFFFFF
    if crc_out != crc_ref:
        raise SystemExit("CRC-32 of the output differs after the timed steps")

    avg = {k: sum(p[k] for p in passes) / len(passes) for k in passes[0]}
    inflate_ms = avg["inflate"]
    # algorithmic bytes of one inflate launch: read the compressed payload once,
    # write one 16-bit symbol per decompressed byte
    inflate_bytes = len(comp) + 2 * len(raw)
    achieved = inflate_bytes / (inflate_ms / 1e3) / 1e9
    kname = f"k_inflate<{window}, false>"
    roofline = {
        "kernel": kname,
        "bound": "hbm",
        "achieved": round(achieved, 3),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 6),
        "traffic": recorded_traffic(kname, args.workload, chunk_bytes, window),
        "algorithmic_bytes": inflate_bytes,
        "avg_ms": round(inflate_ms, 4),
    }
    # the decoder's serial chain: codes and output symbols per wave-cycle
    waves = int(stats["inflate_waves"])
    wave_cycles = inflate_ms * 1e-3 * CLOCK_GHZ * 1e9 * waves
    decoder = {
        "inflate_waves": waves,
        "codes": int(stats["n_syms"]),
        "codes_per_wave_cycle": round(stats["n_syms"] / wave_cycles, 5),
        "out_symbols_per_wave_cycle": round(len(raw) / wave_cycles, 5),
        "note": "wave-cycles = inflate time x 2.4 GHz x decoding waves of the persistent grid",
    }
    copy_gbps = copy_ceiling(dev)
    log(f"copy ceiling: {copy_gbps} GB/s")
    path = {"bytes_per_out_byte": round(path_bytes_per_out(ratio), 4), "copy_ceiling_GBps": copy_gbps,
            **fractions(value, ratio, copy_gbps)}

    extra = {}
    if "c2_1mib" in legs:
        p1 = gz.Plan(d_comp, 0, chunk_bytes=1 << 20)
        dt1, _, _ = timed_plan(gz, p1, out, 3)
        extra["c2_1MiB_chunks"] = {"chunk_bytes": 1 << 20, "n_chunks": p1.n_chunks,
                                   "GBps": round(len(raw) / dt1 / 1e9, 3), **fractions(len(raw) / dt1 / 1e9, ratio,
                                                                                       copy_gbps)}
        log(f"C2 at 1 MiB chunks: {extra['c2_1MiB_chunks']}")
        del p1

    streamed = None
    if "stream" in legs:
        whole_bytes = plan.info.ws_bytes + out.numel()
        log(f"streaming: {args.stream_mib} MiB segments")
        streamed = streaming(gz, d_comp, args.stream_mib << 20, len(raw), crc_ref, whole_bytes)
        log(f"streaming: {streamed}")
    del plan, out, d_comp
    torch.cuda.empty_cache()

    if "c3" in legs:
        pair = []
        for name in ("fastq_4GiB_L1", "fastq_4GiB_L9"):
            log(f"level sweep: {name}")
            res, raw3, comp3, *_ = large_leg(gz, name, args.large_steps, copy_gbps,
                                             chunk_sweep=(256 << 10, 1 << 20, 4 << 20))
            extra[name] = res
            pair.append((raw3, comp3))
            log(f"{name}: {res}")
        log("level sweep pair: plain and batched")
        extra["fastq_4GiB_L1+L9"] = pair_batched(gz, pair, copy_gbps)
        log(f"pair: {extra['fastq_4GiB_L1+L9']}")
        del pair
    if "c4" in legs:
        name = "words_2GiB_L6"
        log(f"word stream: {name}")
        res, raw4, comp4, seg4, tab4, st4 = large_leg(gz, name, args.large_steps, copy_gbps)
        res["false_positives"] = false_positives(tab4, st4, res["stats"]["n_repairs"], gz)
        extra[name] = res
        log(f"{name}: {res}")
        del raw4, comp4

    if "binary" in legs:
        log(f"binary input: {args.binary_mib} MiB")
        extra["binary_records"] = binary_leg(gz, args.binary_mib, args.large_steps, copy_gbps)
        log(f"binary: {extra['binary_records']}")

    bgzf = None
    if "bgzf" in legs:
        log(f"bgzf: {args.bgzf_mib} MiB in 64 KiB members")
        bgzf = bgzf_leg(gz, args.bgzf_mib)
        log(f"bgzf: {bgzf}")

    host_sets = []  # compressed sets kept for the oracle's multi-core aggregate (CPU leg)
    batched = None
    if "batched" in legs:
        torch.cuda.empty_cache()
        log(f"batched vs plain: {args.batch_files} C1-like files")
        batched = batched_vs_plain(args.batch_files, 5, copy_gbps, keep_host=host_sets)
        log(f"batched vs plain: {batched}")

    served = None
    if "serving" in legs:
        torch.cuda.empty_cache()
        log(f"serving: {args.serve_jobs} jobs per load point, pool of {args.serve_files} files")
        served = serving_c5(args.serve_jobs, args.serve_files, args.serve_budget_gib, copy_gbps, keep_host=host_sets)
        log(f"serving: {served}")

    cpu = None
    if "cpu" in legs:
        log("cpu baseline: the oracle's gunzip of the whole member on one core")
        cpu = cpu_baseline(comp, len(raw), crc_ref, args.workload)
        cpu["aggregates"] = []
        for what, comps_h, total in host_sets:
            log(f"cpu baseline: the oracle's gunzip over the {what}, one pinned thread per core")
            cpu["aggregates"].append({"set": what, **oracle_aggregate(comps_h, total)})
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "decompressed GB/s on 1 MI355X (batched vs plain) + p50/p99 job latency; bit-exact",
        "value": round(value, 4),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "path": "plain",
            "uncompressed_bytes": len(raw),
            "compressed_bytes": len(comp),
            "ratio": round(ratio, 4),
            "compression": "zlib level 6, one member; above 64 MiB of text it is compressed as 64 MiB "
                           "segments, each primed with the previous 32 KiB and ended by a sync flush "
                           "(pigz-style, still one member)",
            "chunk_bytes": chunk_bytes,
            "waves_per_chunk": args.waves_per_chunk,
            "n_chunks": n_chunks,
            "window_syms": window,
            "compressed_MBps": round(len(comp) * args.steps / dt / 1e6, 1),
        },
        "passes_ms": {k: round(v, 4) for k, v in avg.items()},
        "stats": {k: stats[k] for k in ("n_nonempty", "n_repairs", "n_extended", "n_retries", "n_syms",
                                         "n_placeholders", "n_blocks")},
        "roofline": roofline,
        "path": path,
        "decoder": decoder,
        "configs": extra,
        "streaming": streamed,
        "bgzf": bgzf,
        "batched_vs_plain": batched,
        "serving": served,
        "cpu_baseline": cpu,
        "host": host_info(),
        "bit_exact": True,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
