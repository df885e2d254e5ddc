#!/usr/bin/env python3
"""Benchmark of the comparable-corpus miner on one MI355X.

One step = one pass of the whole mining path over the batch workload
(10,000 document pairs, 20-200 sentences per side): similarity kernel,
Needleman-Wunsch with device traceback and threshold, compaction.  Inputs
(documents and lexicon) are resident in HBM before the timed region.

Prints one JSON line with throughput (document pairs/s and NW GCUPS), the
dominant kernel's roofline figures (kernel durations measured with HIP events
on the launch stream), the plain per-pair GPU form on the same pairs, and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NW GCUPS + doc pairs/s at 1 GPU; served p50/p99 latency vs plain per-pair GPU"

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ, LANES = 256, 2.4, 64
ALU_PEAK_TOPS = CUS * LANES * CLOCK_GHZ * 1e9 / 1e12  # 32-bit VALU lane operations per second (non-packed)


def profiled_traffic(kernel, workload_name):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when the
    summary is for another workload or the kernel source has changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_name}.md")
    src = os.path.join(ROOT, "paper_1509_08639_amd", "csrc", "kernels.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes " + re.escape(kernel) + r": (\d+)", text)
    h = re.search(r"sha256\s+([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != sha:
        return None
    return int(m.group(1))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload_stats(corpus, lex):
    """Mean sentence lengths and mean fan-out of source tokens (per-cell figures)."""
    n, m = corpus.nm()
    cells = int((n * m).sum())
    src_len = np.diff(corpus.src_sent_off)
    tgt_len = np.diff(corpus.tgt_sent_off)
    # cell-weighted means: sum over cells of a_i equals sum_p m_p * sum_i a_i
    src_tok_pp = np.add.reduceat(src_len, corpus.src_doc_off[:-1]) if src_len.size else np.zeros(0)
    tgt_tok_pp = np.add.reduceat(tgt_len, corpus.tgt_doc_off[:-1]) if tgt_len.size else np.zeros(0)
    sum_a = float((src_tok_pp * m).sum())
    sum_b = float((tgt_tok_pp * n).sum())
    fan = np.zeros(int(max(lex.src_ids.max(initial=0), corpus.src_tok.max(initial=0))) + 1, np.int64)
    fan[lex.src_ids] = np.diff(lex.off)
    k_src = fan[np.clip(corpus.src_tok, 0, fan.size - 1)]
    k_src[corpus.src_tok < 0] = 0
    # sum over cells of k-weighted source length = sum_p m_p * sum_{tokens of p} k
    kt = np.zeros(corpus.src_sent_off.shape[0] - 1, np.float64)
    if corpus.src_tok.size:
        kt = np.add.reduceat(k_src.astype(np.float64), corpus.src_sent_off[:-1]) * (src_len > 0)
    k_pp = np.add.reduceat(kt, corpus.src_doc_off[:-1]) if kt.size else np.zeros(0)
    sum_ka = float((k_pp * m).sum())
    return dict(cells=cells, mean_a=sum_a / cells, mean_b=sum_b / cells, mean_ka=sum_ka / cells,
                src_tokens=int(corpus.src_tok.size), tgt_tokens=int(corpus.tgt_tok.size))


def served(ctx_cls, ymine, synth, seconds, rate, log_every=2.0):
    """Poisson arrivals of single document pairs (the served workload) replayed in
    real time against (a) the continuous-batching server and (b) the plain
    per-pair GPU form, FIFO, one request at a time.  Latency = completion minus
    scheduled arrival."""
    import threading
    cfg = synth.CONFIGS[3]
    n_req = int(seconds * rate)
    lex = synth.make_lexicon(cfg)
    corp = synth.generate(cfg, lex, pair_ids=np.arange(n_req))
    w = synth.weights(cfg.seed)
    arr = synth.arrivals(cfg.seed, rate, n_req)
    reqs = [ymine.prepare(corp.slice(k, k + 1)) for k in range(n_req)]
    n, m = corp.nm()
    ctx = ctx_cls(0)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    prm = ymine.params(w, -0.2, 0.5)
    out = {}

    # (a) server, steps launched eagerly and captured into hipGraphs
    ymine.mine_prepared(ctx, L, reqs[0], prm)  # warm the kernels
    results_srv = {}

    def run_server(use_graph):
        srv = ymine.Server(ctx, L, w, -0.2, 0.5, max_pairs_per_step=512, max_cells_per_step=1 << 25,
                           use_graph=use_graph)
        done_ns = np.zeros(n_req, np.int64)
        ticket_of = {}
        lock = threading.Lock()
        t0 = time.monotonic_ns() + 200_000_000

        def submitter():
            for k in range(n_req):
                due = t0 + int(arr[k] * 1e9)
                while True:
                    now = time.monotonic_ns()
                    if now >= due:
                        break
                    time.sleep(min((due - now) / 1e9, 0.0005))
                t = srv.submit_prepared(reqs[k])
                with lock:
                    ticket_of[t] = k

        th = threading.Thread(target=submitter)
        th.start()
        got = 0
        last = time.time()
        while got < n_req:
            r = srv.next_done(1_000_000)
            if r is None:
                continue
            t, dn = r
            with lock:
                k = ticket_of.get(t)
            while k is None:
                time.sleep(0.0001)
                with lock:
                    k = ticket_of.get(t)
            res = srv.poll(t, 0)
            done_ns[k] = dn
            if k % 97 == 0:
                results_srv.setdefault(k, []).append(res)
            got += 1
            if time.time() - last > log_every:
                log(f"[serve] server (graph={use_graph}): {got}/{n_req} done")
                last = time.time()
        th.join()
        stats = srv.stats()
        gstats = srv.graph_stats()
        srv.stop()
        lat = (done_ns - (t0 + (arr * 1e9).astype(np.int64))) / 1e6
        span = (done_ns.max() - t0) / 1e9
        r = dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                 mean_ms=float(lat.mean()), max_ms=float(lat.max()), throughput_pairs_per_s=n_req / span,
                 steps=stats["steps"], pairs_per_step=stats["completed"] / max(stats["steps"], 1))
        if use_graph:
            r.update(graph_instantiations=gstats["instantiations"], graph_updates=gstats["updates"])
        log(f"[serve] server (graph={use_graph}) {r}")
        return r

    out["server"] = run_server(0)
    out["server_graph"] = run_server(1)

    # (b) plain per-pair GPU form, FIFO on the same trace (bounded to the same wall time + 20 s)
    lat_pp = []
    same = True
    t0b = time.monotonic_ns() + 100_000_000
    deadline = t0b + int((seconds + 20) * 1e9)
    for k in range(n_req):
        due = t0b + int(arr[k] * 1e9)
        now = time.monotonic_ns()
        if now < due:
            time.sleep((due - now) / 1e9)
        res = ymine.mine_prepared(ctx, L, reqs[k], prm, per_pair=True)
        fin = time.monotonic_ns()
        lat_pp.append((fin - due) / 1e6)
        for other in results_srv.get(k, []):
            same &= all(np.array_equal(res[x], other[x]) for x in res)
        if fin > deadline:
            break
    lat_pp = np.array(lat_pp)
    out["plain_per_pair"] = dict(p50_ms=float(np.percentile(lat_pp, 50)), p99_ms=float(np.percentile(lat_pp, 99)),
                                 mean_ms=float(lat_pp.mean()), completed=int(lat_pp.size),
                                 throughput_pairs_per_s=lat_pp.size / ((time.monotonic_ns() - t0b) / 1e9))
    out["results_identical_on_sample"] = bool(same)
    out["workload"] = dict(name=cfg.name, requests=n_req, rate_per_s=rate, seconds=seconds,
                           cells=int((n * m).sum()), max_cells=int((n * m).max()))
    log(f"[serve] plain per-pair {out['plain_per_pair']}")
    L.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=1, help="workload index (default: the 10k-pair batch)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample (0: skip)")
    ap.add_argument("--per-pair-sample", type=int, default=1000, help="pairs timed in the plain per-pair form")
    ap.add_argument("--serve-seconds", type=float, default=5.0, help="length of the served arrival trace (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate of the served trace")
    ap.add_argument("--max-pairs", type=int, default=100000,
                    help="pairs generated for a workload larger than this (its first pairs; 0: all)")
    ap.add_argument("--autotune-pairs", type=int, default=10000,
                    help="sample size for the autotuner before the timed region (0: default configuration)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (calibrates the HBM byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the miner shards document pairs across GPUs with no exchange "
              "step, and this build runs and reports the single-GPU path only (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1509_08639_amd import ymine

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        n = args.copy_probe << 18  # float32 elements in MIB MiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4}))
        return

    cfg = synth.CONFIGS[args.workload]
    log(f"[bench] generating workload {cfg.name} ...")
    t = time.time()
    lex = synth.make_lexicon(cfg)
    n_gen = min(cfg.n_pairs, args.max_pairs) if args.max_pairs > 0 else cfg.n_pairs
    corpus = synth.generate(cfg, lex, pair_ids=np.arange(n_gen)) if n_gen < cfg.n_pairs else synth.generate(cfg, lex)
    w = synth.weights(cfg.seed)
    gap, tau = np.float32(-0.2), np.float32(0.5)
    st = workload_stats(corpus, lex)
    log(f"[bench] {corpus.n_pairs} pairs, {st['cells']} cells, generated in {time.time() - t:.1f}s")

    ctx = ymine.Context(0)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    # autotuner (untimed): launch configuration picked on a sample of the batch
    tuning = None
    if args.autotune_pairs > 0:
        sample = corpus.subset(np.linspace(0, corpus.n_pairs - 1, min(args.autotune_pairs, corpus.n_pairs)).astype(int))
        t = time.time()
        best, best_ms = ymine.autotune(ctx, L, sample, w, gap, tau, reps=5)
        tuning = dict(best, sample_pairs=sample.n_pairs, sample_ms=best_ms, seconds=round(time.time() - t, 2))
        log(f"[bench] autotune: {tuning}")
    dm = ymine.DeviceMiner(ctx, L, corpus)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        dm.run(w, gap, tau)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dm.run(w, gap, tau)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    elapsed = t1 - t0
    ms_per_step = elapsed / args.steps * 1e3
    pairs_per_s = corpus.n_pairs * args.steps / elapsed
    gcups = st["cells"] * args.steps / elapsed / 1e9
    res = dm.result()
    n_mined = int(res["pair_off"][-1])
    log(f"[bench] {ms_per_step:.3f} ms/step, {pairs_per_s:.0f} pairs/s, {gcups:.1f} GCUPS, {n_mined} mined pairs")

    # per-kernel average durations (HIP events on the launch stream)
    kern = {}
    for k, (ms, n) in prof.items():
        kern[k] = dict(avg_ms=ms / max(n, 1), launches=n)
    cells = st["cells"]
    # algorithmic work per cell
    sim_ops_per_cell = st["mean_b"] + st["mean_ka"] + 20.0
    sim_ops = sim_ops_per_cell * cells
    nw_bytes = 4.25 * cells
    sim_ms, nw_ms = kern["similarity"]["avg_ms"], kern["nw"]["avg_ms"]
    kern["similarity"].update(bound="alu", algorithmic_ops=sim_ops,
                              achieved_TOPs=sim_ops / (sim_ms * 1e-3) / 1e12 if sim_ms else None)
    kern["nw"].update(bound="hbm", algorithmic_bytes=nw_bytes,
                      achieved_GBs=nw_bytes / (nw_ms * 1e-3) / 1e9 if nw_ms else None,
                      gcups=cells / (nw_ms * 1e-3) / 1e9 if nw_ms else None)
    if sim_ms >= nw_ms:
        ach = kern["similarity"]["achieved_TOPs"]
        roof = dict(kernel="similarity", bound="alu", achieved=ach, peak=ALU_PEAK_TOPS, unit="TOP/s",
                    frac=ach / ALU_PEAK_TOPS, traffic=profiled_traffic("sim_kernel", cfg.name),
                    per_unit=f"{sim_ops_per_cell:.2f} ops/cell (mean b + mean k*a + 20)")
    else:
        ach = kern["nw"]["achieved_GBs"]
        roof = dict(kernel="nw", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    traffic=profiled_traffic("nw_kernel", cfg.name), per_unit="4.25 B/cell")

    # plain per-pair GPU form vs the batched form on the same pairs (host entry points, both
    # copy inputs in and results out)
    plain = None
    if args.per_pair_sample > 0:
        sub = corpus.subset(np.arange(min(args.per_pair_sample, corpus.n_pairs)))
        ymine.mine(ctx, L, sub, w, gap, tau)  # warm
        ta = time.perf_counter()
        rb = ymine.mine(ctx, L, sub, w, gap, tau)
        tb = time.perf_counter()
        rp = ymine.mine_per_pair(ctx, L, sub, w, gap, tau)
        tc = time.perf_counter()
        same = all(np.array_equal(rb[k], rp[k]) for k in rb)
        plain = dict(pairs=sub.n_pairs, batched_pairs_per_s=sub.n_pairs / (tb - ta),
                     per_pair_pairs_per_s=sub.n_pairs / (tc - tb), speedup=(tc - tb) / (tb - ta), identical=same)
        log(f"[bench] plain per-pair: {plain}")

    # CPU oracle on a bounded sample of the same workload
    cpu = cpu_mt = None
    if args.cpu_seconds > 0:
        import oracle
        O = oracle.default()
        OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
        done, tc0 = 0, time.perf_counter()
        step = 8
        while time.perf_counter() - tc0 < args.cpu_seconds and done < corpus.n_pairs:
            sub = corpus.subset(np.arange(done, min(done + step, corpus.n_pairs)))
            O.mine(OL, sub, w, gap, tau)
            done += sub.n_pairs
        el = time.perf_counter() - tc0
        cpu = dict(value=done / el, unit="doc pairs/s", cores=1, kind="oracle",
                   sample=f"first {done} pairs of the {corpus.n_pairs}-pair batch, single thread, {el:.1f} s")
        log(f"[bench] cpu oracle: {cpu}")
        # all host cores: the same per-pair oracle over worker threads (multi-threaded miner)
        threads = len(os.sched_getaffinity(0))
        nsub = min(corpus.n_pairs, max(threads * 8, int(cpu["value"] * threads * args.cpu_seconds * 0.5)))
        sub = corpus.slice(0, nsub)
        tc0 = time.perf_counter()
        O.mine_threads(OL, sub, w, gap, tau, threads)
        el = time.perf_counter() - tc0
        cpu_mt = dict(value=nsub / el, unit="doc pairs/s", cores=threads, kind="oracle_threads",
                      sample=f"first {nsub} pairs of the batch, {threads} threads, {el:.1f} s")
        log(f"[bench] cpu oracle, all cores: {cpu_mt}")

    serve = None
    if args.serve_seconds > 0:
        serve = served(ymine.Context, ymine, synth, args.serve_seconds, args.serve_rate)

    line = {
        "metric": METRIC,
        "value": pairs_per_s,
        "unit": "doc pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n_pairs": corpus.n_pairs, "workload_pairs": cfg.n_pairs, "cells": cells,
                   "src_tokens": st["src_tokens"], "tgt_tokens": st["tgt_tokens"], "gap": float(gap),
                   "threshold": float(tau), "parallelism": "single GPU", "tuning": tuning},
        "gcups": gcups,
        "mined_pairs": n_mined,
        "kernels": kern,
        "roofline": roof,
        "plain_per_pair": plain,
        "served": serve,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_mt,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
