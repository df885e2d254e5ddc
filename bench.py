#!/usr/bin/env python3
"""Benchmark of the comparable-corpus miner on one MI355X.

One step = one pass of the whole mining path over the headline workload,
scale_1M_lognormal60: 1,000,000 document pairs with lognormal sentence counts
(median 60, sigma 0.8, cap 1500), sentences of 3-60 tokens, vocabulary 1M per
language and a 4M-entry lexicon.  A pass runs the token translation, the
similarity kernel, Needleman-Wunsch with device traceback and threshold, and
the compaction.  Documents and lexicon are resident in HBM before the timed
region.

Prints one JSON line: throughput (document pairs/s, GCUPS), the dominant
kernel's roofline figures (kernel durations from HIP events on the launch
stream), the other batch workloads, the plain per-pair GPU form, the served
stream and an overloaded served stream, and the CPU oracle timed on a bounded
sample of the headline workload: the last pairs of the batch, whose token
offsets lie beyond 2^31, also compared with the GPU's results for them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NW GCUPS + doc pairs/s at 1 GPU; served p50/p99 latency vs plain per-pair GPU"

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
CUS, CLOCK_GHZ, LANES = 256, 2.4, 64
ALU_PEAK_TOPS = CUS * LANES * CLOCK_GHZ * 1e9 / 1e12  # 32-bit VALU lane operations per second (non-packed)
TOL_S = 1e-6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def workload_stats(corpus, lex):
    """Cell-weighted mean sentence lengths and translation counts (per-cell figures)."""
    n, m = corpus.nm()
    cells = int((n * m).sum())
    src_len = np.diff(corpus.src_sent_off)
    tgt_len = np.diff(corpus.tgt_sent_off)
    src_tok_pp = np.add.reduceat(src_len, corpus.src_doc_off[:-1]) * (n > 0) if src_len.size else np.zeros(0)
    tgt_tok_pp = np.add.reduceat(tgt_len, corpus.tgt_doc_off[:-1]) * (m > 0) if tgt_len.size else np.zeros(0)
    sum_a = float((src_tok_pp * m).sum())
    sum_b = float((tgt_tok_pp * n).sum())
    fan = np.zeros(int(max(lex.src_ids.max(initial=0), corpus.src_tok.max(initial=0))) + 1, np.int32)
    fan[lex.src_ids] = np.diff(lex.off)
    k_src = fan[np.clip(corpus.src_tok, 0, fan.size - 1)].astype(np.float64)
    k_src[corpus.src_tok < 0] = 0
    cs = np.concatenate([[0.0], np.cumsum(k_src)])
    kt = cs[corpus.src_sent_off[1:]] - cs[corpus.src_sent_off[:-1]]  # per sentence
    ks = np.concatenate([[0.0], np.cumsum(kt)])
    k_pp = ks[corpus.src_doc_off[1:]] - ks[corpus.src_doc_off[:-1]]
    sum_ka = float((k_pp * m).sum())
    return dict(cells=cells, mean_a=sum_a / cells, mean_b=sum_b / cells, mean_ka=sum_ka / cells,
                src_tokens=int(corpus.src_tok.size), tgt_tokens=int(corpus.tgt_tok.size))


def timed_passes(torch, ctx, dm, w, gap, tau, steps, warmup):
    """Warmup passes, then `steps` timed passes bracketed by synchronisation;
    per-kernel average durations from HIP events on the launch stream."""
    for _ in range(warmup):
        dm.run(w, gap, tau)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dm.run(w, gap, tau)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    kern = {k: dict(avg_ms=ms / max(n, 1), launches=n, launches_per_step=n / steps, ms_per_step=ms / steps)
            for k, (ms, n) in prof.items()}
    return (t1 - t0) / steps, kern


def roofline(kern, st, name):
    """Roofline figures of the dominant kernel.  A pass may launch a kernel
    more than once (one launch per workspace chunk), so the algorithmic work of
    one launch is the pass's work divided by the launches per pass, and the
    achieved rate is that over the kernel's average launch duration (equal to
    the pass's work over the kernel's summed time per pass)."""
    cells = st["cells"]
    sim_ops_per_cell = st["mean_b"] + st["mean_ka"] + 20.0
    sim_ops = sim_ops_per_cell * cells
    nw_bytes = 4.25 * cells
    sim, nw = kern["similarity"], kern["nw"]
    sim_ops_launch = sim_ops / max(sim["launches_per_step"], 1e-9)
    nw_bytes_launch = nw_bytes / max(nw["launches_per_step"], 1e-9)
    sim.update(bound="alu", algorithmic_ops_per_launch=sim_ops_launch,
               achieved_TOPs=sim_ops_launch / (sim["avg_ms"] * 1e-3) / 1e12 if sim["avg_ms"] else None)
    nw.update(bound="hbm", algorithmic_bytes_per_launch=nw_bytes_launch,
              achieved_GBs=nw_bytes_launch / (nw["avg_ms"] * 1e-3) / 1e9 if nw["avg_ms"] else None,
              gcups=cells / (nw["ms_per_step"] * 1e-3) / 1e9 if nw["ms_per_step"] else None)
    if sim["ms_per_step"] >= nw["ms_per_step"]:
        ach = sim["achieved_TOPs"]
        return dict(kernel="similarity", bound="alu", achieved=ach, peak=ALU_PEAK_TOPS, unit="TOP/s",
                    frac=ach / ALU_PEAK_TOPS, traffic=profiled_traffic("sim_kernel", name),
                    per_unit=f"{sim_ops_per_cell:.2f} ops/cell (mean b + mean k*a + 20) x {cells} cells per pass, "
                             f"{sim['launches_per_step']:g} launches per pass")
    ach = nw["achieved_GBs"]
    return dict(kernel="nw", bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                traffic=profiled_traffic("nw_kernel", name),
                per_unit=f"4.25 B/cell x {cells} cells per pass, {nw['launches_per_step']:g} launches per pass")


def compare(got, want, pairs_got):
    """GPU result entries of `pairs_got` against the oracle's result of the same
    pairs (in that order): index pairs equal, scores within TOL_S, H[n][m] bit
    for bit.  Returns the number of pairs that differ."""
    bad = 0
    for k, p in enumerate(pairs_got):
        a, b = int(got["pair_off"][p]), int(got["pair_off"][p + 1])
        c, d = int(want["pair_off"][k]), int(want["pair_off"][k + 1])
        same = (np.array_equal(got["src_idx"][a:b], want["src_idx"][c:d])
                and np.array_equal(got["tgt_idx"][a:b], want["tgt_idx"][c:d])
                and np.max(np.abs(got["score"][a:b] - want["score"][c:d]), initial=0.0) <= TOL_S
                and np.float32(got["align_score"][p]).tobytes() == np.float32(want["align_score"][k]).tobytes())
        bad += not same
    return bad


def served(ymine, synth, ctx, seconds, rate, overload_rate, overload_seconds, log_every=5.0):
    """The served stream: Poisson arrivals of single document pairs (lognormal
    sentence counts, median 80, cap 4000) replayed in real time against the
    continuous-batching server (steps captured in hipGraphs) and against the
    plain per-pair GPU form, FIFO.  Then an overloaded stream at a multiple of
    the rate.  Latency = completion minus scheduled arrival."""
    cfg = synth.CONFIGS[3]
    n_req = int(seconds * rate)
    n_over = int(overload_seconds * overload_rate)
    lex = synth.make_lexicon(cfg)
    corp = synth.generate(cfg, lex, pair_ids=np.arange(n_req))
    w = synth.weights(cfg.seed)
    arr = synth.arrivals(cfg.seed, rate, n_req)
    arr_over = synth.arrivals(cfg.seed + 7, overload_rate, n_over)
    reqs = [ymine.prepare(corp.slice(k, k + 1)) for k in range(n_req)]
    n, m = corp.nm()
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    prm = ymine.params(w, -0.2, 0.5)
    ymine.mine_prepared(ctx, L, reqs[0], prm)  # warm the kernels
    # reference results of every 97th request from the batch entry point
    probe = np.arange(0, n_req, 97)
    ref = {int(k): ymine.mine_prepared(ctx, L, reqs[int(k)], prm) for k in probe}

    def same(a, b):
        return all(np.array_equal(a[x], b[x]) for x in ("pair_off", "src_idx", "tgt_idx", "score", "align_score"))

    def run_server(times, idx, label, use_graph=1, max_pairs=512):
        srv = ymine.Server(ctx, L, w, -0.2, 0.5, max_pairs_per_step=max_pairs, max_cells_per_step=1 << 26,
                           use_graph=use_graph)
        N = len(idx)
        done_ns = np.zeros(N, np.int64)
        ticket_of = {}
        lock = threading.Lock()
        t0 = time.monotonic_ns() + 200_000_000

        def submitter():
            for k in range(N):
                due = t0 + int(times[k] * 1e9)
                while True:
                    now = time.monotonic_ns()
                    if now >= due:
                        break
                    time.sleep(min((due - now) / 1e9, 0.0005))
                t = srv.submit_prepared(reqs[idx[k]])
                with lock:
                    ticket_of[t] = k

        th = threading.Thread(target=submitter)
        th.start()
        got, identical, last = 0, True, time.time()
        while got < N:
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
            if int(idx[k]) in ref:
                identical &= same(res, ref[int(idx[k])])
            got += 1
            if time.time() - last > log_every:
                log(f"[serve] {label}: {got}/{N} done")
                last = time.time()
        th.join()
        stats, gstats = srv.stats(), srv.graph_stats()
        srv.stop()
        lat = (done_ns - (t0 + (np.asarray(times) * 1e9).astype(np.int64))) / 1e6
        span = (done_ns.max() - t0) / 1e9
        r = dict(requests=N, p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                 mean_ms=float(lat.mean()), max_ms=float(lat.max()), throughput_pairs_per_s=N / span,
                 steps=stats["steps"], pairs_per_step=stats["completed"] / max(stats["steps"], 1),
                 cells=stats["cells"], identical_to_batch_on_probes=bool(identical))
        if use_graph:
            r.update(graph_instantiations=gstats["instantiations"], graph_updates=gstats["updates"])
        log(f"[serve] {label}: {r}")
        return r

    def run_plain(times, idx, label, limit_s):
        lat, identical = [], True
        t0 = time.monotonic_ns() + 100_000_000
        deadline = t0 + int(limit_s * 1e9)
        for k in range(len(idx)):
            due = t0 + int(times[k] * 1e9)
            now = time.monotonic_ns()
            if now < due:
                time.sleep((due - now) / 1e9)
            res = ymine.mine_prepared(ctx, L, reqs[idx[k]], prm, per_pair=True)
            fin = time.monotonic_ns()
            lat.append((fin - due) / 1e6)
            if int(idx[k]) in ref:
                identical &= same(res, ref[int(idx[k])])
            if fin > deadline:
                break
        lat = np.array(lat)
        r = dict(requests=len(idx), completed=int(lat.size), p50_ms=float(np.percentile(lat, 50)),
                 p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                 throughput_pairs_per_s=lat.size / ((time.monotonic_ns() - t0) / 1e9),
                 identical_to_batch_on_probes=bool(identical))
        log(f"[serve] {label}: {r}")
        return r

    out = {}
    idx_all = np.arange(n_req)
    out["server_graph"] = run_server(arr, idx_all, "server (hipGraph steps)")
    out["plain_per_pair"] = run_plain(arr, idx_all, "plain per-pair FIFO", seconds + 20)
    # overload: the same requests, arriving at overload_rate (first n_over of them)
    idx_over = np.arange(n_over) % n_req
    ov = dict(rate_per_s=overload_rate, seconds=overload_seconds)
    ov["server_graph"] = run_server(arr_over, idx_over, "overload: server (hipGraph steps)")
    ov["plain_per_pair"] = run_plain(arr_over, idx_over, "overload: plain per-pair FIFO", overload_seconds + 20)
    out["overload"] = ov
    out["workload"] = dict(name=cfg.name, requests=n_req, rate_per_s=rate, seconds=seconds,
                           cells=int((n * m).sum()), max_cells=int((n * m).max()), max_n=int(n.max()),
                           max_m=int(m.max()))
    L.close()
    return out


def batch_leg(torch, ymine, synth, ctx, k, steps, warmup, max_pairs=0, tune=True):
    """A batch workload timed the same way as the headline (secondary
    figures), with its own autotuned launch configuration (on the whole batch
    when it has at most 20,000 pairs, else on 20,000 spread over it)."""
    cfg = synth.CONFIGS[k]
    lex = synth.make_lexicon(cfg)
    ids = np.arange(min(cfg.n_pairs, max_pairs) if max_pairs else cfg.n_pairs)
    corpus = synth.generate(cfg, lex, pair_ids=ids)
    w = synth.weights(cfg.seed)
    st = workload_stats(corpus, lex)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    tuning = None
    if tune:
        sample = corpus if corpus.n_pairs <= 20000 else corpus.subset(
            np.linspace(0, corpus.n_pairs - 1, 20000).astype(np.int64))
        best, best_ms = ymine.autotune(ctx, L, sample, w, np.float32(-0.2), np.float32(0.5), reps=3)
        tuning = dict(best, sample_pairs=sample.n_pairs, sample_ms=best_ms)
    dm = ymine.DeviceMiner(ctx, L, corpus)
    sec, kern = timed_passes(torch, ctx, dm, w, np.float32(-0.2), np.float32(0.5), steps, warmup)
    roof = roofline(kern, st, cfg.name)
    r = dict(workload=cfg.name, n_pairs=corpus.n_pairs, cells=st["cells"], ms_per_step=sec * 1e3,
             pairs_per_s=corpus.n_pairs / sec, gcups=st["cells"] / sec / 1e9, kernels=kern, roofline=roof,
             tuning=tuning)
    log(f"[bench] {cfg.name}: {sec * 1e3:.3f} ms/step, {corpus.n_pairs / sec:.0f} pairs/s, "
        f"{st['cells'] / sec / 1e9:.1f} GCUPS; tuning {tuning}")
    del dm
    L.close()
    torch.cuda.empty_cache()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=4, help="workload index (default: the 1M-pair scale batch)")
    ap.add_argument("--max-pairs", type=int, default=0, help="only the first pairs of the workload (0: all)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample (0: skip)")
    ap.add_argument("--per-pair-sample", type=int, default=1000, help="pairs timed in the plain per-pair form")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the served arrival trace (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate of the served trace")
    ap.add_argument("--overload-rate", type=float, default=30000.0, help="arrival rate of the overloaded trace")
    ap.add_argument("--overload-seconds", type=float, default=4.0, help="length of the overloaded trace")
    ap.add_argument("--secondary", type=str, default="1,2", help="other batch workloads to time (comma list, '' none)")
    ap.add_argument("--tuning", type=str, default="",
                    help="fixed launch configuration 'sim_kernel,item_rows,nw_pairs_per_group,nw_large' "
                         "for every leg instead of the autotuner's choices (profiling runs)")
    ap.add_argument("--autotune-pairs", type=int, default=100000,
                    help="pairs of the autotuner's sample, spread over the batch (0: default configuration)")
    ap.add_argument("--workspace-gib", type=float, default=64.0, help="workspace cap of the device form (GiB)")
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
    corpus = synth.generate(cfg, lex, pair_ids=np.arange(n_gen))
    w = synth.weights(cfg.seed)
    gap, tau = np.float32(-0.2), np.float32(0.5)
    st = workload_stats(corpus, lex)
    log(f"[bench] {corpus.n_pairs} pairs, {st['cells']} cells, {st['src_tokens']} + {st['tgt_tokens']} tokens, "
        f"generated in {time.time() - t:.1f}s")

    ctx = ymine.Context(0)
    L = ctx.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
    # autotuner (untimed): launch configuration picked on pairs spread over the batch
    tuning = None
    fixed = [int(x) for x in args.tuning.split(",")] if args.tuning else None
    if fixed:
        ymine.set_tuning(ctx, *fixed)
        tuning = dict(ymine.get_tuning(ctx), fixed=True)
        log(f"[bench] tuning (fixed): {tuning}")
    elif args.autotune_pairs > 0:
        ids = np.linspace(0, corpus.n_pairs - 1, min(args.autotune_pairs, corpus.n_pairs)).astype(np.int64)
        sample = synth.generate(cfg, lex, pair_ids=ids)
        t = time.time()
        best, best_ms = ymine.autotune(ctx, L, sample, w, gap, tau, reps=3)
        tuning = dict(best, sample_pairs=sample.n_pairs, sample_ms=best_ms, seconds=round(time.time() - t, 2))
        log(f"[bench] autotune: {tuning}")
    t = time.time()
    dm = ymine.DeviceMiner(ctx, L, corpus, workspace_bytes=_workspace(ymine, corpus, args.workspace_gib))
    torch.cuda.synchronize()
    log(f"[bench] inputs resident in HBM ({time.time() - t:.1f}s), workspace {dm.ws_bytes / 2**30:.1f} GiB")

    sec, kern = timed_passes(torch, ctx, dm, w, gap, tau, args.steps, args.warmup)
    ms_per_step = sec * 1e3
    pairs_per_s = corpus.n_pairs / sec
    gcups = st["cells"] / sec / 1e9
    res = dm.result()
    n_mined = int(res["pair_off"][-1])
    log(f"[bench] {ms_per_step:.3f} ms/step, {pairs_per_s:.0f} pairs/s, {gcups:.1f} GCUPS, {n_mined} mined pairs; "
        f"kernels {json.dumps({k: round(v['avg_ms'], 4) for k, v in kern.items()})}")
    roof = roofline(kern, st, cfg.name)

    # plain per-pair GPU form vs the batched host entry point on the same pairs
    plain = None
    if args.per_pair_sample > 0:
        sub = corpus.slice(0, min(args.per_pair_sample, corpus.n_pairs))
        ymine.mine(ctx, L, sub, w, gap, tau)  # warm
        ta = time.perf_counter()
        rb = ymine.mine(ctx, L, sub, w, gap, tau)
        tb = time.perf_counter()
        rp = ymine.mine_per_pair(ctx, L, sub, w, gap, tau)
        tc = time.perf_counter()
        same = all(np.array_equal(rb[k], rp[k]) for k in rb)
        same_dev = compare(res, rb, np.arange(sub.n_pairs)) == 0
        plain = dict(pairs=sub.n_pairs, batched_pairs_per_s=sub.n_pairs / (tb - ta),
                     per_pair_pairs_per_s=sub.n_pairs / (tc - tb), speedup=(tc - tb) / (tb - ta), identical=same,
                     identical_to_device_form=bool(same_dev))
        log(f"[bench] plain per-pair: {plain}")

    # CPU oracle on a bounded sample: the last pairs of the batch (token
    # offsets beyond 2^31 at full size), also checked against the GPU's results
    cpu = cpu_mt = None
    if args.cpu_seconds > 0:
        import oracle
        O = oracle.default()
        OL = O.lexicon(lex.src_ids, lex.off, lex.tgt_ids)
        done, tc0 = 0, time.perf_counter()
        bad = 0
        last = corpus.n_pairs
        step = 8
        while time.perf_counter() - tc0 < args.cpu_seconds and done < corpus.n_pairs:
            p0 = max(0, last - done - step)
            sub = corpus.slice(p0, last - done)
            want = O.mine(OL, sub, w, gap, tau)
            bad += compare(res, want, np.arange(p0, last - done))
            done += sub.n_pairs
        el = time.perf_counter() - tc0
        p_first = last - done
        src_off = int(corpus.src_sent_off[corpus.src_doc_off[p_first]])
        tgt_off = int(corpus.tgt_sent_off[corpus.tgt_doc_off[p_first]])
        cpu = dict(value=done / el, unit="doc pairs/s", cores=1, kind="oracle",
                   sample=f"last {done} pairs of the {corpus.n_pairs}-pair batch (pairs {p_first}..{last - 1}), "
                          f"single thread, {el:.1f} s",
                   parity=dict(pairs=done, first_src_token_offset=src_off, first_tgt_token_offset=tgt_off,
                               beyond_2_31=bool(src_off >= 2**31 and tgt_off >= 2**31), pairs_differing=bad))
        log(f"[bench] cpu oracle: {cpu}")
        threads = min(16, len(os.sched_getaffinity(0)))
        nsub = min(corpus.n_pairs, max(threads * 8, int(cpu["value"] * threads * args.cpu_seconds * 0.5)))
        sub = corpus.slice(corpus.n_pairs - nsub, corpus.n_pairs)
        tc0 = time.perf_counter()
        want = O.mine_threads(OL, sub, w, gap, tau, threads)
        el = time.perf_counter() - tc0
        bad_mt = compare(res, want, np.arange(corpus.n_pairs - nsub, corpus.n_pairs))
        cpu_mt = dict(value=nsub / el, unit="doc pairs/s", cores=threads, kind="oracle_threads",
                      sample=f"last {nsub} pairs of the batch, {threads} threads, {el:.1f} s",
                      parity=dict(pairs=nsub, pairs_differing=bad_mt))
        log(f"[bench] cpu oracle, all cores: {cpu_mt}")
        del OL

    del dm
    L.close()
    del corpus
    torch.cuda.empty_cache()

    secondary = {}
    for k in [int(x) for x in args.secondary.split(",") if x.strip()]:
        if k != args.workload:
            secondary[synth.CONFIGS[k].name] = batch_leg(torch, ymine, synth, ctx, k, max(3, args.steps // 2),
                                                         args.warmup, tune=not fixed)
    if tuning is not None:  # the served legs run with the headline's configuration
        ymine.set_tuning(ctx, tuning["sim_kernel"], tuning["item_rows"], tuning["nw_pairs_per_group"],
                         tuning["nw_large"])

    serve = None
    if args.serve_seconds > 0:
        serve = served(ymine, synth, ctx, args.serve_seconds, args.serve_rate, args.overload_rate,
                       args.overload_seconds)

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
        "config": {"workload": cfg.name, "n_pairs": n_gen, "workload_pairs": cfg.n_pairs, "cells": st["cells"],
                   "src_tokens": st["src_tokens"], "tgt_tokens": st["tgt_tokens"], "gap": float(gap),
                   "threshold": float(tau), "parallelism": "single GPU", "tuning": tuning},
        "gcups": gcups,
        "mined_pairs": n_mined,
        "kernels": kern,
        "roofline": roof,
        "secondary": secondary,
        "plain_per_pair": plain,
        "served": serve,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_mt,
    }
    print(json.dumps(line), flush=True)


def _workspace(ymine, corpus, cap_gib):
    """Workspace of the device form: the whole batch as one chunk, capped."""
    import ctypes as C
    sdo = np.ascontiguousarray(corpus.src_doc_off, np.int64)
    tdo = np.ascontiguousarray(corpus.tgt_doc_off, np.int64)
    P = C.POINTER(C.c_int64)
    full = int(ymine.lib().ym_mine_device_workspace(sdo.ctypes.data_as(P), tdo.ctypes.data_as(P), corpus.n_pairs,
                                                   int(corpus.src_tok.shape[0])))
    least = int(ymine.lib().ym_mine_device_workspace_min(sdo.ctypes.data_as(P), tdo.ctypes.data_as(P),
                                                        corpus.n_pairs, int(corpus.src_tok.shape[0])))
    return max(least, min(full, int(cap_gib * 2**30)))


if __name__ == "__main__":
    main()
