#!/usr/bin/env python3
"""Benchmark of the exact packed string matching scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints ONE JSON line.  Workloads (all synthetic, seeded, generated on the GPU
by the workloads module; texts are resident in HBM before timing starts):

  zipf4g   (default) 4 GiB Zipf(1) English-like text, cut patterns m = 1..16,
           positions and count modes; plus the periodic text a^n with a^m
           (dense output, 8 bytes written per byte read at m = 1).  One step =
           the 64 searches (256 GiB of logical text).  The default run then
           adds the batch and serving legs below as the "batch" and "serve"
           objects of the same line (--scan-only leaves them out).
  sweep1g  1 GiB texts uniform over sigma in {2,4,20,64,128} codes; per sigma
           and m in {1,2,4,8,12,16,24,32} one pattern cut from the text and
           one random; every pattern searched in positions mode and in count
           mode.  One step = the whole sweep (160 searches, 160 GiB of
           logical text).
  serve    256 resident texts (sigma 20, log-uniform lengths in [1, 256] MiB);
           Poisson query streams (text id + 1..256 patterns, m in [2, 32])
           served with continuous batching: saturation throughput from a
           burst, then p50/p99 latency and GB/s at 0.25, 0.5, 0.8 x that rate.
  batch    10,000 texts, log-uniform lengths in [1 KiB, 16 MiB], sigma 4 or
           64, 1..64 patterns each with m uniform in [1, 32] (half cut, half
           random).  One step = the whole batch as one replay of a prepared,
           graph-captured batch; compared with one epsm_search per pair on
           the same texts (identical output checked on the device).

value = logical text bytes scanned per second over the timed steps (GB/s,
1 GB = 1e9 B).  roofline = the positions-mode scan kernel: algorithmic bytes
(n read once + 8 bytes per reported position) / kernel time, timed with
events on the launch stream, against the 8 TB/s HBM peak; traffic and
traffic_frac: the calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE bytes per
launch from profiles/ (when taken on the same kernel sources) and their rate
over the same launch time.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "text GB/s scanned & fraction of HBM peak, batched vs plain; p99 query latency"
HBM_PEAK_GBS = 8000.0
# vector ALU int32 peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_INT32_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
ALU_OPS_PER_PAIR_BYTE = 2


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="zipf4g", choices=["sweep1g", "zipf4g", "batch", "serve", "dna", "long"])
    ap.add_argument("--scan-only", action="store_true",
                    help="zipf4g: leave out the batch and serving legs of the default run")
    ap.add_argument("--serve-queries", type=int, default=1000, help="queries per serving run")
    ap.add_argument("--batch-texts", type=int, default=10_000, help="texts in the batch workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU time budget of the oracle baseline (0 disables it)")
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0 = all host cores)")
    ap.add_argument("--detail", action="store_true", help="per-search timings on stderr")
    ap.add_argument("--tuning", default="auto",
                    help="'auto': the per-user or packaged autotune table of this device, if any; "
                         "'none': built-in tiles; else a cache path")
    ap.add_argument("--positions-only", action="store_true",
                    help="profiling aid: only the positions-mode searches, outputs sized to n "
                         "(no count pass), so every scan dispatch is a positions-mode one")
    ap.add_argument("--count-only", action="store_true",
                    help="profiling aid: only the count-mode searches of the workload")
    ap.add_argument("--no-plain", action="store_true",
                    help="profiling aid (batch): leave out the per-instance searches")
    return ap.parse_args()


class Case:
    def __init__(self, text_idx, plan, pattern, origin, mode):
        self.text_idx, self.plan, self.pattern, self.origin, self.mode = text_idx, plan, pattern, origin, mode
        self.count = 0


def build_sweep1g(torch, W, epsm):
    texts, specs, cases = [], [], []
    for sigma in W.CONFIG2_SIGMAS:
        spec, pcs = W.config2(sigma)
        log(f"generating sigma={sigma} text ({spec.n} B) on the GPU")
        texts.append(W.gen_bytes(spec, device="cuda"))
        specs.append(spec)
        for pc in pcs:
            plan = epsm.Plan(pc.pattern)
            for mode in ("positions", "count"):
                cases.append(Case(len(texts) - 1, plan, pc.pattern, pc.origin, mode))
    config = {"workload": "sweep1g: 1 GiB uniform texts, sigma {2,4,20,64,128}, m {1,2,4,8,12,16,24,32}, "
                          "cut+random patterns, positions+count modes",
              "text_bytes": 1 << 30, "sigmas": list(W.CONFIG2_SIGMAS), "ms": list(W.CONFIG2_MS),
              "searches_per_step": len(cases)}
    return texts, specs, cases, config


def build_zipf4g(torch, W, epsm):
    spec, pcs, per, per_cases = W.config3()
    log("generating 4 GiB Zipf text and 4 GiB periodic text on the GPU")
    texts = [W.gen_bytes(spec, device="cuda"), W.gen_bytes(per, device="cuda")]
    cases = []
    for ti, group in ((0, pcs), (1, per_cases)):
        for pc in group:
            plan = epsm.Plan(pc.pattern)
            for mode in ("positions", "count"):
                cases.append(Case(ti, plan, pc.pattern, pc.origin, mode))
    config = {"workload": "zipf4g: 4 GiB Zipf(1) 96-symbol English-like text, cut patterns m=1..16, plus "
                          "4 GiB a^n with a^m (m=1..16); positions+count modes",
              "text_bytes": 1 << 32, "ms": list(range(1, 17)), "searches_per_step": len(cases)}
    return texts, [spec, per], cases, config


def run_dna_workload(args, torch, W, epsm):
    """Genome-like text of 2^32 symbols (uniform over 4 codes) searched packed
    at 2 bits per symbol (1 GiB) and, for comparison, as bytes (4 GiB), with
    the same cut and random patterns of m in {8, 12, 16, 20, 24, 32}."""
    n = 1 << 32
    spec = W.TextSpec(n=n, kind="uniform", key=W.text_key(6, 0), sigma=4)
    log("generating 2^32 DNA codes on the GPU and packing them")
    codes = W.gen_bytes(spec, device="cuda")
    packed = epsm.pack_dna(codes)
    torch.cuda.synchronize()
    g = W.rng(6, 1)
    pats = []
    for m in (8, 12, 16, 20, 24, 32):
        pats.append((W.cut_pattern(spec, m, g)[0], "cut"))
        pats.append((W.random_pattern(m, W.alphabet_of(spec), g), "random"))
    cases = [(p, o, epsm.Plan(p, epsm.PLAN_DNA), epsm.Plan(p)) for p, o in pats]
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    counts = []
    for p, _, pd, pb in cases:
        epsm.count_dna_into(pd, packed, n, hits)
        c = int(hits.item())
        epsm.count_into(pb, codes, hits)
        if int(hits.item()) != c:
            raise AssertionError("packed and byte counts differ")
        counts.append(c)
    out = torch.empty(max(max(counts), 1), dtype=torch.int64, device="cuda")

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        return e0, e1

    def step(record):
        ev = []
        for (p, _, pd, pb), c in zip(cases, counts):
            ev.append(timed(lambda: epsm.search_dna_into(pd, packed, n, out[:c], hits)))
            ev.append(timed(lambda: epsm.count_dna_into(pd, packed, n, hits)))
        return ev

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    epsm.stream_check()
    # the byte path over the same codes, for comparison (not in the value)
    byte_ms = []
    for (p, _, pd, pb), c in zip(cases, counts):
        e = [timed(lambda: epsm.search_into(pb, codes, out[:c], hits)), timed(lambda: epsm.count_into(pb, codes, hits))]
        torch.cuda.synchronize()
        byte_ms.append([a.elapsed_time(b) for a, b in e])
    detail, pos_ms_total, pos_bytes = [], 0.0, 0
    for i, ((p, o, _, _), c) in enumerate(zip(cases, counts)):
        pm = sum(evs[s][2 * i][0].elapsed_time(evs[s][2 * i][1]) for s in range(args.steps)) / args.steps
        cm = sum(evs[s][2 * i + 1][0].elapsed_time(evs[s][2 * i + 1][1]) for s in range(args.steps)) / args.steps
        pos_ms_total += pm
        pos_bytes += n // 4 + 8 * c
        detail.append({"m": len(p), "origin": o, "hits": c, "positions_ms": round(pm, 4),
                       "count_ms": round(cm, 4), "byte_positions_ms": round(byte_ms[i][0], 4),
                       "byte_count_ms": round(byte_ms[i][1], 4),
                       "gsym_s_positions": round(n / pm / 1e6, 1), "gsym_s_count": round(n / cm / 1e6, 1),
                       "gsym_s_byte_count": round(n / byte_ms[i][1] / 1e6, 1)})
        if args.detail:
            log(f"dna m={len(p):2d} {o:6s} hits={c:9d} packed: positions {pm:7.3f} ms count {cm:7.3f} ms "
                f"({n / cm / 1e6:7.1f} Gsym/s) | bytes: positions {byte_ms[i][0]:7.3f} ms "
                f"count {byte_ms[i][1]:7.3f} ms")
    achieved = pos_bytes / (pos_ms_total / 1e3) / 1e9
    config = {"workload": "dna: 2^32 symbols uniform over 4 codes, packed 2 bits per symbol (1 GiB); "
                          "cut+random patterns m in {8,12,16,20,24,32}; positions+count modes",
              "symbols": n, "packed_bytes": n // 4, "searches_per_step": 2 * len(cases)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "packed-DNA positions-mode search (scan_kernel, with zero_u64 before it for a single-pass "
                          "write, or tile_offsets_kernel + expand_kernel after it for a two-phase write)",
                "launches": len(cases) * args.steps,
                "avg_launch_ms": round(pos_ms_total / len(cases), 4),
                "alg_bytes_per_launch": round(pos_bytes / len(cases))}
    return n * 2 * len(cases) * args.steps / elapsed, elapsed / args.steps, config, detail, roofline


def run_long_workload(args, torch, W, epsm):
    """Long patterns on a 4 GiB Zipf text: the strided filter (one 8-byte
    block per S bytes, S = 256..2048) against the per-block filter, with cut
    patterns of m in {263, 300, 519, 1031, 2055, 4096}; and, with S = 32, 64,
    128 (a variant-table row), m in {40, 72, 136}."""
    spec, _, _, _ = W.config3()
    n = spec.n
    log("generating the 4 GiB Zipf text on the GPU")
    text = W.gen_bytes(spec, device="cuda")
    torch.cuda.synchronize()
    g = W.rng(7, 1)
    cases = []
    for m in (263, 300, 519, 1031, 2055, 4096):
        p, _ = W.cut_pattern(spec, m, g)
        cases.append((p, epsm.Plan(p), epsm.Plan(p, epsm.PLAN_NO_STRIDE)))
    # shorter patterns with the strided filter asked for by a variant-table
    # row (S = 32, 64, 128): whether skipping inside cache lines saves bytes
    g = W.rng(7, 2)
    for m in (40, 72, 136):
        p, _ = W.cut_pattern(spec, m, g)
        epsm.set_variant_table([(39, 262, 0, 256, epsm.VARIANT_STRIDE, 0)])
        ps = epsm.Plan(p)
        epsm.set_variant_table([])
        cases.append((p, ps, epsm.Plan(p, epsm.PLAN_NO_STRIDE)))
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    counts = []
    for p, ps, pb in cases:
        epsm.count_into(ps, text, hits)
        c = int(hits.item())
        epsm.count_into(pb, text, hits)
        if int(hits.item()) != c:
            raise AssertionError("strided and per-block counts differ")
        counts.append(c)
    out = torch.empty(max(max(counts), 1), dtype=torch.int64, device="cuda")

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        return e0, e1

    def step():
        return [(timed(lambda: epsm.search_into(ps, text, out[:c], hits)),
                 timed(lambda: epsm.count_into(ps, text, hits))) for (p, ps, pb), c in zip(cases, counts)]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    epsm.stream_check()
    detail, pos_ms_total = [], 0.0
    for i, ((p, ps, pb), c) in enumerate(zip(cases, counts)):
        pm = sum(evs[s][i][0][0].elapsed_time(evs[s][i][0][1]) for s in range(args.steps)) / args.steps
        cm = sum(evs[s][i][1][0].elapsed_time(evs[s][i][1][1]) for s in range(args.steps)) / args.steps
        e = timed(lambda: epsm.count_into(pb, text, hits))
        torch.cuda.synchronize()
        bm = e[0].elapsed_time(e[1])
        pos_ms_total += pm
        stride = ps.info()["stride"]
        detail.append({"m": len(p), "stride": stride, "hits": c, "positions_ms": round(pm, 4),
                       "count_ms": round(cm, 4), "per_block_count_ms": round(bm, 4),
                       "text_gbs_count": round(n / cm / 1e6, 1), "per_block_text_gbs": round(n / bm / 1e6, 1)})
        if args.detail:
            log(f"long m={len(p):4d} S={stride:4d} hits={c:3d} strided: positions {pm:7.3f} ms count {cm:7.3f} ms "
                f"({n / cm / 1e6:8.1f} GB/s of text) | per-block count {bm:7.3f} ms ({n / bm / 1e6:7.1f} GB/s)")
    config = {"workload": "long: 4 GiB Zipf(1) 96-symbol text, cut patterns m in {263,300,519,1031,2055,4096} "
                          "and, with S = 32/64/128 from a variant-table row, m in {40,72,136}; strided filter; "
                          "positions+count modes",
              "text_bytes": n, "searches_per_step": 2 * len(cases)}
    return n * 2 * len(cases) * args.steps / elapsed, elapsed / args.steps, config, detail, pos_ms_total


def run_batch_workload(args, torch, W, epsm):
    """Config-4 batch: batched graph replay vs per-instance plain searches."""
    import ctypes
    bts = W.config4(n_texts=args.batch_texts)
    log(f"generating {len(bts)} batch texts on the GPU")
    texts = [W.gen_bytes(bt.spec, device="cuda") for bt in bts]
    torch.cuda.synchronize()
    text_bytes = sum(t.numel() for t in texts)
    pairs_host = [(i, epsm.Plan(p, epsm.PLAN_HOST_ONLY)) for i, bt in enumerate(bts) for p in bt.patterns]
    logical = sum(texts[i].numel() for i, _ in pairs_host)
    log(f"{len(pairs_host)} pairs, {text_bytes / 2**30:.2f} GiB of text, {logical / 2**30:.1f} GiB logical")

    # size with a count-only batch, then prepare the full batch (untimed)
    b0 = epsm.Batch(texts, pairs_host, count_only=True)
    b0.run()
    total = int(b0.total.item())
    counts = b0.counts[:len(pairs_host)].clone()
    log(f"{total} positions in total")
    out_b = torch.empty(max(total, 1), dtype=torch.int64, device="cuda")
    batch = epsm.Batch(texts, pairs_host, out=out_b[:total] if total else None)
    bp = epsm.BatchPlan(batch)
    info = bp.info()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        bp.launch(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        bp.launch(stream)
    e1.record()
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / args.steps
    batched_gpu_ms = e0.elapsed_time(e1) / args.steps
    epsm.stream_check()
    if not torch.equal(batch.counts[:len(pairs_host)], counts):
        raise AssertionError("batched counts differ from the count-only batch")

    # one-shot form (descriptors built and uploaded inside the call)
    t0 = time.perf_counter()
    batch.run()
    torch.cuda.synchronize()
    oneshot_s = time.perf_counter() - t0
    if args.no_plain:
        print(json.dumps({"batch_no_plain": True, "batched_gpu_ms": round(batched_gpu_ms, 3),
                          "oneshot_ms": round(oneshot_s * 1e3, 3),
                          "units": info["units"], "entries": info["entries"]}), flush=True)
        sys.exit(0)

    # per-instance plain searches: one epsm_search per pair into its slice
    log("creating device plans for the per-instance baseline")
    dev_plans = {}
    for _, p in pairs_host:
        if id(p) not in dev_plans:
            dev_plans[id(p)] = epsm.Plan(p.pattern)
    out_p = torch.full((max(total, 1),), -1, dtype=torch.int64, device="cuda")
    hits = torch.zeros(len(pairs_host), dtype=torch.int64, device="cuda")
    offs = batch.offsets[:len(pairs_host)].cpu().tolist()
    cnts = counts.cpu().tolist()
    L = epsm.lib()
    sh = stream.cuda_stream or None
    base_out, base_hits = out_p.data_ptr(), hits.data_ptr()
    calls = [(dev_plans[id(p)].handle, texts[i].data_ptr() if texts[i].numel() else None, texts[i].numel(),
              base_out + 8 * offs[k] if cnts[k] else None, cnts[k], base_hits + 8 * k)
             for k, (i, p) in enumerate(pairs_host)]
    fn = L.epsm_search
    torch.cuda.synchronize()
    log(f"timing {len(calls)} per-instance searches")
    t0 = time.perf_counter()
    for c in calls:
        st = fn(c[0], c[1], c[2], c[3], c[4], c[5], sh)
        if st:
            raise epsm.EpsmError(st, "epsm_search")
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    epsm.stream_check()
    identical = bool(torch.equal(out_p[:total], out_b[:total])) and bool(torch.equal(hits, counts))
    if not identical:
        raise AssertionError("batched output differs from the per-instance searches")
    config = {"workload": f"batch: {len(bts)} texts log-uniform [1 KiB, 16 MiB], sigma 4|64, "
                          "1-64 patterns per text, m uniform [1,32], half cut / half random",
              "texts": len(bts), "pairs": len(pairs_host), "text_bytes": text_bytes,
              "logical_bytes": logical, "positions": total, "batch_units": info["units"],
              "batch_entries": info["entries"], "batch_tile_bytes": info["tile_bytes"]}
    # roofline of the replay: ALU-bound (each text byte is compared with
    # every pattern of its text).  Algorithmic work: ALU_OPS_PER_PAIR_BYTE
    # int32 operations per (pattern, text position) pair (cut the window,
    # compare it; the ballot is free), against the vector ALUs' int32 peak.
    # The HBM bytes the replay must move (text read by the count and write
    # passes, 8 bytes per position written) are reported beside it.
    alg_ops = ALU_OPS_PER_PAIR_BYTE * logical
    achieved = alg_ops / (batched_gpu_ms / 1e3) / 1e12
    hbm_bytes = 2 * text_bytes + 8 * total
    traffic = load_traffic("batch")
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": VALU_INT32_PEAK_TOPS,
                "unit": "Top/s", "frac": round(achieved / VALU_INT32_PEAK_TOPS, 4),
                "traffic": traffic["bytes_per_launch"] if traffic else None,
                "kernel": "batch replay (count pass, scan of the (pair, tile) counts, pair counts and offsets, write pass), "
                          "event-timed per replay",
                "alg_ops_per_launch": alg_ops, "avg_launch_ms": round(batched_gpu_ms, 4),
                "hbm": {"bytes_per_launch": hbm_bytes,
                        "gbs": round(hbm_bytes / (batched_gpu_ms / 1e3) / 1e9, 1),
                        "frac": round(hbm_bytes / (batched_gpu_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic_frac": (round(traffic["bytes_per_launch"] / (batched_gpu_ms / 1e3) / 1e9
                                               / HBM_PEAK_GBS, 4) if traffic else None)}}
    extra = {"batched_ms": round(batched_s * 1e3, 3), "batched_gpu_ms": round(batched_gpu_ms, 3),
             "oneshot_ms": round(oneshot_s * 1e3, 3), "plain_ms": round(plain_s * 1e3, 3),
             "speedup_vs_plain": round(plain_s / batched_s, 2),
             "plain_gbs": round(logical / plain_s / 1e9, 1), "identical_output": identical,
             "roofline": roofline}
    return logical, batched_s, config, extra


def run_serve_workload(args, torch, W, epsm):
    """Config-5 serving: saturation from a burst, then Poisson streams."""
    import numpy as np

    from paper_1209_6449_amd import serve
    specs = W.config5_texts()
    log(f"generating {len(specs)} resident texts ({sum(s.n for s in specs) / 2**30:.1f} GiB) on the GPU")
    texts = [W.gen_bytes(sp, device="cuda") for sp in specs]
    torch.cuda.synchronize()
    n_q = args.serve_queries
    srv = serve.Server(slots=4, max_batch_queries=32)
    for t in texts:
        srv.add_text(t)

    def logical(qs):
        return sum(len(q.patterns) * specs[q.text].n for q in qs)

    def split(outs, lat):
        # latency = queueing (arrival -> its micro-batch formed) + service
        # (micro-batch formed -> results in host memory)
        service = np.array([o.done_time - o.start_time for o in outs])
        wait = lat - service
        big = np.argsort(service)[-max(1, len(outs) // 100):]  # the slowest 1% of services
        return {"p99_wait_ms": round(float(np.percentile(wait, 99)) * 1e3, 2),
                "p99_service_ms": round(float(np.percentile(service, 99)) * 1e3, 2),
                "slowest_1pct_logical_gb": round(float(np.mean(
                    [len(qs_cur[i].patterns) * specs[qs_cur[i].text].n for i in big])) / 1e9, 1)}

    base = W.config5_queries(specs, n_q, qps=1.0)
    burst = [W.Query(0.0, q.text, q.patterns) for q in base]
    log(f"saturation run: burst of {n_q} queries")
    qs_cur = burst
    outs, lat, wall = serve.run_queries(srv, burst)
    sat_qps = n_q / wall
    points = [{"load": "burst", "qps": round(sat_qps, 1), "wall_s": round(wall, 3),
               "gbs": round(logical(burst) / wall / 1e9, 1),
               # the batch kernel's ALU roofline over the whole burst, host
               # staging and copies included (wall clock, not kernel time)
               "alu_frac": round(ALU_OPS_PER_PAIR_BYTE * logical(burst) / wall / 1e12 / VALU_INT32_PEAK_TOPS, 4),
               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
               "mean_batch_queries": round(float(np.mean([o.batch_queries for o in outs])), 2)}]
    for frac in (0.25, 0.5, 0.8):
        qps = frac * sat_qps
        qs = W.config5_queries(specs, n_q, qps=qps, seed_stream=10 + int(frac * 100))
        log(f"Poisson stream at {qps:.1f} QPS ({frac} x saturation)")
        qs_cur = qs
        outs, lat, wall = serve.run_queries(srv, qs)
        if any(o.status for o in outs):
            raise AssertionError("a served query failed")
        points.append(dict({"load": frac, "qps": round(qps, 1), "wall_s": round(wall, 3),
                            "gbs": round(logical(qs) / wall / 1e9, 1),
                            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                            "mean_batch_queries": round(float(np.mean([o.batch_queries for o in outs])), 2)},
                           **split(outs, lat)))
    stats = srv.stats()
    srv.close()
    config = {"workload": f"serve: {len(specs)} resident texts sigma 20 log-uniform [1 MiB, 256 MiB], "
                          f"{n_q} Poisson queries per load point, 1-256 patterns per query, m uniform [2,32], "
                          "half cut / half random; 4 stream slots, up to 32 queries per micro-batch",
              "texts": len(specs), "text_bytes": sum(s.n for s in specs), "queries": n_q}
    return points, stats, config


def cpu_baseline(torch, texts, cases, seconds: float, threads: int):
    """The oracle, as it stands, on a bounded sample of the same workload:
    half of the budget on the count-mode searches (oracle_count_mt), half on
    the positions-mode ones (oracle_range_mt over 64M-start ranges, every
    position materialised on the host), in the workload's order; each
    completed search's count must equal the GPU's."""
    import oracle
    if threads <= 0:
        threads = min(16, os.cpu_count() or 1)
    host_cache = {}

    def host(ti):
        if ti not in host_cache:
            host_cache.clear()
            host_cache[ti] = texts[ti].cpu().numpy()
        return host_cache[ti]

    modes = {}
    for mode in ("count", "positions"):
        done_bytes, elapsed, used, positions = 0, 0.0, [], 0
        for c in cases:
            if c.mode != mode:
                continue
            t = host(c.text_idx)
            m = len(c.pattern)
            got = 0
            t0 = time.perf_counter()
            if mode == "count":
                got = oracle.count_mt(t, c.pattern, threads)
            else:
                chunk = 1 << 26
                for lo in range(0, t.size - m + 1, chunk):
                    got += oracle.search_range_mt(t, c.pattern, lo, lo + chunk, threads).size
            dt = time.perf_counter() - t0
            if got != c.count:
                raise AssertionError(f"oracle {mode} count {got} != GPU count {c.count} for m={m}")
            done_bytes += t.size
            elapsed += dt
            positions += got
            used.append(m)
            if elapsed >= seconds / 2:
                break
        modes[mode] = {"gbs": round(done_bytes / elapsed / 1e9, 3), "searches": len(used), "ms": used,
                       "text_gib": round(done_bytes / 2**30, 2), "seconds": round(elapsed, 2),
                       "positions": positions}
    # one thread on the first count-mode search, for the per-core rate
    first = next(c for c in cases if c.mode == "count")
    t = host(first.text_idx)
    t0 = time.perf_counter()
    got = oracle.count_mt(t, first.pattern, 1)
    one_s = time.perf_counter() - t0
    if got != first.count:
        raise AssertionError(f"oracle count {got} != GPU count {first.count} (one thread)")
    host_cache.clear()
    total_bytes = sum(v["text_gib"] for v in modes.values()) * 2**30
    total_s = sum(v["seconds"] for v in modes.values())
    return {
        "value": round(total_bytes / total_s / 1e9, 3),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"the oracle ({threads} threads over contiguous start ranges) on the workload's first "
                   f"{modes['count']['searches']} count-mode searches (m = {modes['count']['ms']}, "
                   f"{modes['count']['text_gib']} GiB, {modes['count']['gbs']} GB/s) and first "
                   f"{modes['positions']['searches']} positions-mode searches (m = {modes['positions']['ms']}, "
                   f"{modes['positions']['text_gib']} GiB, {modes['positions']['positions']} positions "
                   f"materialised, {modes['positions']['gbs']} GB/s); counts equal the GPU's"),
        "count_mode": modes["count"],
        "positions_mode": modes["positions"],
        "single_thread_value": round(t.size / one_s / 1e9, 3),
        "single_thread_sample": f"the first count-mode search (m = {len(first.pattern)}), "
                                f"{t.size / 2**30:.2f} GiB in {one_s:.2f} s",
        "cpu_model": cpu_model(),
    }


def cpu_model() -> str:
    """The host CPU's model name with its family, model and stepping numbers
    (a virtual machine may report only a generic name), from lscpu, else
    /proc/cpuinfo."""
    import subprocess
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        f = {}
        for line in r.stdout.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f.setdefault(k.strip(), v.strip())
        if "Model name" in f:
            ids = ", ".join(f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping") if k in f)
            return f"{f['Model name']} ({ids})" if ids else f["Model name"]
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def load_traffic(workload: str):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    from paper_1209_6449_amd.rocprof_summary import kernel_hash
    if d.get("kernel_hash") != kernel_hash():
        return None  # counters were taken on a different kernel
    return d


def apply_tuning(choice: str, epsm) -> str:
    from paper_1209_6449_amd import autotune
    if choice == "none":
        return "built-in tiles"
    if choice == "auto":
        path = autotune.apply_default(log)
        return os.path.relpath(path, ROOT) if path else "built-in tiles"
    autotune.apply(autotune.load(choice))
    return choice


def main():
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is design-only "
                                   "(see DESIGN.md); run with --gpus 1"}))
        sys.exit(2)

    import torch

    import paper_1209_6449_amd as epsm
    import workloads as W

    torch.cuda.set_device(0)
    tuning = apply_tuning(args.tuning, epsm)
    # A collection pause while searches are queued can drain the queue and
    # leave the GPU idle between the two events of one search; reference
    # counting still frees everything the steps create.
    gc.collect()
    gc.disable()
    if args.workload == "serve":
        points, stats, config = run_serve_workload(args, torch, W, epsm)
        top = points[-1]  # 0.8 x saturation
        result = {
            "metric": METRIC, "value": top["gbs"], "unit": "GB/s", "n_gpus": 1, "steps": 1,
            "warmup": 0, "ms_per_step": round(top["wall_s"] * 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": dict(config, tuning=tuning), "serve": {"points": points, "p50_ms": top["p50_ms"],
                                        "p99_ms": top["p99_ms"], "server_stats": stats},
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(result), flush=True)
        return
    if args.workload == "dna":
        sym_s, step_s, config, detail, roofline = run_dna_workload(args, torch, W, epsm)
        result = {
            "metric": "packed DNA symbols scanned per second", "value": round(sym_s / 1e9, 2),
            "unit": "Gsym/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(step_s * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u2", "data": "synthetic", "config": dict(config, tuning=tuning),
            "dna": detail, "roofline": roofline, "cpu_baseline": None,
        }
        print(json.dumps(result), flush=True)
        return
    if args.workload == "long":
        tb_s, step_s, config, detail, _ = run_long_workload(args, torch, W, epsm)
        result = {
            "metric": METRIC, "value": round(tb_s / 1e9, 1), "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic", "config": dict(config, tuning=tuning), "long": detail,
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(result), flush=True)
        return
    if args.workload == "batch":
        logical, step_s, config, extra = run_batch_workload(args, torch, W, epsm)
        result = {
            "metric": METRIC, "value": round(logical / step_s / 1e9, 1), "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(step_s * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u8", "data": "synthetic", "config": dict(config, tuning=tuning),
            "batch": extra, "roofline": extra["roofline"], "cpu_baseline": None,
        }
        print(json.dumps(result), flush=True)
        return
    build = build_sweep1g if args.workload == "sweep1g" else build_zipf4g
    texts, specs, cases, config = build(torch, W, epsm)
    torch.cuda.synchronize()

    # size outputs with a count pass (untimed)
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    max_hits = 1
    if args.count_only:
        cases = [c for c in cases if c.mode == "count"]
    if args.positions_only:
        # counts from one count-only batch (its own kernel), so that every
        # scan dispatch of the process is a timed positions-mode one
        cases = [c for c in cases if c.mode == "positions"]
        b = epsm.Batch(texts, [(c.text_idx, c.plan) for c in cases], count_only=True)
        b.run()
        counts = b.counts[:len(cases)].cpu().tolist()
        for c, k in zip(cases, counts):
            c.count = int(k)
            max_hits = max(max_hits, c.count)
    else:
        for c in cases:
            epsm.count_into(c.plan, texts[c.text_idx], hits)
            c.count = int(hits.item())
            max_hits = max(max_hits, c.count)
    log(f"{len(cases)} searches, largest output {max_hits} positions")
    out = torch.empty(max_hits, dtype=torch.int64, device="cuda")
    step_bytes = sum(texts[c.text_idx].numel() for c in cases)
    step_alg_bytes = sum(texts[c.text_idx].numel() + (8 * c.count if c.mode == "positions" else 0)
                         for c in cases)
    pos_alg_bytes = sum(texts[c.text_idx].numel() + 8 * c.count for c in cases if c.mode == "positions")
    for c in cases:
        c.events = []

    def step(record: bool):
        for c in cases:
            t = texts[c.text_idx]
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
            if c.mode == "positions":
                epsm.search_into(c.plan, t, out[:c.count], hits)
            else:
                epsm.count_into(c.plan, t, hits)
            if record:
                e1.record()
                c.events.append((e0, e1))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    epsm.stream_check()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    epsm.stream_check()
    elapsed = t1 - t0

    # the last search of the step wrote its count: spot-check it
    if int(hits.item()) != cases[-1].count:
        raise AssertionError("count mismatch after timing")
    if args.positions_only or args.count_only:
        print(json.dumps({"positions_only" if args.positions_only else "count_only": True,
                          "dispatches_per_step": len(cases), "text_bytes_per_step": step_bytes,
                          "ms_per_step": round(elapsed * 1e3 / args.steps, 3)}), flush=True)
        return

    for c in cases:
        c.ms = sum(e0.elapsed_time(e1) for e0, e1 in c.events) / len(c.events)
        if args.detail:
            n = texts[c.text_idx].numel()
            log(f"{c.mode:9s} text{c.text_idx} m={len(c.pattern):2d} {c.origin:11s} hits={c.count:11d} "
                f"{c.ms:8.3f} ms text {n / c.ms / 1e6:7.1f} GB/s "
                f"alg {(n + (8 * c.count if c.mode == 'positions' else 0)) / c.ms / 1e6:7.1f} GB/s")
    pos_cases = [c for c in cases if c.mode == "positions"]
    pos_ms = sum(c.ms for c in pos_cases) * args.steps
    n_pos_launches = len(pos_cases) * args.steps
    achieved = pos_alg_bytes * args.steps / (pos_ms / 1e3) / 1e9
    traffic = load_traffic(args.workload)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "kernel": "positions-mode search (scan_kernel, with zero_u64 before it for a single-pass "
                  "write, or tile_offsets_kernel + expand_kernel after it for a two-phase write), "
                  "event-timed per search",
        "launches": n_pos_launches,
        "avg_launch_ms": round(pos_ms / n_pos_launches, 4),
        "alg_bytes_per_launch": round(pos_alg_bytes / len(pos_cases)),
    }
    if traffic:
        # measured fraction: the calibrated HBM bytes per launch over the
        # same average launch time
        roofline["traffic_frac"] = round(traffic["bytes_per_launch"] / (pos_ms / n_pos_launches / 1e3)
                                         / 1e9 / HBM_PEAK_GBS, 4)

    result = {
        "metric": METRIC,
        "value": round(step_bytes * args.steps / elapsed / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": dict(config, tuning=tuning),
        "alg_gbs": round(step_alg_bytes * args.steps / elapsed / 1e9, 1),
        "roofline": roofline,
        "scan": scan_summary(cases, texts, specs),
    }
    if args.cpu_seconds > 0:
        log("timing the CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(torch, texts, cases, args.cpu_seconds, args.threads)
    else:
        result["cpu_baseline"] = None
    if args.workload == "zipf4g" and not args.scan_only:
        del texts, out, cases
        gc.collect()
        torch.cuda.empty_cache()
        epsm.release()
        logical, step_s, bconfig, extra = run_batch_workload(args, torch, W, epsm)
        result["batch"] = dict(extra, gbs=round(logical / step_s / 1e9, 1), config=bconfig)
        gc.collect()
        torch.cuda.empty_cache()
        epsm.release()
        points, stats, sconfig = run_serve_workload(args, torch, W, epsm)
        top = points[-1]
        result["serve"] = {"points": points, "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
                           "gbs": top["gbs"], "server_stats": stats, "config": sconfig}
    print(json.dumps(result), flush=True)


def scan_summary(cases, texts, specs) -> dict:
    """Per-search rates of the timed step, by text and mode (text GB/s, and
    algorithmic GB/s = (n + 8 per written position) / time), with the count-
    and positions-mode ranges of each text."""
    out = {}
    for ti, spec in enumerate(specs):
        n = texts[ti].numel()
        name = f"{spec.kind}" + (f"_sigma{spec.sigma}" if spec.kind == "uniform" else "")
        rows = []
        for c in cases:
            if c.text_idx != ti:
                continue
            alg = n + (8 * c.count if c.mode == "positions" else 0)
            rows.append({"m": len(c.pattern), "mode": c.mode, "origin": c.origin, "hits": c.count,
                         "ms": round(c.ms, 4), "text_gbs": round(n / c.ms / 1e6, 1),
                         "alg_gbs": round(alg / c.ms / 1e6, 1)})
        summary = {"text_bytes": n, "searches": rows}
        for mode in ("count", "positions"):
            r = [x for x in rows if x["mode"] == mode]
            if r:
                summary[f"{mode}_alg_gbs_min"] = min(x["alg_gbs"] for x in r)
                summary[f"{mode}_alg_gbs_max"] = max(x["alg_gbs"] for x in r)
                summary[f"{mode}_frac_min"] = round(summary[f"{mode}_alg_gbs_min"] / HBM_PEAK_GBS, 3)
        out[name] = summary
    return out


if __name__ == "__main__":
    main()
