#!/usr/bin/env python3
"""Benchmark of the exact packed string matching scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints ONE JSON line.  Workloads (all synthetic, seeded, generated on the GPU
by the workloads module; texts are resident in HBM before timing starts):

  sweep1g  (default) 1 GiB texts uniform over sigma in {2,4,20,64,128} codes;
           per sigma and m in {1,2,4,8,12,16,24,32} one pattern cut from the
           text and one random; every pattern searched in positions mode and
           in count mode.  One step = the whole sweep (160 searches, 160 GiB
           of logical text).
  zipf4g   4 GiB Zipf(1) English-like text, cut patterns m = 1..16, positions
           and count modes; plus the periodic text a^n with a^m (dense
           output, 8 bytes written per byte read at m = 1).

value = logical text bytes scanned per second over the timed steps (GB/s,
1 GB = 1e9 B).  roofline = the positions-mode scan kernel: algorithmic bytes
(n read once + 8 bytes per reported position) / kernel time, timed with
events on the launch stream, against the 8 TB/s HBM peak.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "text GB/s scanned & fraction of HBM peak, batched vs plain; p99 query latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1209_6449_amd/csrc/epsm_kernels.hip", "paper_1209_6449_amd/csrc/epsm_internal.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sweep1g", choices=["sweep1g", "zipf4g"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU time budget of the oracle baseline (0 disables it)")
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0 = all host cores)")
    ap.add_argument("--detail", action="store_true", help="per-search timings on stderr")
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


def cpu_baseline(torch, texts, cases, seconds: float, threads: int):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    if threads <= 0:
        threads = os.cpu_count() or 1
    done_bytes, elapsed, used = 0, 0.0, []
    host_cache = {}
    for c in cases:
        if c.mode != "count":
            continue
        if c.text_idx not in host_cache:
            host_cache.clear()
            host_cache[c.text_idx] = texts[c.text_idx].cpu().numpy()
        t = host_cache[c.text_idx]
        t0 = time.perf_counter()
        got = oracle.count_mt(t, c.pattern, threads)
        dt = time.perf_counter() - t0
        if got != c.count:
            raise AssertionError(f"oracle count {got} != GPU count {c.count} for m={len(c.pattern)}")
        done_bytes += t.size
        elapsed += dt
        used.append(len(c.pattern))
        if elapsed >= seconds:
            break
    host_cache.clear()
    return {
        "value": round(done_bytes / elapsed / 1e9, 3),
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"count mode (oracle_count_mt, {threads} threads) over the first {len(used)} "
                  f"count-mode searches of the workload (m = {used}), {done_bytes / 2**30:.1f} GiB "
                  f"of text in {elapsed:.1f} s; counts equal the GPU's",
    }


def load_traffic(workload: str):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash():
        return None  # counters were taken on a different kernel
    return d


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
    build = build_sweep1g if args.workload == "sweep1g" else build_zipf4g
    texts, specs, cases, config = build(torch, W, epsm)
    torch.cuda.synchronize()

    # size outputs with a count pass (untimed)
    hits = torch.zeros(1, dtype=torch.int64, device="cuda")
    max_hits = 1
    for c in cases:
        epsm.count_into(c.plan, texts[c.text_idx], hits)
        c.count = int(hits.item())
        max_hits = max(max_hits, c.count)
    log(f"{len(cases)} searches, largest output {max_hits} positions")
    out = torch.empty(max_hits, dtype=torch.int64, device="cuda")
    step_bytes = sum(texts[c.text_idx].numel() for c in cases)
    pos_alg_bytes = sum(texts[c.text_idx].numel() + 8 * c.count for c in cases if c.mode == "positions")

    events = []

    def step(record: bool):
        for c in cases:
            t = texts[c.text_idx]
            if c.mode == "positions":
                if record:
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                epsm.search_into(c.plan, t, out[:c.count], hits)
                if record:
                    e1.record()
                    events.append((e0, e1))
            else:
                epsm.count_into(c.plan, t, hits)

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

    # spot-check the last positions search against its count
    if int(hits.item()) != cases[-1].count:
        raise AssertionError("count mismatch after timing")

    pos_ms = sum(e0.elapsed_time(e1) for e0, e1 in events)
    if args.detail:
        pos_cases = [c for c in cases if c.mode == "positions"]
        for i, c in enumerate(pos_cases):
            ms = sum(events[s * len(pos_cases) + i][0].elapsed_time(events[s * len(pos_cases) + i][1])
                     for s in range(args.steps)) / args.steps
            n = texts[c.text_idx].numel()
            log(f"text{c.text_idx} m={len(c.pattern):2d} {c.origin:11s} hits={c.count:11d} {ms:8.3f} ms "
                f"text {n / ms / 1e6:7.1f} GB/s alg {(n + 8 * c.count) / ms / 1e6:7.1f} GB/s")
    n_pos_launches = len(events)
    achieved = pos_alg_bytes * args.steps / (pos_ms / 1e3) / 1e9
    traffic = load_traffic(args.workload)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "kernel": "scan_kernel, positions mode (all its template instances)",
        "launches": n_pos_launches,
        "avg_launch_ms": round(pos_ms / n_pos_launches, 4),
        "alg_bytes_per_launch": round(pos_alg_bytes / (n_pos_launches / args.steps)),
    }

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
        "config": config,
        "roofline": roofline,
    }
    if args.cpu_seconds > 0:
        log("timing the CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(torch, texts, cases, args.cpu_seconds, args.threads)
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
