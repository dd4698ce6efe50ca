"""Serving: continuous batching of pattern queries over HBM-resident texts.

Thin wrapper over the server in the C ABI (epsm_server_*): the scheduler,
admission and batching run natively in libepsm.so; this module marshals
queries and results, and drives Poisson query streams for measurements.
"""
from __future__ import annotations

import ctypes
import threading
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _check, _check_text, _lib, lib


@dataclass
class QueryOutcome:
    query_id: int
    text_id: int
    status: int
    counts: np.ndarray       # int64 [n_patterns]
    offsets: np.ndarray      # int64 [n_patterns]
    positions: np.ndarray    # int64 [total]
    submit_time: float
    start_time: float
    done_time: float
    batch_queries: int

    def pattern_positions(self, k: int) -> np.ndarray:
        o = int(self.offsets[k])
        return self.positions[o:o + int(self.counts[k])]


class Server:
    """epsm_server: resident texts + continuous batching over `slots` streams."""

    def __init__(self, slots: int = 4, max_batch_queries: int = 64, max_batch_entries: int = 0,
                 hbm_budget: int = 0, flags: int = 0):
        cfg = _lib.ServerConfig(slots, max_batch_queries, max_batch_entries, hbm_budget, flags)
        self._h = ctypes.c_void_p()
        _check(lib().epsm_server_create(ctypes.byref(cfg), ctypes.byref(self._h)), "epsm_server_create")
        self._texts = []
        self.text_lengths = []

    def add_text(self, text: torch.Tensor) -> int:
        _check_text(text)
        tid = ctypes.c_uint32()
        _check(lib().epsm_server_add_text(self._h, text.data_ptr() if text.numel() else None,
                                          text.numel(), ctypes.byref(tid)), "epsm_server_add_text")
        self._texts.append(text)  # the caller's tensor must stay alive: keep a reference
        self.text_lengths.append(text.numel())
        return tid.value

    def submit(self, text_id: int, patterns) -> int:
        pats = [bytes(p) for p in patterns]
        blob = b"".join(pats)
        lens = (ctypes.c_uint64 * max(len(pats), 1))(*[len(p) for p in pats])
        buf = ctypes.create_string_buffer(blob, max(len(blob), 1))
        qid = ctypes.c_uint64()
        _check(lib().epsm_server_submit(self._h, text_id, ctypes.cast(buf, ctypes.c_void_p),
                                        ctypes.cast(lens, ctypes.c_void_p), len(pats),
                                        ctypes.byref(qid)), "epsm_server_submit")
        return qid.value

    def poll(self, max_results: int = 64, wait_us: int = 1000) -> list[QueryOutcome]:
        res = (_lib.QueryResult * max_results)()
        n = ctypes.c_uint32()
        _check(lib().epsm_server_poll(self._h, res, max_results, ctypes.byref(n), wait_us),
               "epsm_server_poll")
        out = []
        for i in range(n.value):
            r = res[i]
            npat = r.n_patterns if r.status == 0 else 0  # failed queries carry no arrays
            counts = np.ctypeslib.as_array(r.counts, (npat,)).astype(np.int64) if npat else np.zeros(0, np.int64)
            offs = np.ctypeslib.as_array(r.offsets, (npat,)).astype(np.int64) if npat else np.zeros(0, np.int64)
            pos = (np.ctypeslib.as_array(r.positions, (r.total,)).copy() if r.total and r.status == 0
                   else np.zeros(0, np.int64))
            out.append(QueryOutcome(r.query_id, r.text_id, r.status, counts, offs, pos, r.submit_time,
                                    r.start_time, r.done_time, r.batch_queries))
            _check(lib().epsm_server_release(self._h, r.query_id), "epsm_server_release")
        return out

    def now(self) -> float:
        return lib().epsm_server_now(self._h)

    def stats(self) -> dict:
        st = _lib.ServerStats()
        _check(lib().epsm_server_get_stats(self._h, ctypes.byref(st)), "epsm_server_get_stats")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self) -> None:
        if self._h and self._h.value:
            lib().epsm_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_queries(server: Server, queries, rate_scale: float = 1.0, timeout_s: float = 600.0):
    """Submit queries at their arrival times (seconds, scaled by 1/rate_scale)
    from a client thread and collect every result.

    Latency of a query = time its results are in host memory - its scheduled
    arrival time (both on the server clock).  Returns (outcomes by query
    index, latencies, wall seconds).
    """
    n = len(queries)
    ids = [None] * n
    t0 = server.now() + 0.01
    arrivals = [t0 + q.arrival / rate_scale for q in queries]
    errors = []

    def client():
        try:
            for i, q in enumerate(queries):
                delay = arrivals[i] - server.now()
                if delay > 0:
                    time.sleep(delay)
                ids[i] = server.submit(q.text, q.patterns)
        except Exception as e:  # surfaced by the collector below
            errors.append(e)

    th = threading.Thread(target=client, daemon=True)
    th.start()
    by_id, done = {}, 0
    deadline = time.time() + timeout_s
    while done < n:
        if errors:
            raise errors[0]
        if time.time() > deadline:
            raise TimeoutError(f"{n - done} queries still pending after {timeout_s} s")
        for r in server.poll(64, 2000):
            by_id[r.query_id] = r
            done += 1
    th.join()
    outcomes = [by_id[ids[i]] for i in range(n)]
    lat = np.array([outcomes[i].done_time - arrivals[i] for i in range(n)])
    wall = max(o.done_time for o in outcomes) - t0
    return outcomes, lat, wall
