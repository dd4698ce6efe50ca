"""Exact packed string matching on MI355X (gfx950).

Python binding of the C ABI in include/epsm.h.  Every step of the search runs
in the HIP kernels of libepsm.so; this module only marshals arguments.  torch
supplies device memory (uint8 / int64 / uint64 tensors) and streams.

    import paper_1209_6449_amd as epsm
    text = torch.frombuffer(bytearray(b"..."), dtype=torch.uint8).cuda()
    pos = epsm.search(text, b"pattern")        # int64 tensor of start positions
    n = epsm.count(text, b"pattern")
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (BATCH_COUNT_ONLY, CLASS_BYTES, CLASS_FINGERPRINT, CLASS_WORDS,  # noqa: F401
                   CLASS_DNA, MAX_M, NOALLOC_SCRATCH_BYTES, N_CLASSES, PLAN_COLLIDE, PLAN_DNA,
                   PLAN_FORCE_DIRECT, PLAN_FORCE_FINGERPRINT, PLAN_NO_STRIDE, PLAN_PREFIX4,
                   PLAN_SHORT_RUN, PLAN_SIGMA, VARIANT_DNA, VARIANT_STRIDE,
                   PLAN_HASH_BITS, PLAN_HOST_ONLY, VARIANT_DIRECT, VARIANT_FINGERPRINT,
                   WRITE_AUTO, WRITE_SINGLE_PASS, WRITE_TWO_PHASE)

__all__ = ["EpsmError", "Plan", "search", "count", "search_into", "count_into", "reserve",
           "stream_check", "lib", "library_path", "Batch", "BatchPlan", "search_batch",
           "set_tile_config", "set_batch_config", "tile_configs", "set_tune_table",
           "set_default_hash_bits", "pack_dna", "search_dna", "count_dna", "search_dna_into",
           "count_dna_into", "debug_force_giveup", "search_noalloc_into", "release",
           "set_variant_table", "estimate_alphabet"]


def lib():
    return _lib.load()


def library_path() -> str:
    return _lib.LIB_PATH


class EpsmError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        self.status = status
        self.name = L.epsm_status_string(status).decode()
        self.detail = L.epsm_last_error().decode()
        super().__init__(f"{where}: {self.name}: {self.detail}")


def _check(status: int, where: str) -> None:
    if status != _lib.EPSM_OK:
        raise EpsmError(status, where)


def _stream_handle(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _torch_stream(stream):
    """The torch stream a helper runs on: the caller's, else the current one."""
    if stream is None:
        return torch.cuda.current_stream()
    if isinstance(stream, int):
        return torch.cuda.ExternalStream(stream) if stream else torch.cuda.default_stream()
    return stream


class Plan:
    """A preprocessed pattern (epsm_plan).  Device tables live on the current device."""

    def __init__(self, pattern: bytes, flags: int = 0):
        pattern = bytes(pattern)
        self.pattern = pattern
        self.flags = flags
        self._handle = ctypes.c_void_p()
        self._buf = ctypes.create_string_buffer(pattern, max(len(pattern), 1))
        _check(lib().epsm_plan(ctypes.cast(self._buf, ctypes.c_void_p), len(pattern), flags,
                               ctypes.byref(self._handle)), "epsm_plan")

    @property
    def handle(self) -> int:
        return self._handle.value

    @property
    def m(self) -> int:
        return len(self.pattern)

    def info(self) -> dict:
        inf = _lib.PlanInfo()
        _check(lib().epsm_plan_get_info(self._handle, ctypes.byref(inf)), "epsm_plan_get_info")
        table = None
        if inf.table:
            table = [inf.table[i] for i in range(1 << inf.hash_bits)]
        return {
            "m": inf.m, "variant": inf.variant, "flags": inf.flags, "hash_bits": inf.hash_bits,
            "prefix_words": inf.prefix_words, "words": list(inf.words), "masks": list(inf.masks),
            "table": table, "device": inf.device, "kernel_class": inf.kernel_class, "stride": inf.stride,
            "prefix_bytes": inf.prefix_bytes, "run_blocks": inf.run_blocks, "table_row": inf.table_row,
        }

    def close(self) -> None:
        if self._handle and self._handle.value:
            lib().epsm_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _as_plan(pattern_or_plan, flags: int = 0) -> Plan:
    if isinstance(pattern_or_plan, Plan):
        return pattern_or_plan
    return Plan(pattern_or_plan, flags)


def _check_text(text: torch.Tensor) -> None:
    if not isinstance(text, torch.Tensor) or text.dtype != torch.uint8 or not text.is_cuda:
        raise TypeError("text must be a uint8 CUDA (HIP) tensor")
    if text.dim() != 1 or (text.numel() > 1 and text.stride(0) != 1):
        raise ValueError("text must be a contiguous 1-D tensor")


def search_into(plan: Plan, text: torch.Tensor, out: torch.Tensor | None, n_hits: torch.Tensor,
                stream=None) -> None:
    """epsm_search into caller tensors: out (int64), n_hits (uint64/int64, 1 element)."""
    _check_text(text)
    cap = 0 if out is None else out.numel()
    out_ptr = None if out is None or cap == 0 else out.data_ptr()
    _check(lib().epsm_search(plan.handle, text.data_ptr() if text.numel() else None,
                             text.numel(), out_ptr, cap, n_hits.data_ptr(),
                             _stream_handle(stream)), "epsm_search")


def search_noalloc_into(plan: Plan, text: torch.Tensor, out: torch.Tensor | None, n_hits: torch.Tensor,
                        stream=None) -> None:
    """epsm_search_noalloc into caller tensors (the library's static scratch
    instead of a stream workspace; calls on one device must not overlap)."""
    _check_text(text)
    cap = 0 if out is None else out.numel()
    out_ptr = None if out is None or cap == 0 else out.data_ptr()
    _check(lib().epsm_search_noalloc(plan.handle, text.data_ptr() if text.numel() else None,
                                     text.numel(), out_ptr, cap, n_hits.data_ptr(),
                                     _stream_handle(stream)), "epsm_search_noalloc")


def count_into(plan: Plan, text: torch.Tensor, n_hits: torch.Tensor, stream=None) -> None:
    _check_text(text)
    _check(lib().epsm_count(plan.handle, text.data_ptr() if text.numel() else None,
                            text.numel(), n_hits.data_ptr(), _stream_handle(stream)),
           "epsm_count")


def _sync_and_check(s) -> None:
    """Wait for stream s and raise if a kernel on it gave up a bounded wait."""
    _check(lib().epsm_stream_check(_stream_handle(s)), "epsm_stream_check")


def count(text: torch.Tensor, pattern, flags: int = 0, stream=None) -> int:
    """Number of occurrences (runs on `stream` and synchronises it)."""
    plan = _as_plan(pattern, flags)
    s = _torch_stream(stream)
    with torch.cuda.stream(s):
        hits = torch.zeros(1, dtype=torch.int64, device=text.device)
        count_into(plan, text, hits, s)
        _sync_and_check(s)
        return int(hits.item())


def search(text: torch.Tensor, pattern, flags: int = 0, stream=None) -> torch.Tensor:
    """All occurrence positions as an int64 tensor (counts, allocates, then
    searches, all on `stream`; synchronises it and raises if a bounded wait of
    the search gave up)."""
    plan = _as_plan(pattern, flags)
    s = _torch_stream(stream)
    with torch.cuda.stream(s):
        hits = torch.zeros(1, dtype=torch.int64, device=text.device)
        count_into(plan, text, hits, s)
        _sync_and_check(s)
        n = int(hits.item())
        out = torch.empty(n, dtype=torch.int64, device=text.device)
        search_into(plan, text, out, hits, s)
        _sync_and_check(s)
        if int(hits.item()) != n:
            raise RuntimeError("count changed between passes")
        return out


def pack_dna(codes: torch.Tensor, stream=None) -> torch.Tensor:
    """2-bit packing (epsm_pack_dna) of a uint8 CUDA tensor of codes 0..3."""
    _check_text(codes)
    n = codes.numel()
    packed = torch.empty((n + 3) // 4, dtype=torch.uint8, device=codes.device)
    _check(lib().epsm_pack_dna(codes.data_ptr() if n else None, n, packed.data_ptr() if n else None,
                               _stream_handle(stream)), "epsm_pack_dna")
    return packed


def _check_packed(packed: torch.Tensor, n: int) -> None:
    _check_text(packed)
    if packed.numel() < (n + 3) // 4:
        raise ValueError(f"a packed text of {n} symbols needs {(n + 3) // 4} bytes")


def search_dna_into(plan: Plan, packed: torch.Tensor, n: int, out: torch.Tensor | None,
                    n_hits: torch.Tensor, stream=None) -> None:
    """epsm_search_dna: positions (symbol indices) of plan in n packed symbols."""
    _check_packed(packed, n)
    cap = 0 if out is None else out.numel()
    _check(lib().epsm_search_dna(plan.handle, packed.data_ptr() if n else None, n,
                                 None if out is None or cap == 0 else out.data_ptr(), cap,
                                 n_hits.data_ptr(), _stream_handle(stream)), "epsm_search_dna")


def count_dna_into(plan: Plan, packed: torch.Tensor, n: int, n_hits: torch.Tensor, stream=None) -> None:
    _check_packed(packed, n)
    _check(lib().epsm_count_dna(plan.handle, packed.data_ptr() if n else None, n, n_hits.data_ptr(),
                                _stream_handle(stream)), "epsm_count_dna")


def _as_dna_plan(pattern_or_plan) -> Plan:
    if isinstance(pattern_or_plan, Plan):
        return pattern_or_plan
    return Plan(pattern_or_plan, PLAN_DNA)


def count_dna(packed: torch.Tensor, n: int, pattern, stream=None) -> int:
    """Occurrences of a code pattern (bytes of 0..3, or a PLAN_DNA Plan) in n packed symbols."""
    plan = _as_dna_plan(pattern)
    s = _torch_stream(stream)
    with torch.cuda.stream(s):
        hits = torch.zeros(1, dtype=torch.int64, device=packed.device)
        count_dna_into(plan, packed, n, hits, s)
        _sync_and_check(s)
        return int(hits.item())


def search_dna(packed: torch.Tensor, n: int, pattern, stream=None) -> torch.Tensor:
    """All occurrence positions (symbol indices) as an int64 tensor (on `stream`)."""
    plan = _as_dna_plan(pattern)
    s = _torch_stream(stream)
    with torch.cuda.stream(s):
        hits = torch.zeros(1, dtype=torch.int64, device=packed.device)
        count_dna_into(plan, packed, n, hits, s)
        _sync_and_check(s)
        k = int(hits.item())
        out = torch.empty(k, dtype=torch.int64, device=packed.device)
        search_dna_into(plan, packed, n, out, hits, s)
        _sync_and_check(s)
        if int(hits.item()) != k:
            raise RuntimeError("count changed between passes")
        return out


def set_tile_config(waves: int, pieces: int) -> None:
    """Workgroup tile for later searches: waves x pieces KiB (output is unaffected)."""
    _check(lib().epsm_set_tile_config(waves, pieces), "epsm_set_tile_config")


def stream_check(stream=None) -> None:
    """Synchronise the stream; raise if a kernel on it gave up a bounded wait."""
    _check(lib().epsm_stream_check(_stream_handle(stream)), "epsm_stream_check")


def reserve(max_n: int, batch_bytes: int = 0, stream=None) -> None:
    """epsm_reserve: workspace for texts up to max_n and one-shot batches whose
    workspace (Batch.workspace_bytes) is up to batch_bytes; call it before
    capturing the stream into a graph."""
    _check(lib().epsm_reserve(_stream_handle(stream), max_n, batch_bytes), "epsm_reserve")


def release() -> None:
    """epsm_release: free every cached workspace, fault word and staging block
    (synchronises the device; graphs that captured library calls must not be
    replayed afterwards)."""
    lib().epsm_release()


def debug_force_giveup(enable: bool) -> None:
    """Test hook epsm_debug_force_giveup (process-wide)."""
    lib().epsm_debug_force_giveup(1 if enable else 0)


# ---------------------------------------------------------------------------
# batched search


class Batch:
    """Marshalled epsm_batch: texts (uint8 CUDA tensors) and (text index, Plan) pairs.

    Output tensors are allocated by the caller or by search_batch; this class
    only keeps the ctypes arrays (and the tensors they point into) alive.
    """

    def __init__(self, texts, pairs, out=None, counts=None, offsets=None, total=None,
                 count_only: bool = False, groups: bool = True):
        for t in texts:
            _check_text(t)
        self.texts = list(texts)
        self.pairs = [(int(ti), p) for ti, p in pairs]
        dev = self.texts[0].device if self.texts else torch.device("cuda")
        n_pairs = len(self.pairs)
        self.counts = counts if counts is not None else torch.zeros(max(n_pairs, 1), dtype=torch.int64, device=dev)
        self.offsets = offsets if offsets is not None else torch.zeros(max(n_pairs, 1), dtype=torch.int64, device=dev)
        self.total = total if total is not None else torch.zeros(1, dtype=torch.int64, device=dev)
        self.out = out
        tr = (_lib.TextRef * max(len(self.texts), 1))()
        for i, t in enumerate(self.texts):
            tr[i].d_text = t.data_ptr() if t.numel() else None
            tr[i].n = t.numel()
        pr = (_lib.PairRef * max(n_pairs, 1))()
        for k, (ti, p) in enumerate(self.pairs):
            pr[k].text = ti
            pr[k].plan = p.handle
        self._tr, self._pr = tr, pr
        b = _lib.Batch()
        b.texts = ctypes.cast(tr, ctypes.POINTER(_lib.TextRef))
        b.n_texts = len(self.texts)
        b.pairs = ctypes.cast(pr, ctypes.POINTER(_lib.PairRef))
        b.n_pairs = n_pairs
        b.d_out = out.data_ptr() if out is not None and out.numel() else None
        b.out_capacity = 0 if out is None else out.numel()
        b.d_counts = self.counts.data_ptr()
        b.d_offsets = self.offsets.data_ptr()
        b.d_total = self.total.data_ptr()
        b.flags = (BATCH_COUNT_ONLY if count_only else 0) | (0 if groups else _lib.BATCH_NO_GROUPS)
        self.struct = b

    def run(self, stream=None) -> None:
        """One-shot epsm_search_batch (descriptors go through the stream's workspace)."""
        _check(lib().epsm_search_batch(ctypes.byref(self.struct), _stream_handle(stream)),
               "epsm_search_batch")

    def workspace_bytes(self) -> int:
        """epsm_batch_workspace: stream workspace a one-shot run of this batch needs."""
        b = ctypes.c_uint64()
        _check(lib().epsm_batch_workspace(ctypes.byref(self.struct), ctypes.byref(b)),
               "epsm_batch_workspace")
        return b.value


class BatchPlan:
    """A prepared batch (epsm_batch_prepare); launch() replays a captured graph."""

    def __init__(self, batch: Batch):
        self.batch = batch  # keeps the referenced tensors and plans alive
        self._handle = ctypes.c_void_p()
        _check(lib().epsm_batch_prepare(ctypes.byref(batch.struct), ctypes.byref(self._handle)),
               "epsm_batch_prepare")

    def launch(self, stream=None) -> None:
        _check(lib().epsm_batch_launch(self._handle, _stream_handle(stream)), "epsm_batch_launch")

    def info(self) -> dict:
        u, e, tb = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
        _check(lib().epsm_batch_get_info(self._handle, ctypes.byref(u), ctypes.byref(e),
                                         ctypes.byref(tb)), "epsm_batch_get_info")
        return {"units": u.value, "entries": e.value, "tile_bytes": tb.value}

    def close(self) -> None:
        if self._handle and self._handle.value:
            lib().epsm_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def search_batch(texts, pairs, stream=None, groups: bool = True):
    """All (text, pattern) pairs; returns (positions, counts, offsets) as int64 tensors.

    pairs: iterable of (text index, Plan or bytes).  Runs a count-only batch to
    size the output, then the full batch.  groups=False filters every pair on
    its own in the count pass (EPSM_BATCH_NO_GROUPS).
    """
    pairs = [(ti, _as_plan(p)) for ti, p in pairs]
    s = _torch_stream(stream)
    with torch.cuda.stream(s):
        b0 = Batch(texts, pairs, count_only=True, groups=groups)
        b0.run(s)
        s.synchronize()
        total = int(b0.total.item())
        dev = texts[0].device if texts else torch.device("cuda")
        out = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
        b1 = Batch(texts, pairs, out=out[:total] if total else None, groups=groups)
        b1.run(s)
        s.synchronize()
        n = len(pairs)
        return out[:total], b1.counts[:n], b1.offsets[:n]


def tile_configs() -> list[tuple[int, int]]:
    """Built (waves, pieces) tile configurations, default first."""
    n = lib().epsm_tile_configs(None, None, 0)
    w = (ctypes.c_uint32 * n)()
    p = (ctypes.c_uint32 * n)()
    lib().epsm_tile_configs(w, p, n)
    return [(w[i], p[i]) for i in range(n)]


def set_tune_table(entries) -> None:
    """Install the tile table (epsm_set_tune_table): an iterable of
    (kernel_class, count_only, n_max, waves, pieces[, strategy]); first match
    wins; strategy defaults to WRITE_AUTO."""
    rows = [tuple(int(x) for x in e) + ((WRITE_AUTO,) if len(e) == 5 else ()) for e in entries]
    arr = (_lib.TuneEntry * max(len(rows), 1))(*[_lib.TuneEntry(*r) for r in rows])
    _check(lib().epsm_set_tune_table(arr, len(rows)), "epsm_set_tune_table")


def set_default_hash_bits(k: int) -> None:
    """Fingerprint width for plans made later without PLAN_HASH_BITS (0: 11)."""
    _check(lib().epsm_set_default_hash_bits(k), "epsm_set_default_hash_bits")


def set_variant_table(entries) -> None:
    """Install the variant table (epsm_set_variant_table): an iterable of
    (m_min, m_max, sigma_min, sigma_max, variant, flags); first match wins."""
    rows = [tuple(int(x) for x in e) for e in entries]
    arr = (_lib.VariantEntry * max(len(rows), 1))(*[_lib.VariantEntry(*r) for r in rows])
    _check(lib().epsm_set_variant_table(arr, len(rows)), "epsm_set_variant_table")


def estimate_alphabet(text: torch.Tensor, stream=None) -> int:
    """epsm_estimate_alphabet: effective alphabet size of the text's first
    64 KiB (synchronises the stream); for PLAN_SIGMA."""
    _check_text(text)
    v = ctypes.c_uint32()
    _check(lib().epsm_estimate_alphabet(text.data_ptr() if text.numel() else None, text.numel(),
                                        ctypes.byref(v), _stream_handle(stream)), "epsm_estimate_alphabet")
    return v.value


def set_batch_config(waves: int) -> None:
    _check(lib().epsm_set_batch_config(waves), "epsm_set_batch_config")
