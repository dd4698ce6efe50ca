"""ctypes declarations of the C ABI in include/epsm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libepsm.so")

EPSM_OK = 0
EPSM_EINVAL = 1
EPSM_ENOMEM = 2
EPSM_EDEVICE = 3
EPSM_EUNSUPPORTED = 4

PLAN_HOST_ONLY = 0x1
PLAN_FORCE_DIRECT = 0x2
PLAN_FORCE_FINGERPRINT = 0x4
PLAN_COLLIDE = 0x8
PLAN_DNA = 0x10
PLAN_NO_STRIDE = 0x20
PLAN_PREFIX4 = 0x40
PLAN_SHORT_RUN = 0x80


def PLAN_SIGMA(s: int) -> int:
    return (s & 0x1FF) << 16



def PLAN_HASH_BITS(k: int) -> int:
    return (k & 0xF) << 8


VARIANT_DIRECT = 1
VARIANT_FINGERPRINT = 2
VARIANT_DNA = 3
VARIANT_STRIDE = 4
WRITE_AUTO = 0
WRITE_SINGLE_PASS = 1
WRITE_TWO_PHASE = 2
CLASS_BYTES = 0
CLASS_WORDS = 1
CLASS_FINGERPRINT = 2
CLASS_DNA = 3
N_CLASSES = 4
SERVER_FAIL_OUTPUT_ALLOC = 0x1
BATCH_COUNT_ONLY = 0x1
BATCH_NO_GROUPS = 0x2
MAX_M = 4096
NOALLOC_SCRATCH_BYTES = 8 << 20


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_uint64),
        ("variant", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("hash_bits", ctypes.c_uint32),
        ("prefix_words", ctypes.c_uint32),
        ("words", ctypes.c_uint32 * 8),
        ("masks", ctypes.c_uint32 * 8),
        ("table", ctypes.POINTER(ctypes.c_uint16)),
        ("device", ctypes.c_int32),
        ("kernel_class", ctypes.c_uint32),
        ("stride", ctypes.c_uint32),
        ("prefix_bytes", ctypes.c_uint32),
        ("run_blocks", ctypes.c_uint32),
        ("table_row", ctypes.c_uint32),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [("kernel_class", ctypes.c_uint32), ("count_only", ctypes.c_uint32),
                ("n_max", ctypes.c_uint64), ("waves", ctypes.c_uint32), ("pieces", ctypes.c_uint32),
                ("strategy", ctypes.c_uint32)]


class VariantEntry(ctypes.Structure):
    _fields_ = [("m_min", ctypes.c_uint32), ("m_max", ctypes.c_uint32), ("sigma_min", ctypes.c_uint32),
                ("sigma_max", ctypes.c_uint32), ("variant", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class TextRef(ctypes.Structure):
    _fields_ = [("d_text", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class PairRef(ctypes.Structure):
    _fields_ = [("text", ctypes.c_uint32), ("plan", ctypes.c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [
        ("texts", ctypes.POINTER(TextRef)),
        ("n_texts", ctypes.c_uint32),
        ("pairs", ctypes.POINTER(PairRef)),
        ("n_pairs", ctypes.c_uint32),
        ("d_out", ctypes.c_void_p),
        ("out_capacity", ctypes.c_uint64),
        ("d_counts", ctypes.c_void_p),
        ("d_offsets", ctypes.c_void_p),
        ("d_total", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_uint32),
        ("max_batch_queries", ctypes.c_uint32),
        ("max_batch_entries", ctypes.c_uint64),
        ("hbm_budget", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
    ]


class QueryResult(ctypes.Structure):
    _fields_ = [
        ("query_id", ctypes.c_uint64),
        ("text_id", ctypes.c_uint32),
        ("n_patterns", ctypes.c_uint32),
        ("status", ctypes.c_int32),
        ("batch_queries", ctypes.c_uint32),
        ("total", ctypes.c_uint64),
        ("counts", ctypes.POINTER(ctypes.c_uint64)),
        ("offsets", ctypes.POINTER(ctypes.c_uint64)),
        ("positions", ctypes.POINTER(ctypes.c_int64)),
        ("submit_time", ctypes.c_double),
        ("start_time", ctypes.c_double),
        ("done_time", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("submitted", "completed", "in_flight", "queued", "batches", "bytes_reserved",
                 "bytes_peak")]


# name -> (restype, argtypes); every symbol include/epsm.h declares
SIGNATURES = {
    "epsm_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "epsm_plan_destroy": (None, [ctypes.c_void_p]),
    "epsm_plan_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanInfo)]),
    "epsm_fingerprint": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_int]),
    "epsm_search": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    "epsm_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "epsm_search_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                           ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "epsm_search_batch": (ctypes.c_int, [ctypes.POINTER(Batch), ctypes.c_void_p]),
    "epsm_pack_dna": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "epsm_search_dna": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "epsm_count_dna": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "epsm_set_tile_config": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32]),
    "epsm_set_batch_config": (ctypes.c_int, [ctypes.c_uint32]),
    "epsm_tile_configs": (ctypes.c_uint32, [ctypes.POINTER(ctypes.c_uint32),
                                            ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32]),
    "epsm_set_tune_table": (ctypes.c_int, [ctypes.POINTER(TuneEntry), ctypes.c_uint32]),
    "epsm_set_default_hash_bits": (ctypes.c_int, [ctypes.c_uint32]),
    "epsm_set_variant_table": (ctypes.c_int, [ctypes.POINTER(VariantEntry), ctypes.c_uint32]),
    "epsm_estimate_alphabet": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                              ctypes.POINTER(ctypes.c_uint32), ctypes.c_void_p]),
    "epsm_batch_prepare": (ctypes.c_int, [ctypes.POINTER(Batch), ctypes.POINTER(ctypes.c_void_p)]),
    "epsm_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "epsm_batch_destroy": (None, [ctypes.c_void_p]),
    "epsm_batch_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint32)]),
    "epsm_reserve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]),
    "epsm_release": (None, []),
    "epsm_stream_check": (ctypes.c_int, [ctypes.c_void_p]),
    "epsm_debug_force_giveup": (None, [ctypes.c_int]),
    "epsm_batch_workspace": (ctypes.c_int, [ctypes.POINTER(Batch), ctypes.POINTER(ctypes.c_uint64)]),
    "epsm_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "epsm_server_add_text": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                            ctypes.POINTER(ctypes.c_uint32)]),
    "epsm_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "epsm_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(QueryResult), ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32]),
    "epsm_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "epsm_server_now": (ctypes.c_double, [ctypes.c_void_p]),
    "epsm_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "epsm_server_destroy": (None, [ctypes.c_void_p]),
    "epsm_last_error": (ctypes.c_char_p, []),
    "epsm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "epsm_version": (ctypes.c_int, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libepsm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with paper_1209_6449_amd.build.build() "
            "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
