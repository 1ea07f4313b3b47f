"""ctypes declarations of the C ABI in include/pfac.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfac.so")

PFAC_TEXT_ASCII = 0
PFAC_TEXT_2BIT = 1
PFAC_VARIANT_TILED = 0
PFAC_VARIANT_GLOBAL = 1
PFAC_VARIANT_GLOBAL_TWO_ARRAYS = 2
PFAC_VARIANT_GLOBAL_MERGED = 3
PFAC_LEVELS_NONE = 0xFFFFFFFF
PFAC_HASH_NONE = 0xFFFFFFFF
PFAC_WALKS_INLINE = 1
PFAC_WALKS_DEFERRED = 2
PFAC_PREFIX_NONE = 0xFFFFFFFF
PFAC_PAIR_NONE = 0xFFFFFFFF

EXPORTS = (
    "pfac_build_table", "pfac_build_table_bytes", "pfac_build_table_device",
    "pfac_table_update", "pfac_table_blob", "pfac_table_info", "pfac_free_table", "pfac_match",
    "pfac_match_all", "pfac_match_batch", "pfac_batch_create", "pfac_batch_launch", "pfac_batch_info",
    "pfac_batch_free",
    "pfac_default_plan", "pfac_build_host", "pfac_build_host_image", "pfac_build_host_hash",
    "pfac_build_host_hash1", "pfac_build_host_chain", "pfac_build_host_prefix",
    "pfac_strerror",
    "pfac_version",
)


class PfacPlan(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("depth", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("variant", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("hash_bits", ctypes.c_uint32),
                ("walks", ctypes.c_uint32), ("tile", ctypes.c_uint32),
                ("prefix", ctypes.c_uint32), ("pair", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class PfacTableStats(ctypes.Structure):
    _fields_ = [("num_states", ctypes.c_uint64), ("num_patterns", ctypes.c_uint32),
                ("max_len", ctypes.c_uint32), ("min_len", ctypes.c_uint32),
                ("max_depth_full", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
                ("states_to_depth", ctypes.c_uint64 * 9), ("prefix_k", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("prefix_keys", ctypes.c_uint64)]


class PfacTextDesc(ctypes.Structure):
    _fields_ = [("text_offset", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("match_offset", ctypes.c_uint64), ("table", ctypes.c_uint32),
                ("enc", ctypes.c_uint32)]


_lock = threading.Lock()
_lib = None


class PfacError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = "%s failed: %s (%d)" % (what or "pfac", strerror(code), code)
        super().__init__(msg)
        self.code = code


def lib():
    """The loaded libpfac.so.  Raises if the extension has not been built:
    there is no fallback path."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    "libpfac.so is not built (%s); run `python -m paper_1811_10498_amd.build` "
                    "or __graft_entry__.build()" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            P = ctypes.c_void_p
            u32, u64, i32, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
            L.pfac_build_table.argtypes = [P, P, u32, ctypes.POINTER(P), ctypes.POINTER(i64)]
            L.pfac_build_table.restype = ctypes.c_int
            L.pfac_build_table_bytes.argtypes = [P, P, u32, ctypes.POINTER(P),
                                                 ctypes.POINTER(i64)]
            L.pfac_build_table_bytes.restype = ctypes.c_int
            L.pfac_build_table_device.argtypes = [P, P, P, u32, ctypes.POINTER(P),
                                                  ctypes.POINTER(i64)]
            L.pfac_build_table_device.restype = ctypes.c_int
            L.pfac_table_update.argtypes = [P, P, P, u32, P, u32, ctypes.POINTER(P),
                                            ctypes.POINTER(ctypes.c_int32)]
            L.pfac_table_update.restype = ctypes.c_int
            L.pfac_table_blob.argtypes = [P, P, u64, ctypes.POINTER(u64)]
            L.pfac_table_blob.restype = ctypes.c_int
            L.pfac_table_info.argtypes = [P, ctypes.POINTER(PfacTableStats)]
            L.pfac_table_info.restype = ctypes.c_int
            L.pfac_free_table.argtypes = [P]
            L.pfac_free_table.restype = None
            L.pfac_match.argtypes = [P, P, u64, ctypes.c_int, P, P, u64, P,
                                     ctypes.POINTER(PfacPlan), P]
            L.pfac_match.restype = ctypes.c_int
            L.pfac_match_all.argtypes = [P, P, u64, ctypes.c_int, P, u64, P,
                                         ctypes.POINTER(PfacPlan), P]
            L.pfac_match_all.restype = ctypes.c_int
            L.pfac_match_batch.argtypes = [P, u32, P, u32, P, P, P, u64, P,
                                           ctypes.POINTER(PfacPlan), P]
            L.pfac_match_batch.restype = ctypes.c_int
            L.pfac_batch_create.argtypes = [P, u32, P, u32, ctypes.POINTER(PfacPlan),
                                            ctypes.POINTER(P)]
            L.pfac_batch_create.restype = ctypes.c_int
            L.pfac_batch_launch.argtypes = [P, P, P, P, u64, P, P]
            L.pfac_batch_launch.restype = ctypes.c_int
            L.pfac_batch_info.argtypes = [P, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                          ctypes.POINTER(u64)]
            L.pfac_batch_info.restype = ctypes.c_int
            L.pfac_batch_free.argtypes = [P]
            L.pfac_batch_free.restype = None
            L.pfac_default_plan.argtypes = [P, u64, ctypes.c_int, ctypes.POINTER(PfacPlan)]
            L.pfac_default_plan.restype = ctypes.c_int
            L.pfac_build_host.argtypes = [P, P, u32, P, P, P, u64, u32, P, P, P,
                                          ctypes.POINTER(u64), ctypes.POINTER(i64)]
            L.pfac_build_host.restype = ctypes.c_int
            L.pfac_build_host_image.argtypes = [P, P, u32, u32, P, u64, P, ctypes.POINTER(u64),
                                                ctypes.POINTER(i64)]
            L.pfac_build_host_image.restype = ctypes.c_int
            L.pfac_build_host_hash.argtypes = [P, P, u32, u32, P, ctypes.POINTER(u32),
                                               ctypes.POINTER(i64)]
            L.pfac_build_host_hash.restype = ctypes.c_int
            L.pfac_build_host_hash1.argtypes = [P, P, u32, u32, P, ctypes.POINTER(u32),
                                                ctypes.POINTER(i64)]
            L.pfac_build_host_hash1.restype = ctypes.c_int
            L.pfac_build_host_chain.argtypes = [P, P, u32, P, u64, ctypes.POINTER(u64),
                                                ctypes.POINTER(i64)]
            L.pfac_build_host_chain.restype = ctypes.c_int
            if hasattr(L, "pfac_match_noalloc"):
                L.pfac_match_noalloc.argtypes = [P, P, u64, ctypes.c_int, P, P, u64, P,
                                                 ctypes.POINTER(PfacPlan), P]
                L.pfac_match_noalloc.restype = ctypes.c_int
                L.pfac_noalloc_scratch_bytes.argtypes = []
                L.pfac_noalloc_scratch_bytes.restype = u64
            L.pfac_build_host_prefix.argtypes = [P, P, u32, P, u64, ctypes.POINTER(u32),
                                                 ctypes.POINTER(u64), ctypes.POINTER(i64)]
            L.pfac_build_host_prefix.restype = ctypes.c_int
            L.pfac_strerror.argtypes = [ctypes.c_int]
            L.pfac_strerror.restype = ctypes.c_char_p
            L.pfac_version.argtypes = []
            L.pfac_version.restype = ctypes.c_char_p
            del i32
            _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().pfac_strerror(int(code)).decode()
    except ImportError:
        return "status %d" % code


def check(rc: int, what: str):
    if rc != 0:
        raise PfacError(rc, what)
