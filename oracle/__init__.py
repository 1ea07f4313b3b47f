"""CPU correctness oracle for PFAC DNA matching.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library
(``paper_1811_10498_amd``) never imports this package, and this package
imports nothing from it.

The oracle is the classic sequential Aho-Corasick machine (goto, failure and
output functions; paper Sec. III, Figs. 1-2) written in plain C in
``ac_oracle.c``, wrapped here with ctypes.  It returns, for every start
position, the ID of the longest pattern starting there (PFAC's reporting
rule, Sec. IV) and the total number of (pattern, position) occurrences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ac_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ac_oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_mutant(k: int, out_dir: str) -> str:
    """Compile the oracle with planted mistake k (tests only)."""
    path = os.path.join(out_dir, "liboracle_mutant%d.so" % k)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-DORACLE_MUTANT=%d" % k, "-o", path, _SRC])
    return path


def _declare(lib):
    P = ctypes.c_void_p
    lib.oracle_scan.argtypes = [P, P, ctypes.c_uint32, P, ctypes.c_uint64, P, P, P]
    lib.oracle_scan.restype = ctypes.c_int
    lib.oracle_scan_mt.argtypes = [P, P, ctypes.c_uint32, P, ctypes.c_uint64, P, P, P,
                                   ctypes.c_int]
    lib.oracle_scan_mt.restype = ctypes.c_int
    lib.oracle_goto.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_int64]
    lib.oracle_goto.restype = ctypes.c_int64
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            lib.oracle_scan.argtypes = [P, P, ctypes.c_uint32, P, ctypes.c_uint64, P, P, P]
            lib.oracle_scan.restype = ctypes.c_int
            lib.oracle_scan_mt.argtypes = [P, P, ctypes.c_uint32, P, ctypes.c_uint64, P, P, P,
                                           ctypes.c_int]
            lib.oracle_scan_mt.restype = ctypes.c_int
            lib.oracle_goto.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_int64]
            lib.oracle_goto.restype = ctypes.c_int64
            _lib = lib
    return _lib


class OracleError(ValueError):
    def __init__(self, code: int, bad_index: int):
        super().__init__("oracle error %d (pattern index %d)" % (code, bad_index))
        self.code = code
        self.bad_index = bad_index


def _pattern_args(patterns):
    pats = [bytes(p) if not isinstance(p, bytes) else p for p in patterns]
    bufs = [ctypes.create_string_buffer(p, len(p) + 1) for p in pats]
    arr = (ctypes.c_char_p * max(1, len(pats)))()
    for i, b in enumerate(bufs):
        arr[i] = ctypes.cast(b, ctypes.c_char_p)
    lens = np.array([len(p) for p in pats] or [0], dtype=np.uint32)
    return arr, lens, bufs, len(pats)


def _as_text(text) -> np.ndarray:
    if isinstance(text, (bytes, bytearray)):
        return np.frombuffer(bytes(text), dtype=np.uint8)
    t = np.ascontiguousarray(text)
    if t.dtype != np.uint8:
        raise TypeError("text must be uint8 ASCII bytes")
    return t


def scan(patterns, text, threads: int = 1, lib=None):
    """Run the oracle.  Returns (match int32[n], total occurrences).

    ``patterns`` is a sequence of ASCII byte strings (IDs 1..P in order);
    ``text`` is ASCII bytes or a uint8 array.  ``threads`` > 1 uses the
    chunked multi-threaded scan (identical result).  ``lib`` selects another
    build of the same source (the mutation tests).
    """
    lib = lib or _load()
    arr, lens, keep, num = _pattern_args(patterns)
    t = _as_text(text)
    n = int(t.size)
    match = np.zeros(n, dtype=np.int32)
    total = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    if threads <= 1:
        rc = lib.oracle_scan(ctypes.cast(arr, ctypes.c_void_p), lens.ctypes.data, num,
                             t.ctypes.data if n else None, n,
                             match.ctypes.data if n else None,
                             ctypes.addressof(total), ctypes.addressof(bad))
    else:
        rc = lib.oracle_scan_mt(ctypes.cast(arr, ctypes.c_void_p), lens.ctypes.data, num,
                                t.ctypes.data if n else None, n,
                                match.ctypes.data if n else None,
                                ctypes.addressof(total), ctypes.addressof(bad), int(threads))
    del keep
    if rc != 0:
        raise OracleError(rc, bad.value)
    return match, int(total.value)


def hits_of(match: np.ndarray):
    """Hit list of a match array: (positions uint32, ids int32), ascending position."""
    pos = np.nonzero(match)[0]
    return pos.astype(np.uint32), match[pos].astype(np.int32)


def goto_function(patterns):
    """Insertion-order goto function (before any renumbering).

    Returns (go int64[S,4] in A,C,G,T column order with -1 = fail,
    final int32[S] = smallest keyword ID ending at the state, 0 = none).
    """
    lib = _load()
    arr, lens, keep, num = _pattern_args(patterns)
    cap = 1 + int(lens.sum())
    go = np.full((cap, 4), -1, dtype=np.int64)
    fin = np.zeros(cap, dtype=np.int32)
    S = lib.oracle_goto(ctypes.cast(arr, ctypes.c_void_p), lens.ctypes.data, num,
                        go.ctypes.data, fin.ctypes.data, cap)
    del keep
    if S < 0:
        raise OracleError(int(S), -1)
    return go[:S].copy(), fin[:S].copy()
