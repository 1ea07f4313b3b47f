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
    u32, u64, i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
    lib.oracle_scan.argtypes = [P, P, u32, P, u64, P, P, P]
    lib.oracle_scan.restype = ctypes.c_int
    lib.oracle_scan_mt.argtypes = [P, P, u32, P, u64, P, P, P, ctypes.c_int, P]
    lib.oracle_scan_mt.restype = ctypes.c_int
    lib.oracle_occurrences.argtypes = [P, P, u32, P, u64, P, P, P, P, u64, P, P, P]
    lib.oracle_occurrences.restype = ctypes.c_int
    lib.oracle_scan_bytes_mt.argtypes = [P, P, u32, P, u64, P, P, P, ctypes.c_int, P]
    lib.oracle_scan_bytes_mt.restype = ctypes.c_int
    lib.oracle_occurrences_bytes.argtypes = [P, P, u32, P, u64, P, P, P, P, u64, P, P, P]
    lib.oracle_occurrences_bytes.restype = ctypes.c_int
    lib.oracle_goto.argtypes = [P, P, u32, P, P, i64]
    lib.oracle_goto.restype = i64
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            _lib = _declare(ctypes.CDLL(_LIB_PATH))
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


def scan_bytes(patterns, text, threads: int = 1, lib=None, counts: bool = False):
    """The oracle over the byte alphabet (the general-purpose PFAC setting):
    every byte value is a symbol, patterns are any non-empty byte strings.
    Returns (match int32[n], total) and with ``counts`` the per-position
    occurrence counts, as ``scan``."""
    lib = lib or _load()
    arr, lens, keep, num = _pattern_args(patterns)
    t = _as_text(text)
    n = int(t.size)
    match = np.zeros(n, dtype=np.int32)
    count = np.zeros(n, dtype=np.uint32) if counts else None
    total = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    rc = lib.oracle_scan_bytes_mt(ctypes.cast(arr, ctypes.c_void_p), lens.ctypes.data, num,
                                  t.ctypes.data if n else None, n, match.ctypes.data if n else None,
                                  ctypes.addressof(total), ctypes.addressof(bad),
                                  int(max(1, threads)),
                                  count.ctypes.data if (counts and n) else None)
    del keep
    if rc != 0:
        raise OracleError(rc, bad.value)
    if counts:
        return match, int(total.value), count
    return match, int(total.value)


def scan(patterns, text, threads: int = 1, lib=None, counts: bool = False):
    """Run the oracle.  Returns (match int32[n], total occurrences), and with
    ``counts`` also count uint32[n] = occurrences starting at each position.

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
    count = np.zeros(n, dtype=np.uint32) if counts else None
    total = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    if threads <= 1 and not counts:
        rc = lib.oracle_scan(ctypes.cast(arr, ctypes.c_void_p), lens.ctypes.data, num,
                             t.ctypes.data if n else None, n,
                             match.ctypes.data if n else None,
                             ctypes.addressof(total), ctypes.addressof(bad))
    else:
        rc = lib.oracle_scan_mt(ctypes.cast(arr, ctypes.c_void_p), lens.ctypes.data, num,
                                t.ctypes.data if n else None, n,
                                match.ctypes.data if n else None,
                                ctypes.addressof(total), ctypes.addressof(bad),
                                int(max(1, threads)),
                                count.ctypes.data if (counts and n) else None)
    del keep
    if rc != 0:
        raise OracleError(rc, bad.value)
    if counts:
        return match, int(total.value), count
    return match, int(total.value)


def occurrences(patterns, text, lib=None, alphabet: str = "dna"):
    """Every (start position, pattern ID) pair with the pattern at that start,
    sub-patterns included: an int64 array (k, 2) in ascending position, then
    ascending pattern length, then ascending ID.  The scan reports them by
    end position; the order above is a plain sort of that list.  ``alphabet``
    "bytes": every byte value a symbol (as ``scan_bytes``)."""
    lib = lib or _load()
    entry = lib.oracle_occurrences_bytes if alphabet == "bytes" else lib.oracle_occurrences
    arr, lens, keep, num = _pattern_args(patterns)
    t = _as_text(text)
    n = int(t.size)
    match = np.zeros(max(1, n), dtype=np.int32)
    total = ctypes.c_uint64(0)
    nocc = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    cap = 0
    pos = np.zeros(1, dtype=np.uint32)
    ids = np.zeros(1, dtype=np.int32)
    for _ in range(2):              # first pass sizes the list
        rc = entry(ctypes.cast(arr, ctypes.c_void_p), lens.ctypes.data, num,
                                    t.ctypes.data if n else None, n, match.ctypes.data, None,
                                    pos.ctypes.data, ids.ctypes.data, cap,
                                    ctypes.addressof(nocc), ctypes.addressof(total),
                                    ctypes.addressof(bad))
        if rc != 0:
            raise OracleError(rc, bad.value)
        if nocc.value <= cap:
            break
        cap = int(nocc.value)
        pos = np.zeros(cap, dtype=np.uint32)
        ids = np.zeros(cap, dtype=np.int32)
    del keep
    k = int(nocc.value)
    plen = np.array([len(p) for p in patterns] or [0], dtype=np.int64)
    out = np.stack([pos[:k].astype(np.int64), ids[:k].astype(np.int64)], axis=1)
    order = np.lexsort((out[:, 1], plen[out[:, 1] - 1] if k else out[:, 1], out[:, 0]))
    return out[order]


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
