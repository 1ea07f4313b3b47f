"""Pointwise PFAC oracle -- TEST INFRASTRUCTURE ONLY.

The plain definition of what a PFAC thread reports (Sec. IV: one thread per
start position, longest pattern only), evaluated independently at chosen
start positions, for sampled checks on texts too large to scan in a test:

    match(i) = ID of the longest pattern equal to T[i..i+|p|), the smallest ID
               among equal patterns, 0 if none;
    count(i) = number of pattern IDs whose pattern equals T[i..i+|p|).

Patterns are grouped by length in hash maps; each position is answered by one
lookup per distinct pattern length, longest first.
"""
from __future__ import annotations

import numpy as np


class PointOracle:
    def __init__(self, patterns):
        self.best = {}    # length -> {bytes: smallest id}
        self.count = {}   # length -> {bytes: number of ids}
        for k, p in enumerate(patterns, start=1):
            p = bytes(p)
            if len(p) == 0 or any(c not in b"ACGT" for c in p):
                raise ValueError("pattern %d is empty or holds a byte other than A,C,G,T" % (k - 1))
            L = len(p)
            d = self.best.setdefault(L, {})
            if p not in d:
                d[p] = k
            c = self.count.setdefault(L, {})
            c[p] = c.get(p, 0) + 1
        self.lengths = sorted(self.best, reverse=True)

    def at(self, text, i: int):
        """(match, count) for start position i of ``text`` (bytes-like)."""
        n = len(text)
        m = 0
        cnt = 0
        for L in self.lengths:
            if i + L > n:
                continue
            w = bytes(text[i:i + L])
            if m == 0:
                m = self.best[L].get(w, 0)
            cnt += self.count[L].get(w, 0)
        return m, cnt

    def many(self, text, positions):
        """Arrays (match int32, count int64) at every position in ``positions``."""
        t = bytes(np.asarray(text, dtype=np.uint8)) if not isinstance(text, (bytes, bytearray)) \
            else bytes(text)
        ms = np.zeros(len(positions), dtype=np.int32)
        cs = np.zeros(len(positions), dtype=np.int64)
        for j, i in enumerate(positions):
            ms[j], cs[j] = self.at(t, int(i))
        return ms, cs
