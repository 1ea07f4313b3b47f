"""Independent checkers used to pin the oracle (they share no code with it).

* ``brute``: the definition, pattern by pattern and position by position;
* ``kmer_check``: per distinct pattern length, a sorted table of 2-bit packed
  pattern keys, looked up with every text window of that length;
* ``read_golden``: parser for the fixtures under tests/golden/.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

_CODE = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _CODE[_c] = _i


def brute(patterns, text):
    """(match list, total) straight from the definition."""
    text = bytes(text)
    n = len(text)
    match = [0] * n
    best = [0] * n
    total = 0
    for i in range(n):
        for k, p in enumerate(patterns, start=1):
            if text.startswith(p, i):
                total += 1
                if len(p) > best[i]:
                    best[i] = len(p)
                    match[i] = k
    return match, total


def brute_pairs(patterns, text):
    """Every (start, pattern ID) pair with the pattern at that start, sorted
    by start, then pattern length, then ID."""
    text = bytes(text)
    out = []
    for i in range(len(text)):
        for k, p in enumerate(patterns, start=1):
            if text.startswith(p, i):
                out.append((i, len(p), k))
    out.sort()
    return [(i, k) for i, _, k in out]


def kmer_check(patterns, text):
    """(match int32[n], total) by per-length packed-key lookup."""
    t = np.asarray(np.frombuffer(bytes(text), dtype=np.uint8) if isinstance(text, (bytes, bytearray))
                   else text, dtype=np.uint8)
    n = t.size
    codes = _CODE[t]
    bad = codes == 255
    codes = np.where(bad, 0, codes).astype(np.uint64)
    by_len = {}
    for k, p in enumerate(patterns, start=1):
        by_len.setdefault(len(p), []).append((p, k))
    match = np.zeros(n, dtype=np.int32)
    total = 0
    if n == 0 or not by_len:
        return match, total
    Lmax = max(by_len)
    lo = np.zeros(n, dtype=np.uint64)
    hi = np.zeros(n, dtype=np.uint64)
    anybad = np.zeros(n, dtype=bool)
    for L in range(1, Lmax + 1):
        j = L - 1
        m = n - j  # windows of length L exist for i < n - j
        if m <= 0:
            break
        if j < 32:
            lo[:m] |= codes[j:j + m] << np.uint64(2 * j)
        else:
            hi[:m] |= codes[j:j + m] << np.uint64(2 * (j - 32))
        anybad[:m] |= bad[j:j + m]
        if L not in by_len:
            continue
        keys = {}
        for p, k in by_len[L]:
            c = [b"ACGT".index(x) for x in p]
            kl = sum(c[q] << (2 * q) for q in range(min(L, 32)))
            kh = sum(c[q] << (2 * (q - 32)) for q in range(32, L))
            key = (kh, kl)
            if key in keys:
                keys[key] = (keys[key][0], keys[key][1] + 1)
            else:
                keys[key] = (k, 1)
        if L <= 32:
            items = sorted(keys.items(), key=lambda a: a[0][1])
            kl = np.array([a[0][1] for a in items], dtype=np.uint64)
            ids = np.array([a[1][0] for a in items], dtype=np.int32)
            cnt = np.array([a[1][1] for a in items], dtype=np.int64)
            wl = lo[:m]
            pos = np.minimum(np.searchsorted(kl, wl), kl.size - 1)
            found = (kl[pos] == wl) & ~anybad[:m]
            fi = np.nonzero(found)[0]
            match[fi] = ids[pos[fi]]          # longer lengths come later and override
            total += int(cnt[pos[fi]].sum())
        else:
            # first 32 bases filter, then an exact lookup of the few candidates
            kl = np.unique(np.array([a[0][1] for a in keys.items()], dtype=np.uint64))
            cand = np.nonzero(np.isin(lo[:m], kl) & ~anybad[:m])[0]
            for i in cand:
                hit = keys.get((int(hi[i]), int(lo[i])))
                if hit is not None:
                    match[i] = hit[0]
                    total += hit[1]
    return match, total


def read_golden(name):
    out = {}
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            val = val.strip()
            if key.startswith("row"):
                rows[int(key[3:])] = [tuple(int(x) for x in cell.split(",")) for cell in val.split()]
            else:
                out[key] = val
    if rows:
        out["rows"] = [rows[i] for i in range(len(rows))]
    return out
