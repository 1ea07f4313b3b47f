"""Launch-plan autotuner for one-text and batched calls.

A plan (threads per workgroup, filter depth D, trie levels kept in LDS, size
of the hashed second filter, the exact prefix filter, walks at once or
deferred, positions per tile) never changes results, only speed.  The tuner
times the candidate plans the library accepts on a sample of the caller's
own input and keeps the fastest, cached per (table, encoding, size class) for
one-text calls and per (table, batch shape class) for batches.  Timing uses
HIP events on the current stream; a batch is timed as a prepared batch (one
launch = its kernels only).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from .matcher import Batch, Table, match, n_bases

BLOCKS = (256, 512, 768, 1024)
DEPTHS = (7, 8, 9, 10)
LEVELS = (0, L.PFAC_LEVELS_NONE)
HASHES = (0, L.PFAC_HASH_NONE, 19, 20)
PREFIXES = (0, 1, L.PFAC_PREFIX_NONE)
# library choice (deferred behind a filter when patterns fit the copied
# window) or at once: which is faster depends on how many windows the text
# lets through, which only the text shows
WALKS = (0, L.PFAC_WALKS_INLINE)
TILES_ONE = (2048, 1024)
TILES_BATCH = (0, 1024, 2048, 256)


def candidate_plans(blocks=BLOCKS, depths=DEPTHS, levels=LEVELS, hashes=HASHES,
                    walks=WALKS, prefixes=PREFIXES, tiles=TILES_ONE) -> List[dict]:
    out = []
    for b in blocks:
        for d in depths:
            for lv in levels:
                for hb in hashes:
                    for pf in prefixes:
                        for wk in walks:
                            if hb == L.PFAC_HASH_NONE and pf == L.PFAC_PREFIX_NONE and wk != 0:
                                continue        # without filters walks are at once
                            if lv != L.PFAC_LEVELS_NONE and hb not in (0, L.PFAC_HASH_NONE):
                                continue        # explicit hash sizes go with the bare bitmap
                            for t in tiles:
                                out.append(dict(block=b, depth=d, levels=lv, hash_bits=hb,
                                                prefix=pf, walks=wk, tile=t))
    return out


def focused_plans(table: Table, batch: bool = False) -> List[dict]:
    """A short candidate list around the library's choice: the default, its
    neighbours in depth and workgroup size, each filter on and off, and the
    other tile sizes."""
    base = table.default_plan()
    tiles = TILES_BATCH if batch else TILES_ONE
    out = [dict()]
    for t in tiles:
        out.append(dict(tile=t))
    for w in (L.PFAC_WALKS_INLINE, L.PFAC_WALKS_DEFERRED):
        out.append(dict(walks=w))
    for hb in (L.PFAC_HASH_NONE, 18, 19, 20):
        for pf in (1, L.PFAC_PREFIX_NONE):
            out.append(dict(depth=base["depth"], hash_bits=hb, prefix=pf))
    for d in (base["depth"] - 1, base["depth"] + 1):
        if 6 <= d <= 10:
            out.append(dict(depth=d))
            out.append(dict(depth=d, block=512))
    for b in (512, 768):
        out.append(dict(block=b))
    out.append(dict(levels=0, hash_bits=L.PFAC_HASH_NONE))
    seen, uniq = set(), []
    for p in out:
        k = tuple(sorted(p.items()))
        if k not in seen:
            seen.add(k)
            uniq.append(p)
    return uniq


def size_class(n: int) -> int:
    """Texts within a factor of 4 share a tuning result."""
    c = 0
    while n >= 4 ** (c + 1) * 65536:
        c += 1
    return c


@dataclass
class TuneResult:
    plan: dict
    ms: float
    tried: List[Tuple[dict, float]] = field(default_factory=list)


def _timed(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


class Autotuner:
    def __init__(self, cache_path: Optional[str] = None, reps: int = 3,
                 sample_bases: int = 128 << 20):
        self.cache: Dict[str, TuneResult] = {}
        self.cache_path = cache_path
        self.reps = reps
        self.sample_bases = sample_bases
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                for k, v in json.load(f).items():
                    self.cache[k] = TuneResult(v["plan"], v["ms"])

    @staticmethod
    def _table_key(table: Table) -> str:
        return "%d:%d:%d:%d" % (table.num_states, table.num_patterns, table.min_len,
                                table.max_len)

    @staticmethod
    def key(table: Table, enc: str, n: int) -> str:
        return "%s:%s:%d" % (Autotuner._table_key(table), enc, size_class(n))

    @staticmethod
    def batch_key(tables: Sequence[Table], lengths: np.ndarray) -> str:
        lengths = np.asarray(lengths, dtype=np.int64)
        med = int(np.median(lengths)) if lengths.size else 0
        return "batch:%s:%d:%d:%d" % ("+".join(Autotuner._table_key(t) for t in tables),
                                      size_class(int(lengths.sum())), size_class(med * 64),
                                      int(np.mean(lengths <= 512) * 4) if lengths.size else 0)

    def _time(self, table, text, n, enc, plan) -> Optional[float]:
        try:
            r = match(table, text, n=n, enc=enc, plan=plan, hits=True)
        except L.PfacError:
            return None                      # plan does not fit this device / table
        return _timed(lambda: match(table, text, n=n, enc=enc, plan=plan, out=r), self.reps)

    def tune(self, table: Table, text: torch.Tensor, n: Optional[int] = None,
             enc: str = "ascii", candidates: Optional[List[dict]] = None) -> TuneResult:
        n = n_bases(text, enc) if n is None else n
        k = self.key(table, enc, n)
        if k in self.cache:
            return self.cache[k]
        sample = min(n, self.sample_bases)
        if enc == "2bit":
            sample -= sample % 4
            view = text[: (sample + 3) // 4]
        else:
            view = text[:sample]
        best = None
        tried = []
        for plan in candidates or focused_plans(table):
            ms = self._time(table, view, sample, enc, plan)
            if ms is None:
                continue
            tried.append((plan, ms))
            if best is None or ms < best[1]:
                best = (plan, ms)
        if best is None:
            best = (table.default_plan(n, enc), float("nan"))
        res = TuneResult(best[0], best[1], tried)
        self.cache[k] = res
        self._save()
        return res

    def tune_batch(self, tables: Sequence[Table], text_base: torch.Tensor, offsets, lengths,
                   table_index=None, enc="ascii",
                   candidates: Optional[List[dict]] = None) -> TuneResult:
        """The fastest plan for a batch of this shape, timed as prepared
        launches of the caller's own batch (every plan gives the same result)."""
        k = self.batch_key(tables, lengths)
        if k in self.cache:
            return self.cache[k]
        best = None
        tried = []
        for plan in candidates or focused_plans(tables[0], batch=True):
            try:
                b = Batch(tables, offsets, lengths, table_index=table_index, enc=enc, plan=plan,
                          device=text_base.device)
            except L.PfacError:
                continue
            try:
                ms = _timed(lambda: b.launch(text_base), self.reps)
            finally:
                b.close()
            tried.append((plan, ms))
            if best is None or ms < best[1]:
                best = (plan, ms)
        if best is None:
            best = (dict(), float("nan"))
        res = TuneResult(best[0], best[1], tried)
        self.cache[k] = res
        self._save()
        return res

    def _save(self):
        if not self.cache_path:
            return
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({k: {"plan": v.plan, "ms": v.ms} for k, v in self.cache.items()}, f)
        os.replace(tmp, self.cache_path)
