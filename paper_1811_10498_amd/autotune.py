"""Launch-plan autotuner.

A plan (threads per workgroup, filter depth D, trie levels kept in LDS, size
of the second filter, walks at once or deferred) never changes results, only
speed.  The tuner times every candidate plan the
library accepts on a sample of the caller's own text and keeps the fastest,
cached per (table, encoding, size class).  Timing uses HIP events on the
current stream.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import torch

from . import _lib as L
from .matcher import Table, match, n_bases

BLOCKS = (256, 512, 768, 1024)
DEPTHS = (7, 8, 9, 10)
LEVELS = (0, L.PFAC_LEVELS_NONE)
HASHES = (0, L.PFAC_HASH_NONE)
# library choice (deferred behind the second filter when patterns fit the
# copied window) or at once: which is faster depends on how many windows the
# text lets through, which only the text shows
WALKS = (0, L.PFAC_WALKS_INLINE)


def candidate_plans(blocks=BLOCKS, depths=DEPTHS, levels=LEVELS, hashes=HASHES,
                    walks=WALKS) -> List[dict]:
    out = []
    for b in blocks:
        for d in depths:
            for lv in levels:
                for hb in hashes:
                    for wk in walks:
                        if hb == L.PFAC_HASH_NONE and wk != 0:
                            continue            # without the filter walks are at once
                        out.append(dict(block=b, depth=d, levels=lv, hash_bits=hb, walks=wk))
    return out


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
    def key(table: Table, enc: str, n: int) -> str:
        return "%d:%d:%d:%d:%s:%d" % (table.num_states, table.num_patterns, table.min_len,
                                      table.max_len, enc, size_class(n))

    def _time(self, table, text, n, enc, plan) -> Optional[float]:
        try:
            r = match(table, text, n=n, enc=enc, plan=plan, hits=True)
        except L.PfacError:
            return None                      # plan does not fit this device / table
        torch.cuda.synchronize()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(self.reps):
            match(table, text, n=n, enc=enc, plan=plan, out=r)
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / self.reps

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
        for plan in candidates or candidate_plans():
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

    def _save(self):
        if not self.cache_path:
            return
        tmp = self.cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({k: {"plan": v.plan, "ms": v.ms} for k, v in self.cache.items()}, f)
        os.replace(tmp, self.cache_path)
