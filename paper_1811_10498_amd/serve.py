"""Continuous-batching request server for PFAC matching.

Tables stay resident on the device.  Requests (one or many texts against one
table) arrive over time; the server admits a request when its device memory
fits an HBM budget, packs every admitted request that is not yet running into
one batched launch per dispatch (``pfac_match_batch``: one persistent launch
per table present), and keeps up to ``max_inflight`` dispatches queued on the
device so new requests join the next launch while earlier ones still run.
A request completes when the event recorded after its dispatch has passed;
its results are views into the dispatch's output buffers.

Texts are host arrays (copied through a pinned staging buffer to the device
on the dispatch's stream: the end-to-end path) or device tensors already
resident (the matching path alone).  Many small texts (a batch of reads) are
given as one ``TextBatch``: a buffer plus per-text offsets and lengths, so a
request of 10,000 reads costs a few array operations, not 10,000 Python
objects.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from .matcher import Table, match, match_batch

ALIGN = 16


@dataclass
class TextBatch:
    """Many texts inside one uint8 buffer (host array or device tensor)."""
    base: object                     # np.ndarray or torch.Tensor (uint8)
    offsets: np.ndarray              # byte offset of each text in `base`
    lengths: np.ndarray              # bases of each text

    def __post_init__(self):
        self.offsets = np.asarray(self.offsets, dtype=np.int64)
        self.lengths = np.asarray(self.lengths, dtype=np.int64)

    def __len__(self) -> int:
        return int(self.lengths.size)

    def text(self, i: int):
        o, n = int(self.offsets[i]), int(self.lengths[i])
        return self.base[o:o + n]


def _nbytes(t) -> int:
    return int(t.numel() if torch.is_tensor(t) else t.size)


@dataclass
class Request:
    rid: int
    table: int
    texts: object                    # list of host arrays / device tensors, or a TextBatch
    arrival: float = 0.0             # seconds, relative to the server clock
    admitted: float = -1.0
    dispatched: float = -1.0
    completed: float = -1.0
    result: Optional["RequestResult"] = None

    def segments(self):
        """(buffer, offsets, lengths) runs of the request's texts, in order."""
        if isinstance(self.texts, TextBatch):
            return [(self.texts.base, self.texts.offsets, self.texts.lengths)]
        return [(t, np.zeros(1, dtype=np.int64), np.array([_nbytes(t)], dtype=np.int64))
                for t in self.texts]

    @property
    def lengths(self) -> np.ndarray:
        if isinstance(self.texts, TextBatch):
            return self.texts.lengths
        return np.array([_nbytes(t) for t in self.texts], dtype=np.int64)

    @property
    def num_texts(self) -> int:
        return len(self.texts)

    def text(self, i: int):
        return self.texts.text(i) if isinstance(self.texts, TextBatch) else self.texts[i]

    @property
    def bases(self) -> int:
        return int(self.lengths.sum())

    def device_bytes(self) -> int:
        """What the request holds on the device while admitted: its texts
        (padded), its dense match arrays, its share of the hit buffer and
        counters."""
        L = self.lengths
        text = int(((L + ALIGN - 1) // ALIGN * ALIGN).sum())
        total = int(L.sum())
        return text + 4 * total + 12 * (total // 16 + 64) + 16 * (L.size + 1)


@dataclass
class RequestResult:
    match: torch.Tensor              # int32, the texts' dense outputs back to back
    offsets: np.ndarray              # start of each text's run in `match`
    lengths: np.ndarray
    hits: torch.Tensor               # int32 (k, 3): text index within the request, pos, pid
    num_hits: np.ndarray             # per text
    occurrences: np.ndarray          # per text

    def text_match(self, i: int) -> torch.Tensor:
        o = int(self.offsets[i])
        return self.match[o:o + int(self.lengths[i])]


class Admission:
    """First-come first-served admission against a device-memory budget.
    Pure bookkeeping (no device calls): ``offer`` queues a request, ``admit``
    moves queued requests into service while their reservations fit, and
    ``release`` returns a finished request's bytes."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.reserved = 0
        self.queue: collections.deque = collections.deque()

    def offer(self, req: "Request"):
        need = req.device_bytes()
        if need > self.budget:
            raise ValueError("request %d needs %d bytes, above the %d-byte budget"
                             % (req.rid, need, self.budget))
        self.queue.append(req)

    def admit(self) -> List["Request"]:
        out = []
        while self.queue:
            need = self.queue[0].device_bytes()
            if self.reserved + need > self.budget:
                break
            r = self.queue.popleft()
            self.reserved += need
            out.append(r)
        return out

    def release(self, req: "Request"):
        self.reserved -= req.device_bytes()
        assert self.reserved >= 0


@dataclass
class _Dispatch:
    reqs: List[Request]
    event: torch.cuda.Event
    res: object
    first_text: List[int]
    staging: Optional[torch.Tensor]
    dev_text: torch.Tensor
    offsets: np.ndarray
    lengths: np.ndarray
    tids: np.ndarray


class Server:
    def __init__(self, tables: Sequence[Table], budget_bytes: int = 32 << 30,
                 max_inflight: int = 2, max_dispatch_bases: int = 512 << 20,
                 plan=None, device=None):
        self.tables = list(tables)
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.max_dispatch_bases = int(max_dispatch_bases)
        self.plan = plan
        self.device = torch.device(device or "cuda")
        self.stream = torch.cuda.Stream(device=self.device)
        self.gate = Admission(budget_bytes)                      # arrived, not admitted
        self.admitted: collections.deque = collections.deque()  # admitted, not dispatched
        self.inflight: collections.deque = collections.deque()
        self.done: List[Request] = []
        self.max_seen_inflight = 0
        self.dispatch_sizes: List[int] = []
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------ admission
    def submit(self, req: Request):
        self.gate.offer(req)

    def _admit(self):
        t = self.now()
        for r in self.gate.admit():
            r.admitted = t
            self.admitted.append(r)

    # ------------------------------------------------------------ dispatch
    def _place(self, segs):
        """Device buffer and per-text byte offsets for the dispatch's texts:
        in place when every text already lives in one device allocation,
        else copied (host texts through pinned staging), each run of texts
        as one copy at a 16-byte aligned destination."""
        bufs = [b for b, _, _ in segs]
        if all(torch.is_tensor(b) and b.is_cuda and b.dtype == torch.uint8 and b.is_contiguous()
               for b in bufs):
            if len({b.untyped_storage().data_ptr() for b in bufs}) == 1:
                dev = torch.empty(0, dtype=torch.uint8, device=self.device).set_(
                    bufs[0].untyped_storage())
                offs = np.concatenate([b.storage_offset() + o for b, o, _ in segs])
                return dev, offs, None
        spans, cur = [], 0
        for b, o, L in segs:
            lo = int(o.min()) if o.size else 0
            hi = int((o + L).max()) if o.size else 0
            spans.append((cur, lo, hi))
            cur += (hi - lo + ALIGN - 1) // ALIGN * ALIGN
        total = max(ALIGN, cur)
        dev = torch.empty(total, dtype=torch.uint8, device=self.device)
        staging = None
        if any(not torch.is_tensor(b) for b in bufs):
            # host runs: fill a pinned buffer, one host-to-device copy
            staging = torch.empty(total, dtype=torch.uint8, pin_memory=True)
            sv = staging.numpy()
            for b, (dst, lo, hi) in zip(bufs, spans):
                if not torch.is_tensor(b) and hi > lo:
                    sv[dst:dst + hi - lo] = b[lo:hi]
            dev.copy_(staging, non_blocking=True)
        # device runs: copied after it on the same stream
        for b, (dst, lo, hi) in zip(bufs, spans):
            if torch.is_tensor(b) and hi > lo:
                dev[dst:dst + hi - lo].copy_(b[lo:hi], non_blocking=True)
        offs = np.concatenate([dst + (o - lo) for (_, o, _), (dst, lo, _) in zip(segs, spans)])
        return dev, offs, staging

    def _dispatch(self):
        if not self.admitted or len(self.inflight) >= self.max_inflight:
            return
        reqs = []
        bases = 0
        while self.admitted and (not reqs or bases + self.admitted[0].bases <= self.max_dispatch_bases):
            r = self.admitted.popleft()
            reqs.append(r)
            bases += r.bases
        segs, tids, first = [], [], []
        ntext = 0
        for r in reqs:
            first.append(ntext)
            for s in r.segments():
                segs.append(s)
                ntext += int(s[2].size)
            tids.append(np.full(r.num_texts, r.table, dtype=np.uint32))
        lengths = np.concatenate([s[2] for s in segs]).astype(np.int64)
        tids = np.concatenate(tids)
        with torch.cuda.stream(self.stream):
            dev, offsets, staging = self._place(segs)
            res = match_batch(self.tables, dev, offsets, lengths, table_index=tids,
                              plan=self.plan, stream=self.stream,
                              hit_cap=int(lengths.sum()) // 16 + 64 * ntext)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        t = self.now()
        for r in reqs:
            r.dispatched = t
        self.inflight.append(_Dispatch(reqs, ev, res, first, staging, dev, offsets, lengths,
                                       tids))
        self.max_seen_inflight = max(self.max_seen_inflight, len(self.inflight))
        self.dispatch_sizes.append(len(reqs))

    # ------------------------------------------------------------ completion
    def _complete(self):
        while self.inflight and self.inflight[0].event.query():
            d = self.inflight.popleft()
            t = self.now()
            counters = d.res.counters.cpu().numpy()
            if d.res.hits is not None and counters[0] > d.res.hits.shape[0]:
                # the hit buffer was too small: redo this dispatch with room for all
                with torch.cuda.stream(self.stream):
                    d.res = match_batch(self.tables, d.dev_text, d.offsets, d.lengths,
                                        table_index=d.tids, plan=self.plan, stream=self.stream,
                                        hit_cap=int(counters[0]) + 64)
                self.stream.synchronize()
                counters = d.res.counters.cpu().numpy()
            per_hits, per_occ = counters[2::2], counters[3::2]
            hit_start = np.concatenate([[0], np.cumsum(per_hits)]).astype(np.int64)
            mo = np.asarray(d.res.match_offsets, dtype=np.int64)
            for r, f in zip(d.reqs, d.first_text):
                k = r.num_texts
                L = d.lengths[f:f + k]
                m0 = int(mo[f]) if k else 0
                mats = d.res.match[m0:m0 + int(L.sum())]
                h0, h1 = int(hit_start[f]), int(hit_start[f + k])
                h = d.res.hits[h0:h1].clone()
                h[:, 0] -= f
                r.result = RequestResult(mats, mo[f:f + k] - m0, L, h,
                                         per_hits[f:f + k].copy(), per_occ[f:f + k].copy())
                r.completed = t
                self.gate.release(r)
                self.done.append(r)

    def step(self):
        self._complete()
        self._admit()
        self._dispatch()

    def idle(self) -> bool:
        return not (self.gate.queue or self.admitted or self.inflight)

    # ------------------------------------------------------------ driver
    def run(self, requests: Sequence[Request], poll_s: float = 50e-6) -> dict:
        """Feed requests at their arrival times (seconds from now) and serve
        until all complete.  Returns throughput and latency statistics."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = time.perf_counter()
        while pending or not self.idle():
            t = self.now()
            while pending and pending[0].arrival <= t:
                self.submit(pending.popleft())
            self.step()
            if not pending and self.idle():
                break
            if not self.inflight or not self.inflight[0].event.query():
                time.sleep(poll_s)
        torch.cuda.synchronize()
        return summarize(self.done)


def summarize(done: Sequence[Request]) -> dict:
    if not done:
        return {"requests": 0}
    lat = np.array([r.completed - r.arrival for r in done])
    bases = sum(r.bases for r in done)
    span = max(r.completed for r in done) - min(r.arrival for r in done)
    return {
        "requests": len(done),
        "bases": int(bases),
        "wall_s": float(span),
        "gbases_per_s": float(bases / span / 1e9) if span > 0 else float("nan"),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
    }


def plain_per_request(tables: Sequence[Table], requests: Sequence[Request], device=None,
                      plan=None) -> dict:
    """The baseline the server is compared with: requests handled one after
    another, each text with its own single-text ``pfac_match`` call, copied
    in and synchronised before the next request."""
    device = torch.device(device or "cuda")
    done = []
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    for r in sorted(requests, key=lambda r: r.arrival):
        while clock() < r.arrival:
            time.sleep(50e-6)
        for i in range(r.num_texts):
            t = r.text(i)
            dt = t if torch.is_tensor(t) else torch.from_numpy(np.ascontiguousarray(t)).to(device)
            match(tables[r.table], dt, plan=plan, hit_cap=int(dt.numel()) // 16 + 64)
        torch.cuda.synchronize()
        r.completed = clock()
        done.append(r)
    return summarize(done)
