"""Continuous-batching request server for PFAC matching.

Tables stay resident on the device.  Requests (one or many texts against one
table) arrive over time; the server admits a request when its device memory
fits an HBM budget, packs every admitted request that is not yet running into
one batched launch per dispatch (``pfac_match_batch``: one persistent launch
per table present), and keeps up to ``max_inflight`` dispatches queued on the
device so new requests join the next launch while earlier ones still run.
A request completes when the event recorded after its dispatch has passed;
its results are views into the dispatch's output buffers.

Texts are either host arrays (copied into a pinned staging buffer and then
to the device on the dispatch's stream: the end-to-end path) or device
tensors already resident (the matching path alone).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from .matcher import Table, match, match_batch

ALIGN = 16


@dataclass
class Request:
    rid: int
    table: int
    texts: list                      # host uint8 arrays, or device uint8 tensors
    arrival: float = 0.0             # seconds, relative to the server clock
    admitted: float = -1.0
    dispatched: float = -1.0
    completed: float = -1.0
    result: Optional["RequestResult"] = None

    @property
    def lengths(self) -> List[int]:
        return [int(t.numel() if torch.is_tensor(t) else t.size) for t in self.texts]

    @property
    def bases(self) -> int:
        return sum(self.lengths)

    def device_bytes(self) -> int:
        """What the request holds on the device while admitted: its texts
        (padded), its dense match arrays, its share of the hit buffer and
        counters."""
        L = self.lengths
        text = sum((x + ALIGN - 1) // ALIGN * ALIGN for x in L)
        return text + 4 * sum(L) + 12 * (sum(L) // 16 + 64) + 16 * (len(L) + 1)


@dataclass
class RequestResult:
    match: List[torch.Tensor]        # int32 per text (views into the dispatch buffer)
    hits: torch.Tensor               # int32 (k, 3): text index within the request, pos, pid
    num_hits: np.ndarray             # per text
    occurrences: np.ndarray          # per text


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
    dev_text: Optional[torch.Tensor]
    res_offsets: Optional[np.ndarray] = None


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
    def _dispatch(self):
        if not self.admitted or len(self.inflight) >= self.max_inflight:
            return
        reqs = []
        bases = 0
        while self.admitted and (not reqs or bases + self.admitted[0].bases <= self.max_dispatch_bases):
            r = self.admitted.popleft()
            reqs.append(r)
            bases += r.bases
        texts, tids, first = [], [], []
        for r in reqs:
            first.append(len(texts))
            texts += list(r.texts)
            tids += [r.table] * len(r.texts)
        lengths = np.array([int(t.numel() if torch.is_tensor(t) else t.size) for t in texts],
                           dtype=np.int64)
        padded = (lengths + ALIGN - 1) // ALIGN * ALIGN
        offsets = np.concatenate([[0], np.cumsum(padded)[:-1]]).astype(np.int64)
        total = int(padded.sum())
        staging = None
        shared = None
        if texts and all(torch.is_tensor(t) for t in texts):
            ptrs = {t.untyped_storage().data_ptr() for t in texts}
            if len(ptrs) == 1 and all(t.is_contiguous() and t.dtype == torch.uint8 for t in texts):
                shared = texts[0].untyped_storage()
        with torch.cuda.stream(self.stream):
            if shared is not None:
                # texts are views of one device buffer: match them in place
                dev = torch.empty(0, dtype=torch.uint8, device=self.device).set_(shared)
                offsets = np.array([t.storage_offset() for t in texts], dtype=np.int64)
            else:
                dev = torch.empty(max(ALIGN, total), dtype=torch.uint8, device=self.device)
            if shared is not None:
                pass
            elif texts and not torch.is_tensor(texts[0]):
                staging = torch.empty(max(ALIGN, total), dtype=torch.uint8, pin_memory=True)
                sv = staging.numpy()
                for t, o in zip(texts, offsets):
                    sv[o:o + t.size] = t
                dev.copy_(staging, non_blocking=True)
            else:
                for t, o in zip(texts, offsets):
                    dev[o:o + t.numel()].copy_(t, non_blocking=True)
            res = match_batch(self.tables, dev, offsets, lengths, table_index=tids,
                              plan=self.plan, stream=self.stream,
                              hit_cap=int(lengths.sum()) // 16 + 64 * len(texts))
            ev = torch.cuda.Event()
            ev.record(self.stream)
        t = self.now()
        for r in reqs:
            r.dispatched = t
        self.inflight.append(_Dispatch(reqs, ev, res, first, staging, dev, offsets))
        self.max_seen_inflight = max(getattr(self, "max_seen_inflight", 0), len(self.inflight))
        self.dispatch_sizes = getattr(self, "dispatch_sizes", []) + [len(reqs)]

    # ------------------------------------------------------------ completion
    def _complete(self):
        while self.inflight and self.inflight[0].event.query():
            d = self.inflight.popleft()
            t = self.now()
            counters = d.res.counters.cpu().numpy()
            if d.res.hits is not None and counters[0] > d.res.hits.shape[0]:
                # the hit buffer was too small: redo this dispatch with room for all
                with torch.cuda.stream(self.stream):
                    lengths = [n for r in d.reqs for n in r.lengths]
                    offs = d.res_offsets
                    tids = [r.table for r in d.reqs for _ in r.texts]
                    d.res = match_batch(self.tables, d.dev_text, offs, lengths,
                                        table_index=tids, plan=self.plan, stream=self.stream,
                                        hit_cap=int(counters[0]) + 64)
                self.stream.synchronize()
                counters = d.res.counters.cpu().numpy()
            per_hits, per_occ = counters[2::2], counters[3::2]
            hit_start = np.concatenate([[0], np.cumsum(per_hits)]).astype(np.int64)
            for r, f in zip(d.reqs, d.first_text):
                k = len(r.texts)
                mats = [d.res.match[int(d.res.match_offsets[f + i]):
                                    int(d.res.match_offsets[f + i]) + r.lengths[i]]
                        for i in range(k)]
                h0, h1 = int(hit_start[f]), int(hit_start[f + k])
                h = d.res.hits[h0:h1].clone()
                h[:, 0] -= f
                r.result = RequestResult(mats, h, per_hits[f:f + k].copy(), per_occ[f:f + k].copy())
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
        for t in r.texts:
            dt = t if torch.is_tensor(t) else torch.from_numpy(t).to(device)
            match(tables[r.table], dt, plan=plan, hit_cap=int(dt.numel()) // 16 + 64)
        torch.cuda.synchronize()
        r.completed = clock()
        done.append(r)
    return summarize(done)
