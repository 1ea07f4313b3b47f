"""Continuous-batching request server for PFAC matching.

Tables stay resident on the device.  Requests (one or many texts against one
table) arrive over time; the server admits a request when the device memory
it will hold fits an HBM budget, and dispatches admitted requests onto a
small pool of HIP streams: every dispatch is one batched call
(``pfac_match_batch``, one persistent launch per table and tile size) over
the requests waiting when a stream frees up, so work of requests admitted
while others run overlaps with theirs on the device.  A dispatch that holds
one request of a shape seen before reuses a prepared batch (layout, work
items and scratch built once, launch = kernels only).

Memory.  A request reserves what its dispatch allocates for it: the bytes of
its host texts (copied once, through pinned memory, 16-byte aligned), its
dense int32 outputs, its share of the hit buffer and counters.  Device texts
are read in place.  Results are views into the dispatch's buffers; the
reservation of a dispatch's requests is returned when the last of their
results is dropped, so what the server has admitted and not yet released is
an upper bound of the device memory its requests hold.

Texts are host arrays (the end-to-end path) or uint8 device tensors already
resident (the matching path alone).  Many small texts (a batch of reads) are
given as one ``TextBatch``: a buffer plus per-text offsets and lengths.
"""
from __future__ import annotations

import collections
import ctypes
import time
import weakref
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

try:                                   # 128-bit digests of request layouts
    import xxhash

    def _digest(a: np.ndarray) -> int:
        return xxhash.xxh3_128_intdigest(np.ascontiguousarray(a))
except ImportError:                    # pragma: no cover
    import hashlib

    def _digest(a: np.ndarray) -> int:
        return int.from_bytes(hashlib.blake2b(np.ascontiguousarray(a), digest_size=16).digest(),
                              "little")

from . import _lib as L
from .matcher import DESC_DTYPE, ENCODINGS, Batch, Table, match, match_batch, match_layout

ALIGN = 16
MAX_STREAMS = 4          # hardware queues per process on the target (HIP's default)


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


def _on_device(t) -> bool:
    return torch.is_tensor(t) and t.is_cuda


def hit_cap_of(lengths: np.ndarray) -> int:
    """Hit slots a dispatch gives a request of these text lengths."""
    return int(lengths.sum()) // 16 + 64 * int(lengths.size)


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
    ready: Optional[torch.cuda.Event] = None   # device texts: written by the submitter's stream
    # sizes derived from the texts, computed once (a request's texts do not
    # change while it is served)
    _memo: dict = field(default_factory=dict, repr=False, compare=False)

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
        if "lengths" not in self._memo:
            self._memo["lengths"] = np.array([_nbytes(t) for t in self.texts], dtype=np.int64)
        return self._memo["lengths"]

    @property
    def num_texts(self) -> int:
        return len(self.texts)

    def text(self, i: int):
        return self.texts.text(i) if isinstance(self.texts, TextBatch) else self.texts[i]

    @property
    def bases(self) -> int:
        if "bases" not in self._memo:
            self._memo["bases"] = int(self.lengths.sum())
        return self._memo["bases"]

    def host_text_bytes(self) -> int:
        """Bytes its host texts take once copied (16-byte aligned runs)."""
        total = 0
        for b, o, n in self.segments():
            if not _on_device(b) and o.size:
                total += (int((o + n).max()) - int(o.min()) + ALIGN - 1) // ALIGN * ALIGN
        return total

    def device_bytes(self) -> int:
        """What a dispatch allocates for the request: its copied host texts,
        its dense match arrays, its hit slots (12 bytes each) and counters."""
        if "device_bytes" not in self._memo:
            self._memo["device_bytes"] = self._device_bytes()
        return self._memo["device_bytes"]

    def _device_bytes(self) -> int:
        L_ = self.lengths
        padded = self.bases + int(((-L_) & 3).sum())     # runs padded to 4 elements
        cap = self.bases // 16 + 64 * int(L_.size)       # hit_cap_of(L_)
        return self.host_text_bytes() + 4 * padded + 12 * cap + 16 * (int(L_.size) + 1)


@dataclass
class RequestResult:
    match: torch.Tensor              # int32, the texts' dense outputs, each at its offset
    offsets: np.ndarray              # start of each text's run in `match`
    lengths: np.ndarray
    hits_all: torch.Tensor           # int32 (k, 3) rows of the dispatch: text, pos, pid
    first_text: int                  # dispatch index of the request's first text
    num_hits: np.ndarray             # per text
    occurrences: np.ndarray          # per text

    def text_match(self, i: int) -> torch.Tensor:
        o = int(self.offsets[i])
        return self.match[o:o + int(self.lengths[i])]

    @property
    def hits(self) -> torch.Tensor:
        """(k, 3) hits of the request: text index within the request, pos, pid."""
        if self.hits_all.shape[1] == 2:
            # a one-text launch: (pos, pid) rows of text 0
            z = torch.zeros((self.hits_all.shape[0], 1), dtype=self.hits_all.dtype,
                            device=self.hits_all.device)
            return torch.cat([z, self.hits_all], dim=1)
        h = self.hits_all.clone()
        h[:, 0] -= self.first_text
        return h


class Admission:
    """First-come first-served admission against a device-memory budget.
    Pure bookkeeping (no device calls): ``offer`` queues a request, ``admit``
    moves queued requests into service while their reservations fit, and
    ``release`` returns bytes (of a request, or an explicit amount)."""

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

    def reserve(self, nbytes: int):
        self.reserved += int(nbytes)

    def release(self, req: Optional["Request"] = None, nbytes: Optional[int] = None):
        self.reserved -= req.device_bytes() if req is not None else int(nbytes)
        assert self.reserved >= 0


class _Lease:
    """Live results of one dispatch; the last one dropped returns the
    dispatch's reservation."""

    def __init__(self, gate: Admission, nbytes: int, count: int):
        self.gate = gate
        self.nbytes = nbytes
        self.live = count

    def drop(self):
        self.live -= 1
        if self.live == 0:
            self.gate.release(nbytes=self.nbytes)


@dataclass
class _Dispatch:
    reqs: List[Request]
    stream_idx: int
    event: torch.cuda.Event
    counters_host: torch.Tensor
    match: Optional[torch.Tensor]
    hits: torch.Tensor
    counters: torch.Tensor
    first_text: List[int]
    match_offsets: np.ndarray
    lengths: np.ndarray
    args: tuple                      # what a retry with a larger hit buffer needs
    hold: list = field(default_factory=list)   # staging / device texts kept alive
    prepared: Optional["_Prepared"] = None     # the prepared batch it launched


class Server:
    """``streams`` HIP streams (at most 4, the hardware queues a process gets
    by default), one dispatch in flight per stream."""

    def __init__(self, tables: Sequence[Table], budget_bytes: int = 32 << 30,
                 streams: int = MAX_STREAMS, max_dispatch_bases: int = 64 << 20,
                 plan=None, device=None, keep_results: bool = True,
                 on_complete: Optional[Callable[[Request], None]] = None,
                 prepared_cache: int = 64, trace: bool = False,
                 single_min_bases: int = 4 << 20, alone_min_texts: int = 1000,
                 short_depth: int = 1):
        self.tables = list(tables)
        # a request of one text at least this long gets a launch of its own
        # (pfac_match: 2048-position tiles, its totals from the finish kernel)
        # instead of joining a batched launch, where the per-text reduction
        # of such a text is one wave's serial loop
        self.single_min_bases = int(single_min_bases)
        self.alone_min_texts = int(alone_min_texts)
        self._lib = L.lib()
        self._tabs = (ctypes.c_void_p * len(self.tables))(*[t.handle.value for t in self.tables])
        self.budget = int(budget_bytes)
        self.max_dispatch_bases = int(max_dispatch_bases)
        self.plan = plan
        self._plan = None
        if plan is not None:
            from .matcher import _plan_struct
            self._plan = _plan_struct(plan)
        self.device = torch.device(device or "cuda")
        if self.device.index is None:
            # an explicit index: torch resolves the current device on every
            # call that is given a device without one
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._dev = self.device.index
        n = max(1, min(int(streams), MAX_STREAMS))
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n)]
        # dispatches in flight per stream: a long one-text launch fills the
        # device by itself, so those go to stream 0 only, up to three queued
        # there (the next starts as the previous ends, no host round trip);
        # the other dispatches take the other streams, `short_depth` each
        self.busy = [0] * n
        self.depth = [3] + [max(1, int(short_depth))] * (n - 1)
        self.gate = Admission(budget_bytes)                      # arrived, not admitted
        self.admitted: collections.deque = collections.deque()  # admitted, not dispatched
        self.inflight: List[_Dispatch] = []
        self.done: List[Request] = []
        self.keep_results = keep_results
        self.on_complete = on_complete
        self.max_seen_inflight = 0
        self.dispatch_sizes: List[int] = []
        self.prepared_hits = 0
        self._events: List[torch.cuda.Event] = []
        self._prepared: "collections.OrderedDict" = collections.OrderedDict()
        self._prepared_cap = int(prepared_cache)
        # with `trace`, every dispatch's device interval: timing events recorded
        # on its stream right before its first and after its last kernel
        self.trace: Optional[List[tuple]] = [] if trace else None
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------ admission
    def submit(self, req: Request):
        """Queue a request.  Device texts must stay unchanged until it
        completes; the dispatch waits for the work the submitting stream has
        queued so far (the producer of those texts)."""
        for b, o, n in req.segments():
            if not o.size:
                continue
            end = o + n
            if int(end.max()) > _nbytes(b) and int(end[n > 0].max(initial=0)) > _nbytes(b):
                # (empty texts may sit anywhere)
                raise ValueError("request %d: a text runs past the end of its buffer" % req.rid)
            if torch.is_tensor(b) and (b.dtype != torch.uint8 or not b.is_contiguous()):
                raise TypeError("request %d: texts must be contiguous uint8" % req.rid)
        if any(_on_device(b) for b, _, _ in req.segments()):
            req.ready = torch.cuda.Event()
            req.ready.record(torch.cuda.current_stream(self._dev))
        self.gate.offer(req)

    def _admit(self):
        t = self.now()
        for r in self.gate.admit():
            r.admitted = t
            self.admitted.append(r)

    # ------------------------------------------------------------ dispatch
    def _texts(self, reqs, stream):
        """Per text of the dispatch: absolute device address; host texts are
        copied through one pinned buffer into one device buffer."""
        segs = [s for r in reqs for s in r.segments()]
        if len(segs) == 1 and _on_device(segs[0][0]):
            b, o, _ = segs[0]
            return o.view(np.uint64) + np.uint64(b.data_ptr()), [b]
        host = [(b, o, n) for b, o, n in segs if not _on_device(b)]
        hold = []
        dev_buf = None
        spans = {}
        if host:
            total, cur = 0, 0
            for i, (b, o, n) in enumerate(segs):
                if _on_device(b) or not o.size:
                    continue
                lo, hi = int(o.min()), int((o + n).max())
                spans[i] = (cur, lo, hi)
                cur += (hi - lo + ALIGN - 1) // ALIGN * ALIGN
            total = max(ALIGN, cur)
            staging = torch.empty(total, dtype=torch.uint8, pin_memory=True)
            sv = staging.numpy()
            for i, (dst, lo, hi) in spans.items():
                sv[dst:dst + hi - lo] = segs[i][0][lo:hi]
            dev_buf = torch.empty(total, dtype=torch.uint8, device=self.device)
            self._on_stream(stream, dev_buf.copy_, staging, non_blocking=True)
            hold += [staging, dev_buf]
        addrs = []
        for i, (b, o, n) in enumerate(segs):
            if _on_device(b):
                addrs.append(b.data_ptr() + o)
                hold.append(b)
            elif o.size:
                dst, lo, _ = spans[i]
                addrs.append(dev_buf.data_ptr() + dst + (o - lo))
            else:
                addrs.append(np.zeros(0, dtype=np.int64))
        return np.concatenate(addrs).astype(np.uint64), hold

    def _signature(self, r: Request, addrs: np.ndarray):
        base = int(addrs.min()) if addrs.size else 0
        rel = (addrs - np.uint64(base)).view(np.int64)
        L_ = r.lengths
        return (r.table, int(L_.size), _digest(L_), _digest(rel)), base, rel

    def _single(self, r: Request) -> bool:
        return r.num_texts == 1 and r.bases >= self.single_min_bases

    def _alone(self, r: Request) -> bool:
        """Many texts: dispatched on its own, so a request of a shape seen
        before reuses a prepared batch (launch = kernels only, no per-text
        host layout), which coalescing would forgo."""
        return r.num_texts >= self.alone_min_texts

    def _free(self, long_text: bool):
        """A stream that can take a dispatch of this kind, or None."""
        n = len(self.streams)
        lanes = [0] if (long_text or n == 1) else range(1, n)
        for si in lanes:
            if self.busy[si] < self.depth[si]:
                return si
        return None

    def _dispatch(self):
        """Start one dispatch from the head of the admitted queue; False when
        no stream can take it now."""
        if not self.admitted:
            return False
        big = self._single(self.admitted[0])
        si = self._free(big)
        pick = 0
        if si is None:
            if not big:
                return False
            # the long-text stream is full: a short request behind may go
            pick = next((i for i, q in enumerate(self.admitted) if not self._single(q)), None)
            si = None if pick is None else self._free(False)
            if si is None:
                return False
            big = False
        stream = self.streams[si]
        if big:
            self._dispatch_single(self.admitted.popleft(), si)
            return True
        r = self.admitted[pick]
        del self.admitted[pick]
        reqs = [r]
        bases = r.bases
        if not self._alone(r):
            # coalesce the short requests waiting behind it
            while self.admitted:
                h = self.admitted[0]
                if (self._single(h) or self._alone(h)
                        or bases + h.bases > self.max_dispatch_bases):
                    break
                reqs.append(self.admitted.popleft())
                bases += h.bases
        for r in reqs:
            if r.ready is not None:
                stream.wait_event(r.ready)
        addrs, hold = self._texts(reqs, stream)
        # a one-request dispatch of a shape seen before: its prepared batch,
        # with the layout arrays computed when it was made
        sig = b = None
        if len(reqs) == 1 and reqs[0].num_texts > 0:
            sig, base, rel = self._signature(reqs[0], addrs)
            b = self._instance(sig, si)
        if b is not None:
            lengths, tids, cap, match_offsets, extent = b.shape
            first, ntext = [0], int(lengths.size)
        else:
            first, lens, tids = [], [], []
            ntext = 0
            for r in reqs:
                first.append(ntext)
                ntext += r.num_texts
                lens.append(r.lengths)
                tids.append(np.full(r.num_texts, r.table, dtype=np.uint32))
            lengths = np.concatenate(lens).astype(np.int64)
            tids = np.concatenate(tids)
            cap = sum(hit_cap_of(r.lengths) for r in reqs)
            # each text's output starts at a multiple of 4 elements (16-byte stores)
            match_offsets = match_layout(lengths).astype(np.int64)
            extent = int(match_offsets[-1] + lengths[-1]) if ntext else 0
        dev = self.device
        mt = torch.empty(max(1, extent), dtype=torch.int32, device=dev)
        hits = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        counters = torch.empty(2 + 2 * ntext, dtype=torch.int64, device=dev)
        if self.trace is not None:
            ev_start = torch.cuda.Event(enable_timing=True)
            ev_start.record(stream)
        if b is not None:
            self._prepared.move_to_end(sig)
            self.prepared_hits += 1
            b.busy += 1
            b.si = si
            hold.append(b)              # kept until the launch completes, even if evicted
            rc = self._lib.pfac_batch_launch(b.handle, base, mt.data_ptr(), hits.data_ptr(),
                                             cap, counters.data_ptr(), stream.cuda_stream)
            L.check(rc, "pfac_batch_launch")
        else:
            base = int(addrs.min()) if ntext else 0
            descs = np.zeros(max(1, ntext), dtype=DESC_DTYPE)
            descs["text_offset"][:ntext] = addrs - np.uint64(base)
            descs["n"][:ntext] = lengths
            descs["match_offset"][:ntext] = match_offsets
            descs["table"][:ntext] = tids
            descs["enc"][:ntext] = ENCODINGS["ascii"]
            pl = ctypes.byref(self._plan) if self._plan is not None else None
            rc = self._lib.pfac_match_batch(
                ctypes.cast(self._tabs, ctypes.c_void_p), len(self.tables), descs.ctypes.data,
                ntext, base, mt.data_ptr(), hits.data_ptr(), cap, counters.data_ptr(), pl,
                stream.cuda_stream)
            L.check(rc, "pfac_match_batch")
            if sig is not None:
                self._prepare(sig, descs, ntext, (lengths, tids, cap, match_offsets, extent))
        if self.trace is not None:
            ev_end = torch.cuda.Event(enable_timing=True)
            ev_end.record(stream)
            self.trace.append((si, ev_start, ev_end, len(reqs)))
        host_c = torch.empty(counters.numel(), dtype=torch.int64, pin_memory=True)
        self._on_stream(stream, host_c.copy_, counters, non_blocking=True)
        ev = self._event()
        ev.record(stream)
        t = self.now()
        for r in reqs:
            r.dispatched = t
        self.busy[si] += 1
        # the tables this dispatch reads stay alive until it completes (a
        # table replaced meanwhile is freed after its last dispatch)
        hold.append(list(self.tables))
        self.inflight.append(_Dispatch(reqs, si, ev, host_c, mt, hits, counters, first,
                                       match_offsets, lengths, (addrs, tids, stream), hold, b))
        self.max_seen_inflight = max(self.max_seen_inflight, len(self.inflight))
        self.dispatch_sizes.append(len(reqs))
        return True

    def _dispatch_single(self, r: Request, si: int):
        """One long text: pfac_match on stream `si`, hits as (pos, pid) rows."""
        stream = self.streams[si]
        if r.ready is not None:
            stream.wait_event(r.ready)
        addrs, hold = self._texts([r], stream)
        n = int(r.lengths[0])
        cap = hit_cap_of(r.lengths)
        dev = self.device
        mt = torch.empty(max(1, n), dtype=torch.int32, device=dev)
        hits = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        counters = torch.empty(2, dtype=torch.int64, device=dev)
        if self.trace is not None:
            ev_start = torch.cuda.Event(enable_timing=True)
            ev_start.record(stream)
        pl = ctypes.byref(self._plan) if self._plan is not None else None
        addr = int(addrs[0])
        tab = self.tables[r.table]
        rc = self._lib.pfac_match(tab.handle, addr, n, ENCODINGS["ascii"], mt.data_ptr(),
                                  hits.data_ptr(), cap, counters.data_ptr(), pl,
                                  stream.cuda_stream)
        L.check(rc, "pfac_match")
        if self.trace is not None:
            ev_end = torch.cuda.Event(enable_timing=True)
            ev_end.record(stream)
            self.trace.append((si, ev_start, ev_end, 1))
        host_c = torch.empty(2, dtype=torch.int64, pin_memory=True)
        self._on_stream(stream, host_c.copy_, counters, non_blocking=True)
        ev = self._event()
        ev.record(stream)
        r.dispatched = self.now()
        self.busy[si] += 1
        hold.append(tab)
        self.inflight.append(_Dispatch([r], si, ev, host_c, mt, hits, counters, [0],
                                       np.zeros(1, dtype=np.int64), r.lengths.copy(),
                                       ("single", addr, stream, tab), hold))
        self.max_seen_inflight = max(self.max_seen_inflight, len(self.inflight))
        self.dispatch_sizes.append(1)

    def update_table(self, index: int, add: Sequence[bytes] = (),
                     remove_ids: Sequence[int] = ()) -> Table:
        """Replace table `index` by its update (patterns added and removed,
        built on the device; IDs stay stable).  Requests dispatched from now on
        use the new table; dispatches in flight finish on the old one."""
        new = self.tables[index].update(add=add, remove_ids=remove_ids)
        self.tables[index] = new
        self._tabs = (ctypes.c_void_p * len(self.tables))(*[t.handle.value for t in self.tables])
        for k in [k for k in self._prepared if k[0] == index]:
            del self._prepared[k]                 # prepared batches name the old table
        return new

    def _instance(self, sig, si: int) -> Optional["_Prepared"]:
        """A prepared batch of dispatch shape `sig` that stream `si` may
        launch now: one with no launch in flight, or whose launches in flight
        are on `si` (the stream orders them; a prepared batch's scratch is
        its own, so two streams must not run one at once)."""
        for b in self._prepared.get(sig, ()):
            if b.busy == 0 or b.si == si:
                return b
        return None

    def _prepare(self, sig, descs, ntext, shape):
        """Keep a prepared batch for a one-request dispatch shape (offsets
        relative to the request's first text), with the dispatch's layout
        arrays (`shape`: lengths, table indices, hit capacity, output
        offsets, output extent).  A shape gets one for each stream that runs
        such dispatches when it is first seen, so that it can be in flight on
        all of them at once without a later create (about 0.6 ms each, with
        allocations and a synchronisation)."""
        insts = self._prepared.setdefault(sig, [])
        want = max(1, len(self.streams) - 1)
        pl = ctypes.byref(self._plan) if self._plan is not None else None
        while len(insts) < want:
            h = ctypes.c_void_p()
            rc = self._lib.pfac_batch_create(ctypes.cast(self._tabs, ctypes.c_void_p),
                                             len(self.tables), descs.ctypes.data, ntext, pl,
                                             ctypes.byref(h))
            if rc != 0:
                break
            insts.append(_Prepared(self._lib, h, shape))
        while len(self._prepared) > self._prepared_cap:
            self._prepared.popitem(last=False)

    # ------------------------------------------------------------ completion
    def _finish(self, d: _Dispatch):
        c = d.counters_host.numpy()
        if isinstance(d.args[0], str):
            self._finish_single(d, c)
            return
        if d.prepared is not None:
            d.prepared.busy -= 1
        if c[0] > d.hits.shape[0]:
            # the hit buffer was too small: redo the dispatch with room for all
            addrs, tids, stream = d.args
            extra = 12 * (int(c[0]) + 64 - d.hits.shape[0])
            self.gate.reserve(extra)
            d.hits = torch.empty((int(c[0]) + 64, 3), dtype=torch.int32, device=self.device)
            base = int(addrs.min())
            descs = np.zeros(len(d.lengths), dtype=DESC_DTYPE)
            descs["text_offset"] = addrs - np.uint64(base)
            descs["n"] = d.lengths
            descs["match_offset"] = d.match_offsets
            descs["table"] = tids
            pl = ctypes.byref(self._plan) if self._plan is not None else None
            with torch.cuda.stream(stream):
                L.check(self._lib.pfac_match_batch(
                    ctypes.cast(self._tabs, ctypes.c_void_p), len(self.tables), descs.ctypes.data,
                    len(d.lengths), base, d.match.data_ptr(), d.hits.data_ptr(),
                    d.hits.shape[0], d.counters.data_ptr(), pl, stream.cuda_stream),
                    "pfac_match_batch")
            stream.synchronize()
            c = d.counters.cpu().numpy()
        else:
            extra = 0
        t = self.now()
        # per-text counts: views of this dispatch's own pinned counter buffer
        per_hits, per_occ = c[2::2], c[3::2]
        lease = _Lease(self.gate, sum(r.device_bytes() for r in d.reqs) + extra, len(d.reqs))
        h0 = 0
        one = len(d.reqs) == 1
        for r, f in zip(d.reqs, d.first_text):
            k = r.num_texts
            Lr = d.lengths[f:f + k]
            m0 = int(d.match_offsets[f]) if k else 0
            m1 = int(d.match_offsets[f + k - 1]) + int(Lr[-1]) if k else 0
            h1 = int(c[0]) if one else h0 + int(per_hits[f:f + k].sum())
            offs = d.match_offsets[f:f + k]
            res = RequestResult(d.match[m0:m1], offs - m0 if m0 else offs, Lr, d.hits[h0:h1], f,
                                per_hits[f:f + k], per_occ[f:f + k])
            h0 = h1
            weakref.finalize(res, lease.drop)
            r.completed = t
            r.ready = None
            if self.on_complete is not None:
                r.result = res
                self.on_complete(r)
            r.result = res if self.keep_results else None
            del res
            self.done.append(r)
        self.busy[d.stream_idx] -= 1

    def _finish_single(self, d: _Dispatch, c: np.ndarray):
        _, addr, stream, tab = d.args
        extra = 0
        if c[0] > d.hits.shape[0]:
            # the hit buffer was too small: again with room for every hit
            extra = 8 * (int(c[0]) + 64 - d.hits.shape[0])
            self.gate.reserve(extra)
            d.hits = torch.empty((int(c[0]) + 64, 2), dtype=torch.int32, device=self.device)
            pl = ctypes.byref(self._plan) if self._plan is not None else None
            n = int(d.lengths[0])
            with torch.cuda.stream(stream):
                L.check(self._lib.pfac_match(tab.handle, addr, n, ENCODINGS["ascii"],
                                             d.match.data_ptr(), d.hits.data_ptr(),
                                             d.hits.shape[0], d.counters.data_ptr(), pl,
                                             stream.cuda_stream), "pfac_match")
            stream.synchronize()
            c = d.counters.cpu().numpy()
        r = d.reqs[0]
        lease = _Lease(self.gate, r.device_bytes() + extra, 1)
        n = int(d.lengths[0])
        res = RequestResult(d.match[:n], np.zeros(1, dtype=np.int64), d.lengths.copy(),
                            d.hits[:int(c[0])], 0, np.array([c[0]]), np.array([c[1]]))
        weakref.finalize(res, lease.drop)
        r.completed = self.now()
        r.ready = None
        if self.on_complete is not None:
            r.result = res
            self.on_complete(r)
        r.result = res if self.keep_results else None
        del res
        self.done.append(r)
        self.busy[d.stream_idx] -= 1

    def _on_stream(self, stream, fn, *args, **kw):
        """fn(*args, **kw) with `stream` current on the server's device."""
        prev = torch.cuda.current_stream(self._dev)
        torch.cuda.set_stream(stream)
        try:
            return fn(*args, **kw)
        finally:
            torch.cuda.set_stream(prev)

    def _event(self) -> torch.cuda.Event:
        """A completion event from the pool (events of completed dispatches
        are recorded again)."""
        return self._events.pop() if self._events else torch.cuda.Event()

    def _complete(self):
        still = []
        for d in self.inflight:
            if d.event.query():
                self._finish(d)
                self._events.append(d.event)
            else:
                still.append(d)
        self.inflight = still

    def step(self):
        self._complete()
        self._admit()
        while self._dispatch():
            pass

    def idle(self) -> bool:
        return not (self.gate.queue or self.admitted or self.inflight)

    def device_intervals(self) -> List[tuple]:
        """With ``trace``: per dispatch (stream index, start ms, end ms,
        requests), times on the device clock from the earliest dispatch start,
        sorted by start.  Call once the dispatches have completed."""
        if not self.trace:
            return []
        torch.cuda.synchronize(self.device)
        ref = self.trace[0][1]
        rows = [(si, ref.elapsed_time(a), ref.elapsed_time(b), k) for si, a, b, k in self.trace]
        lo = min(r[1] for r in rows)
        out = [(si, a - lo, b - lo, k) for si, a, b, k in rows]
        return sorted(out, key=lambda x: x[1])

    # ------------------------------------------------------------ driver
    def run(self, requests: Sequence[Request], poll_s: float = 0.0) -> dict:
        """Feed requests at their arrival times (seconds from now) and serve
        until all complete.  Returns throughput and latency statistics.
        ``poll_s``: sleep between completion polls while dispatches run (0:
        yield only; a 20 us sleep, which the host stretches to about 60 us,
        measured 5-9 % less closed-loop capacity on the served workload)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = time.perf_counter()
        while pending or not self.idle():
            t = self.now()
            # arrived requests are queued up to a dispatch's worth of bases
            # between dispatch steps: a burst of arrivals does not hold the
            # device idle while all of it is queued (latency counts from
            # arrival anyway), and short requests still coalesce
            queued = 0
            while pending and pending[0].arrival <= t and queued < self.max_dispatch_bases:
                r = pending.popleft()
                self.submit(r)
                queued += r.bases
            self.step()
            if not pending and self.idle():
                break
            if self.gate.queue and not self.inflight and not self.admitted:
                # nothing runs and the next request does not fit: the budget
                # is held by results the caller still keeps
                raise RuntimeError("request %d cannot be admitted: %d of %d budget bytes are "
                                   "held by results not yet dropped"
                                   % (self.gate.queue[0].rid, self.gate.reserved, self.budget))
            if pending and pending[0].arrival <= self.now():
                continue                          # more arrivals to queue first
            if self.inflight and not any(d.event.query() for d in self.inflight):
                time.sleep(poll_s)
            elif not self.inflight and pending:
                time.sleep(min(poll_s, max(0.0, pending[0].arrival - self.now())))
        torch.cuda.synchronize()
        return summarize(self.done)


class _Prepared:
    """A prepared batch kept for a dispatch shape (its own scratch and
    layout; outputs are passed per launch)."""

    def __init__(self, lib, handle, shape):
        self._lib = lib
        self.handle = handle
        self.shape = shape
        self.busy = 0                  # launches in flight
        self.si = -1                   # stream of the last launch

    def __del__(self):
        try:
            if self.handle is not None and self.handle.value:
                self._lib.pfac_batch_free(self.handle)
        except Exception:
            pass


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
    another as they arrive, one launch per request -- ``pfac_match`` for a
    one-text request, one ``pfac_match_batch`` over a request's own texts
    otherwise -- host texts copied in, synchronised before the next request.
    No coalescing across requests, one stream."""
    device = torch.device(device or "cuda")
    done = []
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    for r in sorted(requests, key=lambda r: r.arrival):
        while clock() < r.arrival:
            time.sleep(20e-6)
        if r.num_texts == 1:
            t = r.text(0)
            dt = t if _on_device(t) else torch.from_numpy(np.ascontiguousarray(t)).to(device)
            match(tables[r.table], dt, plan=plan, hit_cap=hit_cap_of(r.lengths))
        else:
            (b, o, n), = r.segments() if isinstance(r.texts, TextBatch) else [(None, None, None)]
            if b is None:
                bufs = [np.asarray(x) if not _on_device(x) else x.cpu().numpy() for x in r.texts]
                o = np.concatenate([[0], np.cumsum([x.size for x in bufs])[:-1]])
                n = np.array([x.size for x in bufs])
                b = np.concatenate(bufs)
            base = b if _on_device(b) else torch.from_numpy(np.ascontiguousarray(b)).to(device)
            match_batch([tables[r.table]], base, o, n, plan=plan, hit_cap=hit_cap_of(n))
        torch.cuda.synchronize()
        r.completed = clock()
        done.append(r)
    return summarize(done)
