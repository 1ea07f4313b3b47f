"""Python binding of the PFAC matcher: tables, single-text and batched matching.

Every step of the matching runs in libpfac.so; this module only marshals
arguments (torch tensors supply device memory and streams).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

ENCODINGS = {"ascii": L.PFAC_TEXT_ASCII, "2bit": L.PFAC_TEXT_2BIT}

# numpy layout of pfac_text_desc (include/pfac.h)
DESC_DTYPE = np.dtype([("text_offset", "<u8"), ("n", "<u8"), ("match_offset", "<u8"),
                       ("table", "<u4"), ("enc", "<u4")])
assert DESC_DTYPE.itemsize == ctypes.sizeof(L.PfacTextDesc)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _plan_struct(plan) -> Optional[L.PfacPlan]:
    if plan is None:
        return None
    if isinstance(plan, L.PfacPlan):
        return plan
    p = L.PfacPlan()
    for k, v in dict(plan).items():
        setattr(p, k, int(v))
    return p


class Table:
    """Failure-less goto trie of a pattern set, resident on the current GPU.
    ``alphabet`` "dna": patterns over A, C, G, T (every other text byte stops a
    walk); "bytes": every byte value is a symbol (hash-compressed table,
    one-text ``match`` only)."""

    def __init__(self, patterns: Sequence[bytes], alphabet: str = "dna", on_device: bool = False,
                 ids: Optional[Sequence[int]] = None, _handle=None):
        if alphabet not in ("dna", "bytes"):
            raise ValueError("alphabet is 'dna' or 'bytes'")
        self.alphabet = alphabet
        if _handle is not None:
            self._h = _handle
            self._lib = L.lib()
            self._read_info()
            return
        pats = [bytes(p) for p in patterns]
        self.num_patterns = len(pats)
        bufs = [ctypes.create_string_buffer(p, max(1, len(p))) for p in pats]
        arr = (ctypes.c_void_p * max(1, len(pats)))()
        for i, b in enumerate(bufs):
            arr[i] = ctypes.addressof(b)
        lens = (ctypes.c_uint32 * max(1, len(pats)))(*[len(p) for p in pats])
        h = ctypes.c_void_p()
        bad = ctypes.c_int64(-1)
        if on_device:
            idarr = None if ids is None else (ctypes.c_int32 * max(1, len(pats)))(*[int(x) for x in ids])
            rc = L.lib().pfac_build_table_device(
                ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(lens, ctypes.c_void_p),
                ctypes.cast(idarr, ctypes.c_void_p) if idarr is not None else None, len(pats),
                ctypes.byref(h), ctypes.byref(bad))
        else:
            build = (L.lib().pfac_build_table_bytes if alphabet == "bytes"
                     else L.lib().pfac_build_table)
            rc = build(ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(lens, ctypes.c_void_p),
                       len(pats), ctypes.byref(h), ctypes.byref(bad))
        if rc != 0:
            e = L.PfacError(rc, "pfac_build_table")
            e.bad_index = bad.value
            raise e
        self._h = h
        self._lib = L.lib()
        self._read_info()

    def update(self, add: Sequence[bytes] = (), remove_ids: Sequence[int] = ()) -> "Table":
        """A new table (built on the device): these patterns minus the IDs in
        ``remove_ids``, plus ``add`` with new IDs from one above the largest.
        The new table's ``first_new_id`` is the first of those."""
        pats = [bytes(p) for p in add]
        bufs = [ctypes.create_string_buffer(p, max(1, len(p))) for p in pats]
        arr = (ctypes.c_void_p * max(1, len(pats)))()
        for i, b in enumerate(bufs):
            arr[i] = ctypes.addressof(b)
        lens = (ctypes.c_uint32 * max(1, len(pats)))(*[len(p) for p in pats])
        rem = (ctypes.c_int32 * max(1, len(remove_ids)))(*[int(x) for x in remove_ids])
        h = ctypes.c_void_p()
        first = ctypes.c_int32(0)
        rc = self._lib.pfac_table_update(self._h, ctypes.cast(arr, ctypes.c_void_p),
                                         ctypes.cast(lens, ctypes.c_void_p), len(pats),
                                         ctypes.cast(rem, ctypes.c_void_p), len(remove_ids),
                                         ctypes.byref(h), ctypes.byref(first))
        L.check(rc, "pfac_table_update")
        t = Table([], _handle=h)
        t.first_new_id = int(first.value)
        return t

    def blob(self) -> np.ndarray:
        """The table's device allocation as bytes (tests)."""
        n = ctypes.c_uint64(0)
        L.check(self._lib.pfac_table_blob(self._h, None, 0, ctypes.byref(n)), "pfac_table_blob")
        out = np.zeros(int(n.value), dtype=np.uint8)
        L.check(self._lib.pfac_table_blob(self._h, out.ctypes.data, out.size, ctypes.byref(n)),
                "pfac_table_blob")
        return out

    def _read_info(self):
        st = L.PfacTableStats()
        L.check(self._lib.pfac_table_info(self._h, ctypes.byref(st)), "pfac_table_info")
        self.num_patterns = int(st.num_patterns)
        self.num_states = int(st.num_states)
        self.max_len = int(st.max_len)
        self.min_len = int(st.min_len)
        self.max_depth_full = int(st.max_depth_full)
        self.device_bytes = int(st.device_bytes)
        self.states_to_depth = [int(x) for x in st.states_to_depth]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pfac_free_table(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def default_plan(self, n: int = 0, enc: str = "ascii") -> dict:
        p = L.PfacPlan()
        L.check(self._lib.pfac_default_plan(self._h, int(n), ENCODINGS[enc], ctypes.byref(p)),
                "pfac_default_plan")
        return p.as_dict()


@dataclass
class MatchResult:
    match: Optional[torch.Tensor]       # int32[n] or None
    hits: Optional[torch.Tensor]        # int32[hit_cap, 2] (pos, pid) or None
    counters: torch.Tensor              # int64[2]: number of hits, total occurrences

    def num_hits(self) -> int:
        return int(self.counters[0].item())

    def total(self) -> int:
        return int(self.counters[1].item())

    def hit_list(self) -> np.ndarray:
        """(k, 2) array of (position, pattern id), k = min(num_hits, hit_cap)."""
        k = min(self.num_hits(), 0 if self.hits is None else self.hits.shape[0])
        h = self.hits[:k].cpu().numpy().astype(np.int64)
        h[:, 0] &= 0xFFFFFFFF
        return h


def n_bases(text: torch.Tensor, enc: str) -> int:
    return int(text.numel()) if enc == "ascii" else 4 * int(text.numel())


def text_bytes(n, enc):
    """Bytes of a text of n bases in encoding ``enc`` (array-friendly)."""
    return n if enc == "ascii" else (n + 3) // 4


def check_match_args(n: int, text_numel: int, enc: str, out: Optional["MatchResult"] = None):
    """Raise ValueError when a one-text call would read past its text buffer or
    write past an output buffer given in ``out`` (checked before any launch)."""
    if enc not in ENCODINGS:
        raise ValueError("unknown encoding %r" % (enc,))
    if n < 0 or n >= 1 << 32:
        raise ValueError("n must be in [0, 2^32)")
    if text_bytes(n, enc) > text_numel:
        raise ValueError("n exceeds the text buffer")
    if out is None:
        return
    if out.match is not None and out.match.numel() < n:
        raise ValueError("out.match holds %d elements, the text has %d positions"
                         % (out.match.numel(), n))
    if out.hits is not None and (out.hits.dim() != 2 or out.hits.shape[1] != 2):
        raise ValueError("out.hits must have shape (cap, 2)")
    if out.counters.numel() < 2:
        raise ValueError("out.counters needs 2 elements")


def check_batch_extents(descs: np.ndarray, T: int, text_numel: int,
                        match_numel: Optional[int], hits_shape=None, counters_numel=None):
    """Raise ValueError when a batched call would read past ``text_base`` or
    write past ``match_out`` (offsets + lengths of every text), or when the
    hit or counter buffers have the wrong shape (checked before any launch)."""
    if T == 0:
        return
    d = descs[:T]
    n = d["n"].astype(np.int64)
    if np.any(n >= 1 << 32):
        raise ValueError("every text must have fewer than 2^32 bases")
    nb = np.where(d["enc"] == ENCODINGS["ascii"], n, (n + 3) // 4)
    live = n > 0
    if np.any(live) and int((d["text_offset"].astype(np.int64) + nb)[live].max()) > text_numel:
        raise ValueError("a text runs past the end of text_base")
    if match_numel is not None and np.any(live) and \
            int((d["match_offset"].astype(np.int64) + n)[live].max()) > match_numel:
        raise ValueError("a text's match array runs past the end of match_out")
    if hits_shape is not None and (len(hits_shape) != 2 or hits_shape[1] != 3):
        raise ValueError("hits must have shape (cap, 3)")
    if counters_numel is not None and counters_numel < 2 + 2 * T:
        raise ValueError("counters need 2 + 2 * num_texts elements")


def match(table: Table, text: torch.Tensor, n: Optional[int] = None, enc: str = "ascii",
          dense: bool = True, hits: bool = True, hit_cap: Optional[int] = None, plan=None,
          stream=None, out: Optional[MatchResult] = None, noalloc: bool = False) -> MatchResult:
    """Match one device text.  ``text`` is a uint8 CUDA tensor (ASCII bytes,
    or 2-bit packed with ``enc='2bit'`` and ``n`` bases).  Asynchronous on
    ``stream`` (default: the current torch stream).  ``noalloc`` calls the
    library's allocation-free entry point (fixed scratch inside the library;
    pass ``out`` too for a call that allocates nothing at all)."""
    if text.device.type != "cuda" or text.dtype != torch.uint8:
        raise TypeError("text must be a uint8 CUDA tensor")
    if not text.is_contiguous():
        raise ValueError("text must be contiguous")
    if n is None:
        n = n_bases(text, enc)
    check_match_args(int(n), int(text.numel()), enc, out)
    dev = text.device
    if out is None:
        m = torch.empty(n, dtype=torch.int32, device=dev) if dense else None
        cap = (n // 16 + 1024) if hit_cap is None else int(hit_cap)
        h = torch.empty((cap, 2), dtype=torch.int32, device=dev) if hits else None
        c = torch.empty(2, dtype=torch.int64, device=dev)
        out = MatchResult(m, h, c)
    p = _plan_struct(plan)
    fn = table._lib.pfac_match_noalloc if noalloc else table._lib.pfac_match
    rc = fn(
        table.handle, text.data_ptr(), int(n), ENCODINGS[enc],
        out.match.data_ptr() if out.match is not None else None,
        out.hits.data_ptr() if out.hits is not None else None,
        int(out.hits.shape[0]) if out.hits is not None else 0,
        out.counters.data_ptr(), ctypes.byref(p) if p is not None else None,
        _stream_handle(stream))
    L.check(rc, "pfac_match_noalloc" if noalloc else "pfac_match")
    return out


@dataclass
class AllResult:
    occ: Optional[torch.Tensor]          # int32[cap, 2] (pos, pid) or None
    counters: torch.Tensor               # int64[2]: positions with a match, total occurrences

    def total(self) -> int:
        return int(self.counters[1].item())

    def occurrences(self) -> np.ndarray:
        """(k, 2) array of (position, pattern id), k = min(total, cap): ascending
        position, then pattern length, then ID."""
        k = min(self.total(), 0 if self.occ is None else self.occ.shape[0])
        o = self.occ[:k].cpu().numpy().astype(np.int64)
        o[:, 0] &= 0xFFFFFFFF
        return o


def match_all(table: Table, text: torch.Tensor, n: Optional[int] = None, enc: str = "ascii",
              cap: Optional[int] = None, plan=None, stream=None) -> AllResult:
    """Every (position, pattern ID) occurrence in one device text, the
    sub-patterns PFAC's longest-only report skips included.  With ``cap``
    None the call is made twice when needed: once to count, again with room
    for every occurrence."""
    if text.device.type != "cuda" or text.dtype != torch.uint8 or not text.is_contiguous():
        raise TypeError("text must be a contiguous uint8 CUDA tensor")
    if n is None:
        n = n_bases(text, enc)
    check_match_args(int(n), int(text.numel()), enc)
    dev = text.device
    c = torch.empty(2, dtype=torch.int64, device=dev)
    p = _plan_struct(plan)
    want = int(n) // 64 + 1024 if cap is None else int(cap)
    for _ in range(2):
        occ = torch.empty((max(1, want), 2), dtype=torch.int32, device=dev)
        rc = table._lib.pfac_match_all(table.handle, text.data_ptr(), int(n), ENCODINGS[enc],
                                       occ.data_ptr(), want, c.data_ptr(),
                                       ctypes.byref(p) if p is not None else None,
                                       _stream_handle(stream))
        L.check(rc, "pfac_match_all")
        if cap is not None:
            break
        total = int(c[1].item())
        if total <= want:
            break
        want = total
    return AllResult(occ, c)


@dataclass
class BatchResult:
    match: Optional[torch.Tensor]        # int32, per-text arrays at match offsets
    hits: Optional[torch.Tensor]         # int32[hit_cap, 3] (text, pos, pid)
    counters: torch.Tensor               # int64[2 + 2T]
    match_offsets: np.ndarray            # per-text element offsets into ``match``

    def per_text(self):
        """(hits, occurrences) per text as numpy int64 arrays."""
        c = self.counters.cpu().numpy()
        return c[2::2], c[3::2]


def match_layout(lengths) -> np.ndarray:
    """Default element offsets of per-text dense outputs in one int32 array:
    back to back, each run starting at a multiple of 4 elements, so that every
    tile of a text writes its output with 16-byte stores."""
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.size == 0:
        return np.zeros(0, dtype=np.uint64)
    padded = (lengths + 3) // 4 * 4
    return np.concatenate([[0], np.cumsum(padded)[:-1]]).astype(np.uint64)


def _descriptors(offsets, lengths, table_index, enc, match_offsets):
    offsets = np.asarray(offsets, dtype=np.uint64)
    lengths = np.asarray(lengths, dtype=np.uint64)
    T = int(lengths.size)
    if table_index is None:
        table_index = np.zeros(T, dtype=np.uint32)
    table_index = np.asarray(table_index, dtype=np.uint32)
    encs = (np.full(T, ENCODINGS[enc], dtype=np.uint32) if isinstance(enc, str)
            else np.array([ENCODINGS[e] for e in enc], dtype=np.uint32))
    if match_offsets is None:
        match_offsets = match_layout(lengths)
    descs = np.zeros(max(1, T), dtype=DESC_DTYPE)
    if T:
        descs["text_offset"][:T] = offsets
        descs["n"][:T] = lengths
        descs["match_offset"][:T] = match_offsets
        descs["table"][:T] = table_index
        descs["enc"][:T] = encs
    return descs, T, int(lengths.sum()), np.asarray(match_offsets, dtype=np.uint64)


class Batch:
    """A batch prepared once (``pfac_batch_create``) and launched many times
    (``pfac_batch_launch``).  A launch only enqueues kernels, so it may run
    inside ``torch.cuda.graph`` capture.  Text sizes, offsets, tables and
    encodings are fixed here; ``launch`` writes into the output tensors made
    here (or given), which the caller reads after the stream has passed."""

    def __init__(self, tables: Sequence[Table], offsets, lengths, table_index=None,
                 enc="ascii", dense: bool = True, hits: bool = True,
                 hit_cap: Optional[int] = None, plan=None, device=None,
                 match_offsets=None):
        self.tables = list(tables)
        self._lib = self.tables[0]._lib
        self.descs, self.num_texts, total, self.match_offsets = _descriptors(
            offsets, lengths, table_index, enc, match_offsets)
        dev = torch.device(device or "cuda")
        self.text_extent, self.match_extent = _extents(self.descs, self.num_texts)
        self.match = (torch.empty(max(1, self.match_extent), dtype=torch.int32, device=dev)
                      if dense else None)
        self.hit_cap = (total // 16 + 1024) if hit_cap is None else int(hit_cap)
        self.hits = (torch.empty((self.hit_cap, 3), dtype=torch.int32, device=dev)
                     if hits else None)
        self.counters = torch.empty(2 + 2 * self.num_texts, dtype=torch.int64, device=dev)
        tabs = (ctypes.c_void_p * len(self.tables))(*[t.handle.value for t in self.tables])
        p = _plan_struct(plan)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            rc = self._lib.pfac_batch_create(
                ctypes.cast(tabs, ctypes.c_void_p), len(self.tables), self.descs.ctypes.data,
                self.num_texts, ctypes.byref(p) if p is not None else None, ctypes.byref(h))
        L.check(rc, "pfac_batch_create")
        self.handle = h

    def launch(self, text_base: torch.Tensor, stream=None) -> BatchResult:
        if text_base.dtype != torch.uint8 or not text_base.is_contiguous():
            raise TypeError("text_base must be a contiguous uint8 tensor")
        if int(text_base.numel()) < self.text_extent:
            raise ValueError("text_base holds %d bytes, the batch's texts reach %d"
                             % (text_base.numel(), self.text_extent))
        rc = self._lib.pfac_batch_launch(
            self.handle, text_base.data_ptr(),
            self.match.data_ptr() if self.match is not None else None,
            self.hits.data_ptr() if self.hits is not None else None,
            self.hit_cap if self.hits is not None else 0, self.counters.data_ptr(),
            _stream_handle(stream))
        L.check(rc, "pfac_batch_launch")
        return BatchResult(self.match, self.hits, self.counters, self.match_offsets)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.pfac_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _extents(descs: np.ndarray, T: int):
    """(bytes of the text base, int32 elements of the match base) the texts reach."""
    if T == 0:
        return 0, 0
    d = descs[:T]
    n = d["n"].astype(np.int64)
    live = n > 0
    if not np.any(live):
        return 0, 0
    nb = np.where(d["enc"] == ENCODINGS["ascii"], n, (n + 3) // 4)
    return (int((d["text_offset"].astype(np.int64) + nb)[live].max()),
            int((d["match_offset"].astype(np.int64) + n)[live].max()))


def match_batch(tables: Sequence[Table], text_base: torch.Tensor, offsets, lengths,
                table_index=None, enc="ascii", dense: bool = True, hits: bool = True,
                hit_cap: Optional[int] = None, plan=None, stream=None,
                match_out: Optional[torch.Tensor] = None,
                match_offsets=None) -> BatchResult:
    """Match many texts stored in one device buffer in one persistent launch.

    ``offsets`` are byte offsets of each text in ``text_base``, ``lengths``
    their base counts, ``table_index`` the table of each text (default 0),
    ``enc`` one encoding name or one per text."""
    descs, T, total, match_offsets = _descriptors(offsets, lengths, table_index, enc,
                                                  match_offsets)
    if text_base.dtype != torch.uint8 or not text_base.is_contiguous():
        raise TypeError("text_base must be a contiguous uint8 tensor")
    dev = text_base.device
    if dense and match_out is None:
        match_out = torch.empty(max(1, _extents(descs, T)[1]), dtype=torch.int32, device=dev)
    if dense and (match_out.dtype != torch.int32 or not match_out.is_contiguous()):
        raise TypeError("match_out must be a contiguous int32 tensor")
    check_batch_extents(descs, T, int(text_base.numel()),
                        int(match_out.numel()) if dense else None)
    cap = (total // 16 + 1024) if hit_cap is None else int(hit_cap)
    h = torch.empty((cap, 3), dtype=torch.int32, device=dev) if hits else None
    c = torch.empty(2 + 2 * T, dtype=torch.int64, device=dev)
    tabs = (ctypes.c_void_p * len(tables))(*[t.handle.value for t in tables])
    p = _plan_struct(plan)
    rc = tables[0]._lib.pfac_match_batch(
        ctypes.cast(tabs, ctypes.c_void_p), len(tables), descs.ctypes.data, T,
        text_base.data_ptr(), match_out.data_ptr() if dense else None,
        h.data_ptr() if h is not None else None, cap if h is not None else 0, c.data_ptr(),
        ctypes.byref(p) if p is not None else None, _stream_handle(stream))
    L.check(rc, "pfac_match_batch")
    return BatchResult(match_out if dense else None, h, c, match_offsets)
