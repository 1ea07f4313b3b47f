"""Helpers of the GPU parity tests: the oracle over many texts at once, and
the check of a batched result against it, text by text."""
import numpy as np

import oracle

SEP = np.frombuffer(b"N", dtype=np.uint8)


def joined_oracle(patterns, texts, threads=16):
    """Per text (match array, occurrence total) from one oracle scan over the
    texts joined by a non-base byte (no walk crosses it)."""
    parts, starts = [], []
    cur = 0
    for t in texts:
        t = np.asarray(t, dtype=np.uint8)
        starts.append(cur)
        parts.append(t)
        parts.append(SEP)
        cur += int(t.size) + 1
    joined = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint8)
    m, _, cnt = oracle.scan(patterns, joined, threads=threads, counts=True)
    out = []
    for s, t in zip(starts, texts):
        L = int(np.asarray(t).size)
        out.append((m[s:s + L], int(cnt[s:s + L].sum())))
    return out


def check_batch(res, refs, lengths, hits_only=False):
    c = res.counters.cpu().numpy()
    m = None if hits_only else res.match.cpu().numpy()
    hits = res.hits.cpu().numpy() if res.hits is not None else None
    hpos = 0
    tot_h = tot_o = 0
    for t, (m_ref, occ_ref) in enumerate(refs):
        L = int(lengths[t])
        pos, ids = oracle.hits_of(m_ref)
        if m is not None:
            o = int(res.match_offsets[t])
            bad = np.nonzero(m[o:o + L] != m_ref)[0]
            assert bad.size == 0, "text %d: first mismatch at %d" % (t, bad[0])
        assert c[2 + 2 * t] == pos.size, t
        assert c[3 + 2 * t] == occ_ref, t
        if hits is not None:
            hh = hits[hpos:hpos + pos.size]
            assert np.all(hh[:, 0] == t), t
            assert np.array_equal(hh[:, 1].astype(np.uint32), pos), t
            assert np.array_equal(hh[:, 2], ids), t
        hpos += pos.size
        tot_h += pos.size
        tot_o += occ_ref
    assert c[0] == tot_h and c[1] == tot_o




def runs_equal(a, b, offsets, lengths):
    """Two dense batch outputs agree on every text's run (the up to three
    elements between runs, left by the 16-byte alignment of each run, are
    not written)."""
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = b.cpu().numpy() if hasattr(b, "cpu") else np.asarray(b)
    for o, n in zip(offsets, lengths):
        o, n = int(o), int(n)
        if not np.array_equal(a[o:o + n], b[o:o + n]):
            return False
    return True
