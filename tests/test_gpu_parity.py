"""GPU parity: the HIP path through the C ABI against the CPU oracle,
bit-exact (integer matching: match array, total occurrences, ordered hit list)."""
import numpy as np
import pytest

import oracle
import workloads as W
from _checkers import read_golden
from _gpu_common import runs_equal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_10498_amd as pf  # noqa: E402

DEV = torch.device("cuda:0")


def _gpu(patterns, text_ascii, plan=None, enc="ascii", hit_cap=None, table=None, offset=0):
    """Run the GPU path on an ASCII host text (packing it when enc='2bit')."""
    t = np.asarray(text_ascii, dtype=np.uint8)
    n = int(t.size)
    if enc == "2bit":
        buf = W.pack2bit(W.ascii_to_codes(t))
    else:
        buf = t
    if offset:
        buf = np.concatenate([np.zeros(offset, dtype=np.uint8), buf])
    dt = torch.from_numpy(np.array(buf, dtype=np.uint8)).to(DEV)
    if offset:
        dt = dt[offset:]
    tab = table or pf.Table(patterns)
    res = pf.match(tab, dt, n=n, enc=enc, plan=plan, hit_cap=n + 16 if hit_cap is None else hit_cap)
    torch.cuda.synchronize()
    return res


def _check(res, patterns, text_ascii, m_ref=None, total_ref=None):
    if m_ref is None:
        m_ref, total_ref = oracle.scan(patterns, np.asarray(text_ascii, dtype=np.uint8), threads=8)
    m = res.match.cpu().numpy()
    bad = np.nonzero(m != m_ref)[0]
    assert bad.size == 0, "first mismatch at %d: gpu %d oracle %d (%d mismatches)" % (
        bad[0], m[bad[0]], m_ref[bad[0]], bad.size)
    assert res.total() == total_ref
    pos, ids = oracle.hits_of(m_ref)
    assert res.num_hits() == pos.size
    h = res.hit_list()
    assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)


def _pats(s):
    return [p.encode() for p in s.split()]


@pytest.mark.parametrize("name", ["ex1_fig1_text.txt", "ex2_table1_text.txt"])
def test_worked_examples(name):
    ex = read_golden(name)
    pats = _pats(ex["patterns"])
    text = np.frombuffer(ex["text"].encode(), dtype=np.uint8)
    res = _gpu(pats, text)
    assert res.match.cpu().numpy().tolist() == [int(x) for x in ex["match"].split()]
    assert res.total() == int(ex["total"])


def test_tiny_workload_full():
    w = W.plain_workload(0)
    print("c0: n=%d patterns=%d" % (w.n, len(w.patterns)), flush=True)
    res = _gpu(w.patterns, w.text)
    _check(res, w.patterns, w.text)


def test_markov_workload_reduced():
    w = W.plain_workload(1, n=8_000_003)
    print("c1 reduced: n=%d patterns=%d" % (w.n, len(w.patterns)), flush=True)
    res = _gpu(w.patterns, w.text)
    _check(res, w.patterns, w.text)


def test_packed_big_trie_reduced():
    w = W.plain_workload(2, n=4_000_037, num_patterns=200_000)
    print("c2 reduced: n=%d patterns=%d" % (w.n, len(w.patterns)), flush=True)
    ascii_text = w.ascii()
    m_ref, total_ref = oracle.scan(w.patterns, ascii_text, threads=8)
    tab = pf.Table(w.patterns)
    dt = torch.from_numpy(w.text).to(DEV)
    res = pf.match(tab, dt, n=w.n, enc="2bit", hit_cap=w.n)
    torch.cuda.synchronize()
    _check(res, w.patterns, ascii_text, m_ref, total_ref)
    # same text as ASCII gives the same answer
    res2 = _gpu(w.patterns, ascii_text, table=tab)
    _check(res2, w.patterns, ascii_text, m_ref, total_ref)


PLANS = [
    dict(variant=pf.PFAC_VARIANT_GLOBAL),
    dict(block=256, depth=6),
    dict(block=512, depth=7),
    dict(block=1024, depth=8),
    dict(block=512, depth=9),
    dict(block=256, depth=10),
    dict(block=1024, depth=9, grid=3),
    dict(block=256, depth=6, grid=1),
]


@pytest.mark.parametrize("plan", range(len(PLANS)))
def test_every_plan_gives_identical_results(plan):
    g = W.rng(31)
    text = W.uniform_ascii(300_017, g)
    pats = (W.cut_patterns(text, 300, 4, 40, g) + W.random_patterns(300, 3, 12, g)
            + [b"A", b"ACGT", b"ACGT", b"CG"])
    text[1000:1010] = ord("N")
    text[5000] = ord("a")
    print("plan", PLANS[plan], flush=True)
    res = _gpu(pats, text, plan=PLANS[plan])
    _check(res, pats, text)


LDS_PLANS = [
    dict(block=256, depth=6, levels=1),
    dict(block=512, depth=7, levels=2),
    dict(block=768, depth=8, levels=3),
    dict(block=1024, depth=9, levels=0),
    dict(block=1024, depth=9, levels=pf.PFAC_LEVELS_NONE),
    dict(block=256, depth=10, levels=pf.PFAC_LEVELS_NONE),
    dict(block=512, depth=6, levels=8),
]


@pytest.mark.parametrize("plan", range(len(LDS_PLANS)))
def test_lds_trie_levels_give_identical_results(plan):
    """Patterns longer than the filter depth: the filter bit is a depth-D
    node found by rank and the walk goes on through the trie levels held in
    LDS, then the global table."""
    w = W.plain_workload(1, n=1_500_007, num_patterns=4000)
    extra = W.cut_patterns(w.text, 200, 11, 14, W.rng(77))      # ends inside LDS levels
    pats = w.patterns + extra
    text = w.text.copy()
    text[5000:5003] = ord("N")
    print("plan", LDS_PLANS[plan], flush=True)
    res = _gpu(pats, text, plan=LDS_PLANS[plan])
    _check(res, pats, text)


HASH_PLANS = [
    dict(block=1024, depth=9, hash_bits=12),
    dict(block=512, depth=8, hash_bits=17, levels=pf.PFAC_LEVELS_NONE),
    dict(block=1024, depth=9, hash_bits=pf.PFAC_HASH_NONE),
    dict(block=256, depth=7, hash_bits=14, levels=2),
    dict(block=256, depth=10, hash_bits=16, levels=pf.PFAC_LEVELS_NONE),
]


@pytest.mark.parametrize("plan", range(len(HASH_PLANS)))
def test_second_filter_gives_identical_results(plan):
    """Every pattern has 16 or more bases: queued windows first test the hash
    of their first 16 bases.  Non-bases planted 10..15 bases after the start
    of pattern occurrences (inside the hashed window, past the first filter)
    must still walk."""
    w = W.plain_workload(1, n=2_000_003, num_patterns=3000)
    pats = w.patterns
    text = w.text.copy()
    m0, _ = oracle.scan(pats, text, threads=8)
    occ = np.nonzero(m0)[0]
    g = W.rng(78)
    for q in g.choice(occ, size=min(40, occ.size), replace=False):
        off = int(g.integers(10, 16))
        if q + off < text.size:
            text[q + off] = ord("N")
    print("plan", HASH_PLANS[plan], "occurrences", occ.size, flush=True)
    res = _gpu(pats, text, plan=HASH_PLANS[plan])
    _check(res, pats, text)


def test_default_plan_uses_second_filter_when_patterns_are_long():
    tab = pf.Table(W.random_patterns(5000, 16, 40, W.rng(79)))
    p = tab.default_plan(1 << 20)
    assert 12 <= p["hash_bits"] <= 18
    short = pf.Table([b"ACG"] + W.random_patterns(100, 16, 40, W.rng(80)))
    assert short.default_plan(1 << 20)["hash_bits"] == pf.PFAC_HASH_NONE
    with pytest.raises(pf.PfacError):
        pf.match(tab, torch.zeros(64, dtype=torch.uint8, device=DEV), plan=dict(hash_bits=21))


def test_edge_sizes_and_ragged_tails():
    g = W.rng(32)
    pats = W.random_patterns(100, 1, 10, g) + [b"ACGTACGTACGTACGTACGT"]
    tab = pf.Table(pats)
    for n in [0, 1, 2, 3, 5, 19, 20, 21, 4095, 4096, 4097, 8191, 8192, 8193, 16384 + 7,
              3 * 8192 - 1, 100_000]:
        text = W.uniform_ascii(n, g)
        print("n=%d" % n, flush=True)
        for plan in (None, dict(block=256, depth=10), dict(variant=pf.PFAC_VARIANT_GLOBAL)):
            res = _gpu(pats, text, plan=plan, table=tab)
            _check(res, pats, text)
            res = _gpu(pats, text, plan=plan, table=tab, enc="2bit")
            _check(res, pats, text)


def test_every_byte_value_and_misaligned_text():
    g = W.rng(33)
    text = W.uniform_ascii(50_000, g)
    junk = g.integers(0, 256, size=5000).astype(np.uint8)
    idx = g.integers(0, text.size, size=5000)
    text[idx] = junk
    text[:256] = np.arange(256, dtype=np.uint8)
    pats = W.random_patterns(200, 1, 6, g) + W.cut_patterns(text[20000:], 50, 5, 30, g)
    pats = [p for p in pats if all(c in b"ACGT" for c in p)]
    for off in (0, 1, 3, 7):
        res = _gpu(pats, text, offset=off)
        _check(res, pats, text)


def test_homopolymer_worst_case_walks():
    """All-A text against A, AA, ..., A^64: every walk runs to the deepest
    state (the longest walks the method has)."""
    pats = [b"A" * L for L in range(1, 65)] + [b"C" * 64]
    text = np.full(70_001, ord("A"), dtype=np.uint8)
    text[40_000] = ord("C")
    for plan in (None, dict(variant=pf.PFAC_VARIANT_GLOBAL), dict(block=256, depth=6)):
        res = _gpu(pats, text, plan=plan)
        _check(res, pats, text)


def test_single_state_trie_and_long_patterns():
    text = W.uniform_ascii(10_000, W.rng(34))
    res = _gpu([b"G"], text)
    _check(res, [b"G"], text)
    long_pats = [bytes(text[100:100 + 5000]), b"ACGT" * 1500]   # halo beyond LDS staging
    res = _gpu(long_pats, text)
    _check(res, long_pats, text)
    short = [b"ACGT" * 3000]                                    # longer than the text
    res = _gpu(short, text[:9000])
    _check(res, short, text[:9000])


def test_duplicates_report_smallest_id_and_count_all():
    text = np.frombuffer(b"ACGTTACGTAACGT" * 1000, dtype=np.uint8)
    pats = [b"CGT", b"ACGT", b"ACGT", b"CGT", b"ACGT"]
    res = _gpu(pats, text)
    _check(res, pats, text)
    assert set(np.unique(res.match.cpu().numpy())) <= {0, 1, 2}


def test_hit_list_overflow_reports_true_count():
    w = W.plain_workload(0, n=300_000)
    pats = w.patterns + W.random_patterns(50, 4, 5, W.rng(35))
    m_ref, total_ref = oracle.scan(pats, w.text)
    pos, ids = oracle.hits_of(m_ref)
    cap = pos.size // 3
    res = _gpu(pats, w.text, hit_cap=cap)
    assert res.num_hits() == pos.size and res.total() == total_ref
    h = res.hits[:cap].cpu().numpy()
    assert np.array_equal(h[:, 0], pos[:cap]) and np.array_equal(h[:, 1], ids[:cap])


def test_outputs_are_optional():
    w = W.plain_workload(0, n=100_000)
    m_ref, total_ref = oracle.scan(w.patterns, w.text)
    tab = pf.Table(w.patterns)
    dt = torch.from_numpy(w.text).to(DEV)
    r1 = pf.match(tab, dt, dense=False, hit_cap=w.n)
    r2 = pf.match(tab, dt, hits=False)
    torch.cuda.synchronize()
    assert r1.match is None and r1.total() == total_ref
    pos, ids = oracle.hits_of(m_ref)
    assert np.array_equal(r1.hit_list()[:, 0], pos)
    assert np.array_equal(r2.match.cpu().numpy(), m_ref) and r2.num_hits() == pos.size


def test_invalid_arguments_are_rejected():
    with pytest.raises(pf.PfacError) as e:
        pf.Table([b"ACGT", b"ACXT"])
    assert e.value.code == -2 and e.value.bad_index == 1
    with pytest.raises(pf.PfacError):
        pf.Table([])
    tab = pf.Table([b"ACGT"])
    dt = torch.zeros(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(pf.PfacError):
        pf.match(tab, dt, plan=dict(block=300))
    with pytest.raises(pf.PfacError):
        pf.match(tab, dt, plan=dict(depth=11))
    with pytest.raises(pf.PfacError):
        pf.match(tab, dt, plan=dict(depth=5))


def test_batch_matches_per_text_oracle():
    wb = W.batch_workload(num_texts=300, num_patterns=3000, median=3000.0, hi=60_000)
    print("batch: texts=%d bases=%d" % (wb.lengths.size, wb.total_bases), flush=True)
    tab = pf.Table(wb.patterns)
    base = torch.from_numpy(wb.buffer).to(DEV)
    for plan in (None, dict(block=256, depth=7), dict(variant=pf.PFAC_VARIANT_GLOBAL)):
        res = pf.match_batch([tab], base, wb.offsets, wb.lengths, plan=plan)
        torch.cuda.synchronize()
        m = res.match.cpu().numpy()
        c = res.counters.cpu().numpy()
        hits = res.hits.cpu().numpy()
        hpos = 0
        tot_h = tot_o = 0
        for t in range(wb.lengths.size):
            txt = wb.text(t)
            m_ref, total_ref = oracle.scan(wb.patterns, txt)
            o = int(res.match_offsets[t])
            assert np.array_equal(m[o:o + txt.size], m_ref), t
            pos, ids = oracle.hits_of(m_ref)
            assert c[2 + 2 * t] == pos.size and c[3 + 2 * t] == total_ref
            hh = hits[hpos:hpos + pos.size]
            assert np.all(hh[:, 0] == t)
            assert np.array_equal(hh[:, 1], pos) and np.array_equal(hh[:, 2], ids)
            hpos += pos.size
            tot_h += pos.size
            tot_o += total_ref
        assert c[0] == tot_h and c[1] == tot_o


def test_batch_several_tables_and_encodings():
    g = W.rng(36)
    sets = [W.random_patterns(50, 3, 9, g), W.random_patterns(500, 8, 20, g), [b"ACGT"]]
    tabs = [pf.Table(s) for s in sets]
    texts = [W.uniform_ascii(int(L), g) for L in [0, 1, 17, 4096, 10_000, 33_333, 7]]
    # ASCII texts at unaligned offsets, then the same texts packed
    parts, offs, encs, lens = [], [], [], []
    cur = 0
    for t in texts:
        pad = 3
        parts.append(np.zeros(pad, dtype=np.uint8))
        cur += pad
        offs.append(cur)
        parts.append(t)
        cur += t.size
        encs.append("ascii")
        lens.append(t.size)
    for t in texts:
        pad = (-cur) % 16
        parts.append(np.zeros(pad, dtype=np.uint8))
        cur += pad
        p = W.pack2bit(W.ascii_to_codes(t))
        offs.append(cur)
        parts.append(p)
        cur += p.size
        encs.append("2bit")
        lens.append(t.size)
    buf = torch.from_numpy(np.concatenate(parts)).to(DEV)
    tid = [i % 3 for i in range(len(lens))]
    res = pf.match_batch(tabs, buf, offs, lens, table_index=tid, enc=encs)
    torch.cuda.synchronize()
    m = res.match.cpu().numpy()
    c = res.counters.cpu().numpy()
    for i, L in enumerate(lens):
        t = texts[i % len(texts)]
        m_ref, total_ref = oracle.scan(sets[tid[i]], t)
        o = int(res.match_offsets[i])
        assert np.array_equal(m[o:o + L], m_ref), i
        assert c[3 + 2 * i] == total_ref


def _batch_check(res, patterns_of, texts, sample):
    """Per-text oracle check of a batched result on the text indices in `sample`."""
    m = res.match.cpu().numpy()
    c = res.counters.cpu().numpy()
    for t in sample:
        txt = texts[t]
        m_ref, total_ref = oracle.scan(patterns_of[t], txt)
        o = int(res.match_offsets[t])
        assert np.array_equal(m[o:o + txt.size], m_ref), t
        assert c[2 + 2 * t] == np.count_nonzero(m_ref) and c[3 + 2 * t] == total_ref, t


def test_prepared_batch_replays_in_a_graph():
    """pfac_batch_launch enqueues kernels only: captured once into a graph, every
    replay over new text contents (same sizes) matches the eager batched call
    and the oracle, with eager work and synchronisation between replays."""
    wb = W.batch_workload(num_texts=120, num_patterns=2000, median=2000.0, hi=40_000, seed=41)
    g = W.rng(42)
    sets = [wb.patterns, W.random_patterns(300, 6, 14, g)]
    tabs = [pf.Table(s) for s in sets]
    tid = np.arange(wb.lengths.size) % 2
    base = torch.from_numpy(wb.buffer.copy()).to(DEV)
    b = pf.Batch(tabs, wb.offsets, wb.lengths, table_index=tid, device=DEV)
    print("prepared batch: texts=%d bases=%d" % (wb.lengths.size, wb.total_bases), flush=True)
    res = b.launch(base)
    torch.cuda.synchronize()
    ref = pf.match_batch(tabs, base, wb.offsets, wb.lengths, table_index=tid)
    torch.cuda.synchronize()
    assert runs_equal(res.match, ref.match, res.match_offsets, wb.lengths)
    assert torch.equal(res.counters, ref.counters)
    nh = int(ref.counters[0])
    assert torch.equal(res.hits[:nh], ref.hits[:nh])

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.launch(base, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.launch(base, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    for k in range(3):
        # new contents: permute the bases (gaps stay), eager copy, then replay
        perm = g.permutation(4)
        lut = np.arange(256, dtype=np.uint8)
        lut[acgt] = acgt[perm]
        buf = lut[wb.buffer]
        base.copy_(torch.from_numpy(buf))
        torch.cuda.synchronize()
        b.match.fill_(-7)
        b.counters.fill_(-7)
        graph.replay()
        torch.cuda.synchronize()
        ref = pf.match_batch(tabs, base, wb.offsets, wb.lengths, table_index=tid)
        torch.cuda.synchronize()
        assert runs_equal(b.match, ref.match, b.match_offsets, wb.lengths), k
        assert torch.equal(b.counters, ref.counters), k
        nh = int(ref.counters[0])
        assert torch.equal(b.hits[:nh], ref.hits[:nh]), k
        texts = [buf[int(o):int(o) + int(n)] for o, n in zip(wb.offsets, wb.lengths)]
        sample = list(range(0, wb.lengths.size, 7))
        _batch_check(ref, [sets[i] for i in tid], texts, sample)
    b.close()


def test_prepared_batch_empty_and_rejections():
    tab = pf.Table([b"ACGT"])
    b = pf.Batch([tab], [0, 16], [0, 0], device=DEV)
    base = torch.zeros(32, dtype=torch.uint8, device=DEV)
    res = b.launch(base)
    torch.cuda.synchronize()
    assert res.counters.cpu().numpy().tolist() == [0] * 6
    b.close()
    with pytest.raises(pf.PfacError):
        pf.Batch([tab], [0], [5], table_index=[1], device=DEV)
    with pytest.raises(pf.PfacError):
        pf.Batch([tab], [0], [5], plan=dict(block=300), device=DEV)


@pytest.mark.parametrize("plan", [None, dict(levels=pf.PFAC_LEVELS_NONE),
                                  dict(block=256, depth=6, levels=2)])
def test_long_single_child_runs(plan):
    """Walks through long runs of single-child trie steps (the walk takes a
    run at once): long patterns, prefixes of them ending inside runs,
    occurrences with a substituted base or a non-base at every offset of a
    run, and occurrences cut short by the end of the text."""
    g = W.rng(90)
    longs = W.random_patterns(60, 40, 64, g)
    pats = list(longs)
    for p in longs[:30]:
        for k in sorted(set(int(x) for x in g.integers(8, len(p), size=3))):
            pats.append(p[:k])                      # finals inside a run
    parts = []
    for i, p in enumerate(longs):
        for off in range(0, len(p), 3):
            q = bytearray(p)
            if i % 3 == 0:
                q[off] = ord("N")
            elif i % 3 == 1:
                q[off] = ord("ACGT"[("ACGT".index(chr(q[off])) + 1) % 4])
            parts.append(bytes(q))
            parts.append(bytes(W.uniform_ascii(int(g.integers(0, 20)), g)))
        parts.append(p)                             # and one clean copy
    text = np.frombuffer(b"".join(parts) + longs[0][:30], dtype=np.uint8).copy()
    print("patterns", len(pats), "text", text.size, "plan", plan, flush=True)
    res = _gpu(pats, text, plan=plan)
    _check(res, pats, text)


WALK_PLANS = [
    dict(walks=pf.PFAC_WALKS_INLINE),
    dict(walks=pf.PFAC_WALKS_DEFERRED),
    dict(walks=pf.PFAC_WALKS_DEFERRED, hash_bits=pf.PFAC_HASH_NONE),   # many, overflows
    dict(walks=pf.PFAC_WALKS_DEFERRED, block=1024, depth=8, hash_bits=12),
]


@pytest.mark.parametrize("plan", range(len(WALK_PLANS)))
def test_deferred_walks_match_inline(plan):
    """Walks deferred to the end of the wave (start + 64 copied bases, continued on
    the text past them) give the oracle's results: patterns up to 120 bases,
    occurrences near tile and text ends, non-bases inside copied windows, and
    a plan whose walks overflow the hand-off buffer (the rest walk inline)."""
    w = W.plain_workload(1, n=2_500_001, num_patterns=2500)
    g = W.rng(93)
    longs = W.cut_patterns(w.text, 40, 65, 120, g)
    pats = w.patterns + longs
    text = w.text.copy()
    m0, _ = oracle.scan(pats, text, threads=8)
    occ = np.nonzero(m0)[0]
    for q in g.choice(occ, size=min(30, occ.size), replace=False):
        off = int(g.integers(16, 70))
        if q + off < text.size:
            text[q + off] = ord("N")
    for t0 in (2048 * 7, 2048 * 300):        # plant long patterns across tile edges
        p = longs[t0 % len(longs)]
        text[t0 - 30:t0 - 30 + len(p)] = np.frombuffer(p, dtype=np.uint8)
    p = longs[0]
    text[-40:] = np.frombuffer(p[:40], dtype=np.uint8)       # cut short by the end
    print("plan", WALK_PLANS[plan], flush=True)
    res = _gpu(pats, text, plan=WALK_PLANS[plan])
    _check(res, pats, text)


def test_deferred_walks_with_optional_outputs():
    w = W.plain_workload(1, n=1_000_003, num_patterns=1500)
    tab = pf.Table(w.patterns)
    dt = torch.from_numpy(w.text).to(DEV)
    m_ref, total_ref = oracle.scan(w.patterns, w.text, threads=8)
    pos, ids = oracle.hits_of(m_ref)
    plan = dict(walks=pf.PFAC_WALKS_DEFERRED)
    r1 = pf.match(tab, dt, plan=plan, dense=False, hit_cap=w.n)
    r2 = pf.match(tab, dt, plan=plan, hits=False)
    r3 = pf.match(tab, dt, plan=plan, dense=False, hits=False)
    torch.cuda.synchronize()
    h = r1.hit_list()
    assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)
    assert np.array_equal(r2.match.cpu().numpy(), m_ref)
    assert r1.total() == r2.total() == r3.total() == total_ref
    assert r3.num_hits() == pos.size
    assert tab.default_plan(w.n)["walks"] == pf.PFAC_WALKS_DEFERRED
    with pytest.raises(pf.PfacError):
        pf.match(tab, dt, plan=dict(walks=3))


READS_PLANS = [
    dict(variant=pf.PFAC_VARIANT_GLOBAL_TWO_ARRAYS),
    dict(variant=pf.PFAC_VARIANT_GLOBAL_MERGED),
    dict(variant=pf.PFAC_VARIANT_GLOBAL),
    dict(depth=6, levels=pf.PFAC_LEVELS_NONE, hash_bits=pf.PFAC_HASH_NONE,
         walks=pf.PFAC_WALKS_INLINE),
    dict(depth=9, levels=pf.PFAC_LEVELS_NONE, hash_bits=pf.PFAC_HASH_NONE,
         walks=pf.PFAC_WALKS_INLINE),
    dict(depth=8, levels=0, hash_bits=pf.PFAC_HASH_NONE, walks=pf.PFAC_WALKS_INLINE),
    dict(depth=9, levels=pf.PFAC_LEVELS_NONE, hash_bits=18, walks=pf.PFAC_WALKS_INLINE),
    None,
]


@pytest.mark.parametrize("plan", range(len(READS_PLANS)))
def test_paper_shaped_reads_every_ladder_plan(plan):
    """The plans of the benchmark's placement ladder on a paper-shaped reads
    file (newline-separated ~100-base reads, 100-base patterns): the oracle's
    results, walks stopping at every newline."""
    w = W.reads_workload(2, 1, num_reads=40_000)
    print("reads: n=%d reads=%d patterns=%d plan=%s" % (w.n, w.num_reads, len(w.patterns),
                                                         READS_PLANS[plan]), flush=True)
    res = _gpu(w.patterns, w.text, plan=READS_PLANS[plan])
    _check(res, w.patterns, w.text)


def test_paper_layouts_on_nested_duplicates_and_non_bases():
    """The two-array and merged-cell layouts (per-cell smallest ID, state
    occurrence counts) on duplicates, nested prefixes and non-base bytes."""
    g = W.rng(72)
    text = W.uniform_ascii(200_003, g)
    pats = (W.cut_patterns(text, 500, 3, 30, g) + [b"A", b"AC", b"ACG", b"ACG", b"CG", b"CG"]
            + W.random_patterns(300, 5, 12, g))
    text[777:790] = ord("N")
    text[5000] = ord("\n")
    for v in (pf.PFAC_VARIANT_GLOBAL_TWO_ARRAYS, pf.PFAC_VARIANT_GLOBAL_MERGED):
        res = _gpu(pats, text, plan=dict(variant=v))
        _check(res, pats, text)
    tab = pf.Table(pats)
    base = torch.zeros(64, dtype=torch.uint8, device=DEV)
    with pytest.raises(pf.PfacError):       # one-text calls only
        pf.match_batch([tab], base, [0], [10], plan=dict(variant=pf.PFAC_VARIANT_GLOBAL_MERGED))


def test_default_plan_defers_walks_only_within_the_copied_window():
    """Deferred walks carry 64 bases: the library defers them only when no
    pattern is longer (100-base patterns walk at once)."""
    g = W.rng(71)
    short = pf.Table(W.random_patterns(2000, 16, 64, g))
    long_ = pf.Table(W.random_patterns(2000, 100, 100, g))
    assert short.default_plan(1 << 24)["walks"] == pf.PFAC_WALKS_DEFERRED
    p = long_.default_plan(1 << 24)
    assert p["walks"] == pf.PFAC_WALKS_INLINE and p["hash_bits"] == 18 and p["depth"] == 9


def test_two_streams_keep_their_own_scratch():
    """Calls on two streams at once (each stream has its own library scratch:
    tile counts, hit slots, look-back words, deferred walks) give each text
    its own results."""
    w = W.plain_workload(1, n=3_000_001, num_patterns=2000)
    tab = pf.Table(w.patterns)
    a = torch.from_numpy(w.text).to(DEV)
    b = torch.flip(a, [0]).contiguous()
    ra0 = pf.match(tab, a, hit_cap=w.n)
    rb0 = pf.match(tab, b, hit_cap=w.n)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for _ in range(4):
        with torch.cuda.stream(s1):
            ra = pf.match(tab, a, hit_cap=w.n)
        with torch.cuda.stream(s2):
            rb = pf.match(tab, b, hit_cap=w.n)
        outs.append((ra, rb))
    torch.cuda.synchronize()
    for ra, rb in outs:
        for r, r0 in ((ra, ra0), (rb, rb0)):
            assert torch.equal(r.match, r0.match)
            assert r.total() == r0.total() and r.num_hits() == r0.num_hits()
            assert np.array_equal(r.hit_list(), r0.hit_list())
    m_ref, total_ref = oracle.scan(w.patterns, w.text, threads=8)
    assert np.array_equal(ra0.match.cpu().numpy(), m_ref) and ra0.total() == total_ref
