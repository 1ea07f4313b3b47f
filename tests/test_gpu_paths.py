"""GPU parity for kernel paths and configurations at their real shapes:

* a batched call against the largest served pattern set (200,000 patterns of
  12..64 bases), whose default plan is the 512-thread, depth-10 kernel with no
  second filter, and the same plan forced;
* hits-only output (no dense array) on texts whose tiles hold more than the
  32 hit slots a tile parks, so the finish step rebuilds those tiles' hits by
  walking their positions again -- in one-text calls (walks at once and
  deferred) and in a batch;
* a served run on the eight served pattern sets at their full sizes.

Every text is compared with the oracle position by position, with its hit
count and its occurrence total."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_10498_amd as pf  # noqa: E402
from paper_1811_10498_amd.serve import Request, Server, TextBatch  # noqa: E402
from _gpu_common import check_batch as _check_batch, joined_oracle  # noqa: E402

DEV = torch.device("cuda:0")
@pytest.fixture(scope="module")
def served_sets():
    return W.served_tries(seed=4)


@pytest.fixture(scope="module")
def largest_table(served_sets):
    return pf.Table(served_sets[-1])


def _mixed_texts(g, pool):
    """150-base reads, texts of assorted lengths, a 3 Mbase text and a few
    ragged small ones, as (buffer, offsets, lengths, host texts)."""
    lens = ([150] * 200 + [int(x) for x in g.integers(1, 5000, size=40)]
            + [int(x) for x in g.integers(5000, 400_000, size=12)] + [3_000_017, 0, 1, 15, 17])
    texts = []
    for L in lens:
        if L and L < pool.size and g.random() < 0.5:   # cut from the pool: plenty of matches
            o = int(g.integers(0, pool.size - L))
            texts.append(pool[o:o + L].copy())
        else:
            texts.append(W.uniform_ascii(L, g))
    offs, cur = [], 0
    for t in texts:
        cur += int(g.integers(0, 3)) * 16 + int(g.integers(0, 16) if g.random() < 0.2 else 0)
        offs.append(cur)
        cur += t.size
    buf = np.full(cur + 16, ord("N"), dtype=np.uint8)
    for o, t in zip(offs, texts):
        buf[o:o + t.size] = t
    return buf, np.array(offs), np.array(lens), texts


def test_largest_served_table_batch_default_and_forced_plan(served_sets, largest_table):
    pats = served_sets[-1]
    tab = largest_table
    print("largest served set: %d patterns, %d states, default plan %s"
          % (len(pats), tab.num_states, tab.default_plan()), flush=True)
    g = W.rng(501)
    pool = W.uniform_ascii(4_000_000, g)
    # plant patterns of the set into the pool so long walks and hits occur
    for k in g.integers(0, len(pats), size=20_000):
        p = np.frombuffer(pats[int(k)], dtype=np.uint8)
        o = int(g.integers(0, pool.size - p.size))
        pool[o:o + p.size] = p
    buf, offs, lens, texts = _mixed_texts(g, pool)
    refs = joined_oracle(pats, texts)
    base = torch.from_numpy(buf).to(DEV)
    # the depth-10 bitmap fills the LDS beside 512 threads' text, no room for
    # a hashed filter: the 512-thread depth-10 kernel without second filter
    forced = dict(block=512, depth=10, hash_bits=pf.PFAC_HASH_NONE, prefix=pf.PFAC_PREFIX_NONE)
    for p in (None, forced):
        print("batch plan", p, "texts", len(texts), "bases", int(lens.sum()), flush=True)
        res = pf.match_batch([tab], base, offs, lens, plan=p, hit_cap=int(lens.sum()) // 4)
        torch.cuda.synchronize()
        _check_batch(res, refs, lens)
    # the one-text call on the long text with the same plans
    long_t = texts[int(np.argmax(lens))]
    m_ref, occ_ref = refs[int(np.argmax(lens))]
    dt = torch.from_numpy(long_t).to(DEV)
    for p in (None, forced):
        r = pf.match(tab, dt, plan=p, hit_cap=long_t.size)
        torch.cuda.synchronize()
        assert np.array_equal(r.match.cpu().numpy(), m_ref)
        assert r.total() == occ_ref
        pos, ids = oracle.hits_of(m_ref)
        h = r.hit_list()
        assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)


def _dense_hit_text(g, n, k_lo, k_hi, count, planted_from=None):
    text = W.uniform_ascii(n, g)
    src = text if planted_from is None else planted_from
    pats = W.cut_patterns(src, count, k_lo, k_hi, g)
    return text, pats


HITS_ONLY_CASES = [
    # short patterns: about a fifth of all positions match; walks at once
    dict(name="short", n=700_001, lo=4, hi=6, count=200, random=True, plan=None),
    # 12..14-base patterns cut from the text (about 10 % of positions match):
    # second filter on, walks deferred, the walk buffer overflows
    dict(name="deferred", n=1_000_003, lo=12, hi=14, count=100_000, random=False, plan=None),
    dict(name="inline", n=1_000_003, lo=12, hi=14, count=100_000, random=False,
         plan=dict(walks=pf.PFAC_WALKS_INLINE)),
]


@pytest.mark.parametrize("case", range(len(HITS_ONLY_CASES)))
def test_hits_only_with_more_hits_than_tile_slots(case):
    c = HITS_ONLY_CASES[case]
    g = W.rng(600 + case)
    text = W.uniform_ascii(c["n"], g)
    if c["random"]:
        pats = W.random_patterns(c["count"], c["lo"], c["hi"], g)
    else:
        pats = W.cut_patterns(text, c["count"], c["lo"], c["hi"], g)
    m_ref, total_ref = oracle.scan(pats, text, threads=8)
    pos, ids = oracle.hits_of(m_ref)
    per_tile = np.bincount(pos // 2048)
    print(c["name"], "hits", pos.size, "max per 2048-tile", per_tile.max(), flush=True)
    assert per_tile.max() > 32
    tab = pf.Table(pats)
    print("plan", tab.default_plan() if c["plan"] is None else c["plan"], flush=True)
    dt = torch.from_numpy(text).to(DEV)
    r = pf.match(tab, dt, dense=False, hit_cap=pos.size + 10, plan=c["plan"])
    torch.cuda.synchronize()
    assert r.match is None
    assert r.num_hits() == pos.size and r.total() == total_ref
    h = r.hit_list()
    assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)
    # batched, hits only: 1024-position tiles, many of them over their slots
    buf, offs, lens, texts = _mixed_texts(g, text)
    refs = joined_oracle(pats, texts)
    base = torch.from_numpy(buf).to(DEV)
    res = pf.match_batch([tab], base, offs, lens, dense=False, hit_cap=int(lens.sum()),
                         plan=c["plan"])
    torch.cuda.synchronize()
    _check_batch(res, refs, lens, hits_only=True)


def test_served_run_on_the_full_served_sets(served_sets):
    """The eight served pattern sets (1,000 .. 200,000 patterns) resident,
    full-size requests of every kind (10,000 reads of 150 bases, a 1 Mbase
    contig, a 50 Mbase text) arriving together; every text of every request
    checked against the oracle."""
    tables = [pf.Table(s) for s in served_sets]
    specs = W.served_requests(9, rate_bases_per_s=1e12, seed=7)
    g = W.rng(700)
    reqs = []
    for r in specs:
        if r.kind == "reads":
            n = int(r.lengths.size)
            L = int(r.lengths[0])
            buf = W.uniform_ascii(n * 160, g)
            reqs.append(Request(r.rid, r.trie, TextBatch(buf, 160 * np.arange(n), r.lengths),
                                0.0))
        else:
            reqs.append(Request(r.rid, r.trie, r.texts(), 0.0))
    print("requests", [(r.kind, r.trie) for r in specs], flush=True)
    srv = Server(tables, budget_bytes=32 << 30)
    stats = srv.run(reqs)
    print(stats, flush=True)
    assert stats["requests"] == len(reqs)
    by_trie = {}
    for r in srv.done:
        by_trie.setdefault(r.table, []).append(r)
    for tr, rs in by_trie.items():
        texts = []
        for r in rs:
            texts += [np.asarray(r.text(i)) for i in range(r.num_texts)]
        refs = iter(joined_oracle(served_sets[tr], texts))
        for r in rs:
            res = r.result
            for i in range(r.num_texts):
                m_ref, occ_ref = next(refs)
                assert np.array_equal(res.text_match(i).cpu().numpy(), m_ref), (r.rid, i)
                assert res.occurrences[i] == occ_ref, (r.rid, i)
                assert res.num_hits[i] == np.count_nonzero(m_ref), (r.rid, i)
        print("trie", tr, "requests", len(rs), "texts", len(texts), "checked", flush=True)
