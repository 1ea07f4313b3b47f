"""GPU parity of the launch plans: the prefix filter, the larger hashed
filters, tile sizes and deferred walks, in one-text and batched calls, each
compared with the oracle position by position (match array, hit list,
occurrence totals)."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_10498_amd as pf  # noqa: E402
from _gpu_common import check_batch as _check_batch, joined_oracle  # noqa: E402

DEV = torch.device("cuda:0")
NONE_H = pf.PFAC_HASH_NONE
NONE_P = pf.PFAC_PREFIX_NONE


@pytest.fixture(scope="module")
def long_set():
    """60,000 patterns of 12..32 bases (every one longer than any filter
    depth), half cut from a text that also holds non-bases, plus that text."""
    g = W.rng(801)
    text = W.uniform_ascii(3_000_029, g)
    pats = (W.cut_patterns(text, 30_000, 12, 32, g) + W.random_patterns(30_000, 12, 32, g))
    text[5000:5010] = ord("N")
    text[77_777] = ord("\n")
    text[200_003] = ord("a")
    # a homopolymer stretch and a repeated pattern: long walks, dense hits
    text[300_000:300_400] = ord("A")
    p = np.frombuffer(pats[7], dtype=np.uint8)
    for k in range(200):
        text[400_000 + 40 * k:400_000 + 40 * k + p.size] = p
    m_ref, total_ref = oracle.scan(pats, text, threads=16)
    return pats, text, pf.Table(pats), m_ref, total_ref


SINGLE_PLANS = [
    dict(prefix=1, hash_bits=NONE_H, depth=8),
    dict(prefix=1, hash_bits=18, depth=9),
    dict(prefix=1, hash_bits=NONE_H, depth=10, block=512, walks=pf.PFAC_WALKS_DEFERRED),
    dict(prefix=1, depth=7, tile=1024, walks=pf.PFAC_WALKS_INLINE),
    dict(hash_bits=19, depth=9, prefix=NONE_P),
    dict(hash_bits=20, depth=7, block=512, prefix=NONE_P),
    dict(tile=1024),
    dict(tile=1024, walks=pf.PFAC_WALKS_INLINE, prefix=1),
    dict(prefix=1, levels=0, depth=8, hash_bits=NONE_H),
    # the filter as a pair table (one LDS byte per two neighbouring windows)
    # and as the plain bitmap
    dict(pair=1, depth=9, hash_bits=NONE_H, prefix=NONE_P),
    dict(pair=1, depth=8, hash_bits=18),
    dict(pair=pf.PFAC_PAIR_NONE, depth=9, hash_bits=18),
    dict(pair=1, depth=7, tile=1024, prefix=1),
    dict(pair=1, depth=6, block=512),
    None,
]


@pytest.mark.parametrize("plan", range(len(SINGLE_PLANS)))
def test_one_text_plans_match_oracle(long_set, plan):
    pats, text, tab, m_ref, total_ref = long_set
    p = SINGLE_PLANS[plan]
    print("plan", p, "default", tab.default_plan(), flush=True)
    dt = torch.from_numpy(text).to(DEV)
    res = pf.match(tab, dt, plan=p, hit_cap=text.size)
    torch.cuda.synchronize()
    m = res.match.cpu().numpy()
    bad = np.nonzero(m != m_ref)[0]
    assert bad.size == 0, "first mismatch at %d: gpu %d oracle %d" % (bad[0], m[bad[0]],
                                                                       m_ref[bad[0]])
    assert res.total() == total_ref
    pos, ids = oracle.hits_of(m_ref)
    h = res.hit_list()
    assert res.num_hits() == pos.size
    assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)
    # hits only
    r2 = pf.match(tab, dt, plan=p, dense=False, hit_cap=text.size)
    torch.cuda.synchronize()
    assert r2.total() == total_ref and r2.num_hits() == pos.size
    assert np.array_equal(r2.hit_list()[:, 0], pos)


def test_prefix_filter_on_packed_text(long_set):
    pats, text, tab, m_ref, total_ref = long_set
    clean = np.where(np.isin(text, np.frombuffer(b"ACGT", dtype=np.uint8)), text, ord("A"))
    m_c, tot_c = oracle.scan(pats, clean, threads=16)
    packed = torch.from_numpy(W.pack2bit(W.ascii_to_codes(clean))).to(DEV)
    for p in (dict(prefix=1, hash_bits=NONE_H, depth=10, block=512), dict(prefix=1, tile=1024)):
        res = pf.match(tab, packed, n=clean.size, enc="2bit", plan=p, hit_cap=clean.size)
        torch.cuda.synchronize()
        assert np.array_equal(res.match.cpu().numpy(), m_c), p
        assert res.total() == tot_c


def _batch_texts(g, pool, reads=300):
    """150-base reads, short and mid-size texts and two long ones, at mixed
    (some unaligned) offsets; some cut from `pool`."""
    lens = ([150] * reads + [int(x) for x in g.integers(1, 1200, size=60)]
            + [int(x) for x in g.integers(2000, 200_000, size=20)] + [1_500_007, 700_001, 0, 513,
                                                                      512, 511, 257, 256, 255])
    texts = []
    for L in lens:
        if L and g.random() < 0.6:
            o = int(g.integers(0, pool.size - L))
            texts.append(pool[o:o + L].copy())
        else:
            texts.append(W.uniform_ascii(L, g))
    offs, cur = [], 0
    for t in texts:
        cur += int(g.integers(0, 2)) * 16 + (int(g.integers(1, 16)) if g.random() < 0.15 else 0)
        offs.append(cur)
        cur += t.size
    buf = np.full(cur + 64, ord("N"), dtype=np.uint8)
    for o, t in zip(offs, texts):
        buf[o:o + t.size] = t
    return buf, np.array(offs), np.array(lens), texts


BATCH_PLANS = [
    None,
    dict(tile=256),
    dict(tile=2048),
    dict(walks=pf.PFAC_WALKS_DEFERRED),
    dict(prefix=1, walks=pf.PFAC_WALKS_DEFERRED, tile=256),
    dict(prefix=1, hash_bits=NONE_H, depth=10, block=512),
    dict(walks=pf.PFAC_WALKS_INLINE, hash_bits=19),
    dict(pair=1, depth=9, hash_bits=18),
    dict(pair=1, depth=8, tile=256, walks=pf.PFAC_WALKS_DEFERRED),
    dict(pair=pf.PFAC_PAIR_NONE, depth=9),
    dict(variant=pf.PFAC_VARIANT_GLOBAL),
]


@pytest.mark.parametrize("plan", range(len(BATCH_PLANS)))
def test_batch_plans_match_oracle(long_set, plan):
    pats, text, tab, _, _ = long_set
    g = W.rng(900 + plan)
    buf, offs, lens, texts = _batch_texts(g, text)
    refs = joined_oracle(pats, texts)
    base = torch.from_numpy(buf).to(DEV)
    p = BATCH_PLANS[plan]
    print("batch plan", p, "texts", len(texts), flush=True)
    res = pf.match_batch([tab], base, offs, lens, plan=p, hit_cap=int(lens.sum()))
    torch.cuda.synchronize()
    _check_batch(res, refs, lens)
    res2 = pf.match_batch([tab], base, offs, lens, plan=p, dense=False, hit_cap=int(lens.sum()))
    torch.cuda.synchronize()
    _check_batch(res2, refs, lens, hits_only=True)


def test_prepared_batch_with_short_tiles_and_deferred_walks_in_a_graph(long_set):
    """A prepared batch with 256-position tiles for its reads and deferred
    walks, captured once and replayed over new contents."""
    pats, text, tab, _, _ = long_set
    g = W.rng(950)
    buf, offs, lens, texts = _batch_texts(g, text, reads=1000)
    base = torch.from_numpy(buf.copy()).to(DEV)
    b = pf.Batch([tab], offs, lens, plan=dict(walks=pf.PFAC_WALKS_DEFERRED), device=DEV)
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
        lut = np.arange(256, dtype=np.uint8)
        lut[acgt] = acgt[g.permutation(4)]
        nb = lut[buf]
        base.copy_(torch.from_numpy(nb))
        torch.cuda.synchronize()
        b.match.fill_(-7)
        b.counters.fill_(-7)
        graph.replay()
        torch.cuda.synchronize()
        new_texts = [nb[int(o):int(o) + int(n)] for o, n in zip(offs, lens)]
        refs = joined_oracle(pats, new_texts)
        res = pf.BatchResult(b.match, b.hits, b.counters, b.match_offsets)
        _check_batch(res, refs, lens)
    b.close()
