"""GPU parity of the all-occurrence output (pfac_match_all): the list of
every (position, pattern ID) pair -- shorter patterns at a position where a
longer one matches, and every copy of duplicate patterns, included --
compared entry by entry with the oracle's list (ascending position, then
pattern length, then ID)."""
import numpy as np
import pytest

import oracle
import workloads as W
from _checkers import read_golden

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_10498_amd as pf  # noqa: E402

DEV = torch.device("cuda:0")


def _check(pats, text, plan=None, enc="ascii", table=None):
    t = np.asarray(text, dtype=np.uint8)
    tab = table or pf.Table(pats)
    buf = W.pack2bit(W.ascii_to_codes(t)) if enc == "2bit" else t
    dt = torch.from_numpy(np.array(buf)).to(DEV)
    res = pf.match_all(tab, dt, n=t.size, enc=enc, plan=plan)
    torch.cuda.synchronize()
    ref = oracle.occurrences(pats, t)
    got = res.occurrences()
    assert res.total() == len(ref)
    assert got.shape == ref.shape
    bad = np.nonzero(np.any(got != ref, axis=1))[0]
    assert bad.size == 0, "first difference at %d: gpu %s oracle %s" % (
        bad[0], got[bad[0]].tolist(), ref[bad[0]].tolist())
    m_ref, _ = oracle.scan(pats, t)
    assert int(res.counters[0]) == np.count_nonzero(m_ref)
    return res


@pytest.mark.parametrize("name", ["ex1_fig1_text.txt", "ex2_table1_text.txt"])
def test_worked_examples(name):
    ex = read_golden(name)
    pats = [p.encode() for p in ex["patterns"].split()]
    text = np.frombuffer(ex["text"].encode(), dtype=np.uint8)
    res = _check(pats, text)
    want = [tuple(int(x) for x in c.split(",")) for c in ex["occurrences"].split()]
    assert [tuple(r) for r in res.occurrences().tolist()] == want


def _nested_set(g, text):
    """Patterns with many prefixes of each other and duplicates: cut from the
    text, then every prefix of some of them, then copies."""
    base = W.cut_patterns(text, 400, 14, 40, g)
    pats = list(base)
    for p in base[:150]:
        for L in range(12, len(p), 3):
            pats.append(p[:L])
    pats += base[:60] + [p[:12] for p in base[:30]]        # duplicates
    pats += W.random_patterns(2000, 12, 30, g)
    return pats


ALL_PLANS = [None, dict(walks=pf.PFAC_WALKS_INLINE), dict(walks=pf.PFAC_WALKS_DEFERRED),
             dict(tile=1024), dict(variant=pf.PFAC_VARIANT_GLOBAL),
             dict(prefix=1, hash_bits=pf.PFAC_HASH_NONE, depth=10, block=512),
             dict(depth=8, levels=0, hash_bits=pf.PFAC_HASH_NONE)]


@pytest.mark.parametrize("plan", range(len(ALL_PLANS)))
def test_nested_and_duplicate_patterns_every_plan(plan):
    g = W.rng(1200)
    text = W.uniform_ascii(800_003, g)
    pats = _nested_set(g, text)
    # repeats of one pattern and non-bases
    p = np.frombuffer(pats[3], dtype=np.uint8)
    for k in range(300):
        text[100_000 + 50 * k:100_000 + 50 * k + p.size] = p
    text[20_000:20_007] = ord("N")
    print("plan", ALL_PLANS[plan], "patterns", len(pats), flush=True)
    _check(pats, text, plan=ALL_PLANS[plan])


def test_tiles_with_more_hits_than_slots():
    g = W.rng(1201)
    text = W.uniform_ascii(300_007, g)
    pats = W.random_patterns(300, 3, 6, g) + [b"ACG", b"ACG", b"ACGT"]
    m_ref, _ = oracle.scan(pats, text)
    assert np.bincount(np.nonzero(m_ref)[0] // 2048).max() > 32
    _check(pats, text)


def test_packed_text_and_overflowing_cap():
    g = W.rng(1202)
    text = W.uniform_ascii(500_001, g)
    pats = _nested_set(g, text)
    _check(pats, text, enc="2bit")
    tab = pf.Table(pats)
    dt = torch.from_numpy(text).to(DEV)
    ref = oracle.occurrences(pats, text)
    cap = len(ref) // 3
    res = pf.match_all(tab, dt, cap=cap)
    torch.cuda.synchronize()
    assert res.total() == len(ref)
    assert np.array_equal(res.occ[:cap].cpu().numpy().astype(np.int64), ref[:cap])


def test_tiny_workload_and_empty_text():
    w = W.plain_workload(0)
    _check(w.patterns, w.text)
    tab = pf.Table(w.patterns)
    res = pf.match_all(tab, torch.zeros(0, dtype=torch.uint8, device=DEV), n=0)
    torch.cuda.synchronize()
    assert res.counters.cpu().tolist() == [0, 0]
