"""GPU parity for output layouts and filter forms the default workloads do not
reach:

* a batch whose per-text output runs are back to back (most of them not
  16-byte aligned): the pre-zeroing scan writes those texts' zeros at their
  ends instead, in 4-byte stores;
* one text whose dense output starts 4 bytes past an aligned address (the
  scan without pre-zeroing), with a ragged last tile;
* a large pattern set with K = 12 (the one-hash second filter) on ASCII text
  with non-bases and lower case, so that tiles holding them test the filter
  entry by entry instead of while classifying;
* walks kept for the end of the wave (and walks at once) with patterns
  shorter than the filter depth, whose finals lie within the jump.

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
from _gpu_common import check_batch, joined_oracle  # noqa: E402

DEV = torch.device("cuda:0")


def test_batch_with_back_to_back_output_runs():
    wb = W.batch_workload(num_texts=200, num_patterns=3000, median=6000.0, hi=60_000, seed=91)
    tab = pf.Table(wb.patterns)
    base = torch.from_numpy(wb.buffer).to(DEV)
    offs = np.concatenate([[0], np.cumsum(wb.lengths)[:-1]]).astype(np.uint64)
    assert (offs % 4 != 0).sum() > 100
    print("batch: texts=%d bases=%d" % (wb.lengths.size, wb.total_bases), flush=True)
    res = pf.match_batch([tab], base, wb.offsets, wb.lengths, match_offsets=offs,
                         hit_cap=wb.total_bases // 8 + 1024)
    torch.cuda.synchronize()
    refs = joined_oracle(wb.patterns, [wb.text(t) for t in range(wb.lengths.size)])
    check_batch(res, refs, wb.lengths)
    # the same batch in the default layout gives the same runs
    res2 = pf.match_batch([tab], base, wb.offsets, wb.lengths,
                          hit_cap=wb.total_bases // 8 + 1024)
    torch.cuda.synchronize()
    check_batch(res2, refs, wb.lengths)


def test_one_text_with_unaligned_dense_output():
    n = 1_000_003
    w = W.plain_workload(0, n=n, num_patterns=400)
    tab = pf.Table(w.patterns)
    text = torch.from_numpy(w.text).to(DEV)
    m_ref, total_ref = oracle.scan(w.patterns, w.text)
    pos, ids = oracle.hits_of(m_ref)
    buf = torch.full((n + 1,), -7, dtype=torch.int32, device=DEV)
    view = buf[1:]                        # 4 bytes past a 256-byte aligned allocation
    assert view.data_ptr() % 16 == 4
    out = pf.MatchResult(view, torch.empty((pos.size + 64, 2), dtype=torch.int32, device=DEV),
                         torch.empty(2, dtype=torch.int64, device=DEV))
    print("one text: n=%d hits=%d" % (n, pos.size), flush=True)
    r = pf.match(tab, text, out=out)
    torch.cuda.synchronize()
    assert int(buf[0]) == -7
    assert np.array_equal(r.match.cpu().numpy(), m_ref)
    assert r.num_hits() == pos.size and r.total() == total_ref
    h = r.hit_list()
    assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)


def test_one_hash_filter_on_text_with_non_bases():
    g = W.rng(93)
    n = 1 << 21
    codes = W.uniform_codes(n, g)
    text = W.codes_to_ascii(codes).copy()
    planted = W.cut_patterns(text, 60_000, 12, 20, g)
    pats = planted + W.random_patterns(100_000, 12, 20, g)
    # non-bases: N runs, lower case, newlines
    for i in g.choice(n - 8, size=4000, replace=False):
        text[i:i + int(g.integers(1, 6))] = ord("N")
    low = g.choice(n, size=3000, replace=False)
    text[low] = np.frombuffer(b"acgt", dtype=np.uint8)[codes[low]]
    text[g.choice(n, size=500, replace=False)] = ord("\n")
    tab = pf.Table(pats)
    plan = tab.default_plan(n, "ascii")
    assert plan["depth"] == 9 and plan["hash_bits"] != pf.PFAC_HASH_NONE and plan["prefix"] == 1
    dt = torch.from_numpy(text).to(DEV)
    m_ref, total_ref = oracle.scan(pats, text, threads=16)
    pos, ids = oracle.hits_of(m_ref)
    print("one-hash filter: n=%d patterns=%d hits=%d" % (n, len(pats), pos.size), flush=True)
    r = pf.match(tab, dt, hit_cap=pos.size + 64)
    torch.cuda.synchronize()
    assert np.array_equal(r.match.cpu().numpy(), m_ref)
    assert r.num_hits() == pos.size and r.total() == total_ref
    h = r.hit_list()
    assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)
    # hits only (no dense output: the scan without pre-zeroing)
    r2 = pf.match(tab, dt, hit_cap=pos.size + 64, dense=False)
    torch.cuda.synchronize()
    assert r2.num_hits() == pos.size and r2.total() == total_ref
    assert np.array_equal(r2.hit_list()[:, 0], pos)


def test_deferred_walks_with_patterns_shorter_than_the_filter_depth():
    """Walks kept for the end of the wave on a set with patterns of 3..12
    bases: the depth-D jump entry then passes finals on the way (or leads to
    no state at all past a short pattern), which the deferred and the inline
    walks both count from the jump table's output."""
    g = W.rng(95)
    n = 1 << 20
    text = W.uniform_ascii(n, g).copy()
    pats = W.random_patterns(300, 3, 12, g) + W.cut_patterns(text, 200, 5, 30, g)
    text[g.choice(n, size=2000, replace=False)] = ord("N")
    tab = pf.Table(pats)
    m_ref, total_ref = oracle.scan(pats, text, threads=16)
    pos, ids = oracle.hits_of(m_ref)
    dt = torch.from_numpy(text).to(DEV)
    for plan in ({"walks": pf.PFAC_WALKS_DEFERRED},
                 {"walks": pf.PFAC_WALKS_DEFERRED, "depth": 6},
                 {"walks": pf.PFAC_WALKS_DEFERRED, "depth": 10, "levels": pf.PFAC_LEVELS_NONE},
                 {"walks": pf.PFAC_WALKS_INLINE, "depth": 9, "levels": pf.PFAC_LEVELS_NONE}):
        print("plan", plan, flush=True)
        r = pf.match(tab, dt, hit_cap=pos.size + 64, plan=plan)
        torch.cuda.synchronize()
        assert np.array_equal(r.match.cpu().numpy(), m_ref), plan
        assert r.num_hits() == pos.size and r.total() == total_ref, plan
        h = r.hit_list()
        assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids), plan
        r2 = pf.match(tab, dt, hit_cap=pos.size + 64, plan=plan, dense=False)
        torch.cuda.synchronize()
        assert r2.num_hits() == pos.size and r2.total() == total_ref, plan
        assert np.array_equal(r2.hit_list()[:, 1], ids), plan
