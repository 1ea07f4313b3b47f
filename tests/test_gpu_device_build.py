"""The table built on the device against the host build: every array of the
one device allocation byte for byte (so every plan reads the same table),
the planner's metadata, and matching results against the oracle -- also for
tables updated by adding and removing patterns."""
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


def _sets():
    g = W.rng(1400)
    fig1 = [p.encode() for p in read_golden("fig1_goto.txt")["patterns"].split()]
    text = W.uniform_ascii(200_000, g)
    nested = W.cut_patterns(text, 300, 14, 40, g)
    nested += [p[:L] for p in nested[:100] for L in range(7, len(p), 5)] + nested[:50]
    return {
        "fig1": fig1,
        "tiny": W.plain_workload(0, n=100_000).patterns,
        "short": W.random_patterns(3000, 3, 9, g) + [b"A", b"ACGT", b"ACGT"],
        "nested_dups": nested,
        "min7": W.random_patterns(5000, 7, 20, g),
        "min12_long": W.random_patterns(20000, 12, 64, g) + [b"T" * 64, b"A" * 64, b"A" * 63],
        "markov10k": W.plain_workload(1, n=2_000_000).patterns,
    }


SETS = _sets()


@pytest.mark.parametrize("name", sorted(SETS))
def test_device_build_equals_host_build_byte_for_byte(name):
    pats = SETS[name]
    th = pf.Table(pats)
    td = pf.Table(pats, on_device=True)
    print(name, "patterns", len(pats), "states", th.num_states, "bytes", th.device_bytes,
          flush=True)
    assert td.num_states == th.num_states and td.device_bytes == th.device_bytes
    assert td.states_to_depth == th.states_to_depth and td.max_depth_full == th.max_depth_full
    bh, bd = th.blob(), td.blob()
    diff = np.nonzero(bh != bd)[0]
    assert diff.size == 0, "first differing byte %d of %d" % (diff[0], bh.size)
    for n in (None, 1000):
        assert td.default_plan() == th.default_plan()


def test_device_build_of_the_packed_big_trie_set():
    w = W.plain_workload(2, n=4_000_000)
    th = pf.Table(w.patterns)
    td = pf.Table(w.patterns, on_device=True)
    assert np.array_equal(th.blob(), td.blob())
    dt = torch.from_numpy(w.text).to(DEV)
    r = pf.match(td, dt, n=w.n, enc="2bit", hit_cap=w.n // 8)
    torch.cuda.synchronize()
    m_ref, total_ref = oracle.scan(w.patterns, w.ascii(), threads=16)
    assert np.array_equal(r.match.cpu().numpy(), m_ref) and r.total() == total_ref


def _oracle_with_ids(pairs, text):
    """Oracle over (pattern, id) pairs: patterns handed to it in ascending ID
    order (so its smallest-index rule is the smallest-ID rule), its indices
    mapped back to the IDs."""
    pairs = sorted(pairs, key=lambda x: x[1])
    m, total = oracle.scan([p for p, _ in pairs], text, threads=8)
    idmap = np.array([0] + [i for _, i in pairs], dtype=np.int64)
    return idmap[m].astype(np.int32), total


def test_update_adds_and_removes_patterns():
    g = W.rng(1401)
    text = W.uniform_ascii(2_000_003, g)
    base = W.cut_patterns(text, 3000, 12, 40, g) + W.random_patterns(3000, 12, 40, g)
    tab = pf.Table(base)
    add = W.cut_patterns(text, 1500, 10, 50, g) + base[:20]          # some copies of old ones
    remove = [int(x) for x in g.choice(np.arange(1, len(base) + 1), size=800, replace=False)]
    new = tab.update(add=add, remove_ids=remove)
    assert new.first_new_id == len(base) + 1
    keep = set(range(1, len(base) + 1)) - set(remove)
    pairs = [(base[i - 1], i) for i in sorted(keep)] + [(p, new.first_new_id + k)
                                                        for k, p in enumerate(add)]
    dt = torch.from_numpy(text).to(DEV)
    m_ref, total_ref = _oracle_with_ids(pairs, text)
    for plan in (None, dict(variant=pf.PFAC_VARIANT_GLOBAL), dict(walks=pf.PFAC_WALKS_INLINE)):
        r = pf.match(new, dt, plan=plan, hit_cap=text.size)
        torch.cuda.synchronize()
        m = r.match.cpu().numpy()
        bad = np.nonzero(m != m_ref)[0]
        assert bad.size == 0, (plan, bad[0], m[bad[0]], m_ref[bad[0]])
        assert r.total() == total_ref
    # the base table is unchanged and still matches its own set
    rb = pf.match(tab, dt)
    torch.cuda.synchronize()
    mb, tb = oracle.scan(base, text, threads=8)
    assert np.array_equal(rb.match.cpu().numpy(), mb) and rb.total() == tb
    # updating again from the updated table
    newer = new.update(add=[b"ACGTACGTACGTACGT"], remove_ids=[new.first_new_id])
    assert newer.first_new_id == new.first_new_id + len(add)
    pairs2 = [(p, i) for p, i in pairs if i != new.first_new_id] + [(b"ACGTACGTACGTACGT",
                                                                     newer.first_new_id)]
    r2 = pf.match(newer, dt, hit_cap=text.size)
    torch.cuda.synchronize()
    m2, t2 = _oracle_with_ids(pairs2, text)
    assert np.array_equal(r2.match.cpu().numpy(), m2) and r2.total() == t2
    # all occurrences on an updated table (duplicate IDs across old and new)
    ra = pf.match_all(new, dt[:300_000])
    torch.cuda.synchronize()
    occ = ra.occurrences()
    assert ra.total() == len(occ)


def test_device_build_rejections():
    with pytest.raises(pf.PfacError) as e:
        pf.Table([b"ACGT", b"A" * 65], on_device=True)
    assert e.value.bad_index == 1
    with pytest.raises(pf.PfacError) as e:
        pf.Table([b"ACGT", b"ACNT"], on_device=True)
    assert e.value.bad_index == 1 and e.value.code == -2
    tab = pf.Table([b"ACGT"])
    with pytest.raises(pf.PfacError):
        tab.update(remove_ids=[1])                          # nothing left
