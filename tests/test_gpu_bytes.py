"""GPU parity of the byte-alphabet tables (every byte value a symbol,
hash-compressed transition table) against the byte-alphabet oracle:
match array, occurrence total and the ordered hit list."""
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


def _check(pats, text, dense=True, table=None, grid=None):
    t = np.asarray(text, dtype=np.uint8)
    tab = table or pf.Table(pats, alphabet="bytes")
    dt = torch.from_numpy(t.copy()).to(DEV)
    plan = dict(grid=grid) if grid else None
    res = pf.match(tab, dt, dense=dense, hit_cap=t.size + 16, plan=plan)
    torch.cuda.synchronize()
    m_ref, total_ref = oracle.scan_bytes(pats, t, threads=8)
    if dense:
        m = res.match.cpu().numpy()
        bad = np.nonzero(m != m_ref)[0]
        assert bad.size == 0, "first mismatch at %d: gpu %d oracle %d" % (bad[0], m[bad[0]],
                                                                           m_ref[bad[0]])
    assert res.total() == total_ref
    pos, ids = oracle.hits_of(m_ref)
    assert res.num_hits() == pos.size
    h = res.hit_list()
    assert np.array_equal(h[:, 0], pos) and np.array_equal(h[:, 1], ids)
    return res


def test_worked_example():
    ex = read_golden("bytes_ushers.txt")
    pats = [p.encode() for p in ex["patterns"].split()]
    res = _check(pats, np.frombuffer(ex["text"].encode(), dtype=np.uint8))
    assert res.match.cpu().numpy().tolist() == [int(x) for x in ex["match"].split()]


@pytest.mark.parametrize("k", [2, 5, 20, 256])
def test_random_bytes_every_alphabet_size(k):
    """k distinct byte values (a small k gives long walks and dense hits),
    nested prefixes and duplicates, ragged length."""
    g = W.rng(1300 + k)
    syms = g.choice(256, size=k, replace=False).astype(np.uint8)
    pats = [syms[g.integers(0, k, size=int(g.integers(1, 12)))].tobytes() for _ in range(3000)]
    pats += [p[:max(1, len(p) // 2)] for p in pats[:500]] + pats[:200]
    text = syms[g.integers(0, k, size=1_000_003)]
    for i in range(0, 400):                       # plant some long patterns
        p = np.frombuffer(pats[i], dtype=np.uint8)
        o = int(g.integers(0, text.size - p.size))
        text[o:o + p.size] = p
    print("k", k, "patterns", len(pats), flush=True)
    _check(pats, text)
    _check(pats, text, dense=False)
    _check(pats, text, grid=3)


def test_iupac_and_case_patterns_on_dna_text():
    """Patterns with IUPAC codes and lower case as plain bytes: they match
    only those exact bytes."""
    g = W.rng(1310)
    alpha = np.frombuffer(b"ACGTacgtNRYKMSW", dtype=np.uint8)
    text = alpha[g.integers(0, alpha.size, size=500_001)]
    pats = [alpha[g.integers(0, alpha.size, size=int(g.integers(2, 9)))].tobytes()
            for _ in range(5000)]
    _check(pats, text)


def test_dna_patterns_agree_with_the_dna_table():
    """On A, C, G, T texts the byte table and the DNA table give the same."""
    w = W.plain_workload(0, n=700_001)
    rb = _check(w.patterns, w.text)
    tab = pf.Table(w.patterns)
    rd = pf.match(tab, torch.from_numpy(w.text).to(DEV))
    torch.cuda.synchronize()
    assert torch.equal(rb.match, rd.match) and rb.total() == rd.total()


def test_byte_table_rejections():
    with pytest.raises(pf.PfacError):
        pf.Table([b"ab", b""], alphabet="bytes")
    tab = pf.Table([b"ab", b"\x00\xff"], alphabet="bytes")
    base = torch.zeros(64, dtype=torch.uint8, device=DEV)
    with pytest.raises(pf.PfacError):
        pf.match(tab, base, n=64, enc="2bit")
    with pytest.raises(pf.PfacError):
        pf.match_batch([tab], base, [0], [10])
    with pytest.raises(pf.PfacError):
        pf.match(tab, base, plan=dict(depth=8))
    r = pf.match(tab, torch.zeros(0, dtype=torch.uint8, device=DEV), n=0)
    torch.cuda.synchronize()
    assert r.counters.cpu().tolist() == [0, 0]
