"""Pins for the CPU oracle: worked examples printed in the paper, brute force
on tiny inputs, textbook special cases, an independent k-mer checker and
invariants.  None of these uses the GPU library."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.pointwise import PointOracle
from _checkers import brute, brute_pairs, kmer_check, read_golden

COLS_ACGT = {c: i for i, c in enumerate("ACGT")}


def _pats(s):
    return [p.encode() for p in s.split()]


# ---------------------------------------------------------------- paper examples

def test_fig1_goto_numbering():
    g = read_golden("fig1_goto.txt")
    pats = _pats(g["patterns"])
    go, fin = oracle.goto_function(pats)
    finals = [int(s) for s in g["final_states"].split()]
    assert [int(np.nonzero(fin == k)[0][0]) for k in range(1, len(pats) + 1)] == finals
    assert go.shape[0] == 10          # root + 9 states (Fig. 1)


def test_table1_edges():
    """Every pattern walked through the paper's Table I ends with its own ID,
    and the non-empty cells are exactly the trie's edges (one per state)."""
    g = read_golden("table1.txt")
    pats = _pats(g["patterns"])
    cols = g["columns"].split()
    rows = g["rows"]
    go, fin = oracle.goto_function(pats)
    nonempty = {(r, cols[c]) for r, row in enumerate(rows) for c, cell in enumerate(row)
                if cell != (0, 0)}
    assert len(nonempty) == go.shape[0] - 1      # 14 edges, 15 states incl. root
    used = set()
    for k, p in enumerate(pats, start=1):
        r = 0
        s = 0
        for t, ch in enumerate(p.decode()):
            nxt, pid = rows[r][cols.index(ch)]
            assert nxt != 0
            used.add((r, ch))
            s = go[s, COLS_ACGT[ch]]
            assert s > 0
            last = t == len(p) - 1
            assert (pid == k) == last and (fin[s] == k) == last
            r = nxt
    assert used == nonempty


def test_table1_literal_walker_disagrees_at_reused_state():
    """The reading that Table I's reused state numbers are a slip: a walker
    faithful to the table reports the wrong pattern at position 0."""
    g = read_golden("table1.txt")
    ex = read_golden("ex2_table1_text.txt")
    cols = g["columns"].split()
    rows = g["rows"]
    text = ex["text"]
    r, best = 0, 0
    for ch in text:
        nxt, pid = rows[r][cols.index(ch)]
        if nxt == 0:
            break
        if pid:
            best = pid
        r = nxt
    assert best == int(ex["table_walker_match0"]) == 2
    m, _ = oracle.scan(_pats(ex["patterns"]), text.encode())
    assert m[0] == 1


@pytest.mark.parametrize("name", ["ex1_fig1_text.txt", "ex2_table1_text.txt"])
def test_worked_examples(name):
    ex = read_golden(name)
    pats = _pats(ex["patterns"])
    m, total = oracle.scan(pats, ex["text"].encode())
    assert m.tolist() == [int(x) for x in ex["match"].split()]
    assert total == int(ex["total"])
    bm, bt = brute(pats, ex["text"].encode())
    assert bm == m.tolist() and bt == total


@pytest.mark.parametrize("name", ["ex1_fig1_text.txt", "ex2_table1_text.txt"])
def test_worked_examples_every_occurrence(name):
    """The all-occurrence list and per-position counts on the hand-derived examples."""
    ex = read_golden(name)
    pats = _pats(ex["patterns"])
    text = ex["text"].encode()
    occ = oracle.occurrences(pats, text)
    want = [tuple(int(x) for x in c.split(",")) for c in ex["occurrences"].split()]
    assert [tuple(r) for r in occ.tolist()] == want
    m, total, cnt = oracle.scan(pats, text, counts=True)
    assert int(cnt.sum()) == total == len(want)
    assert cnt.tolist() == [sum(1 for i, _ in want if i == q) for q in range(len(text))]


# ---------------------------------------------------------------- brute force

PATTERN_SETS = [
    [b"A"],
    [b"AC", b"ACG", b"CTGT", b"TG"],
    [b"A", b"AA", b"AAA", b"AAAA"],                   # nested prefixes
    [b"CG", b"ACGT", b"G", b"GT", b"TACG"],             # suffix-only outputs (dictionary links)
    [b"ACG", b"ACG", b"CG", b"CG", b"G"],               # duplicates: smaller ID wins
    [b"TTTTTTTTT", b"GATTACA", b"CAT"],                 # longer than many texts
    [b"AT", b"TA", b"ATA", b"TAT", b"ATAT", b"TATA"],
]


@pytest.mark.parametrize("pset", range(len(PATTERN_SETS)))
def test_exhaustive_short_texts(pset):
    """All texts of length <= 6 over {A,C,G,T}, joined by 'N' separators."""
    pats = PATTERN_SETS[pset]
    texts = []
    for L in range(0, 7):
        texts += ["".join(t) for t in itertools.product("ACGT", repeat=L)]
    big = ("N".join(texts)).encode()
    m, total = oracle.scan(pats, big)
    bm, bt = brute(pats, big)
    assert m.tolist() == bm
    assert total == bt
    occ = oracle.occurrences(pats, big)
    assert [tuple(r) for r in occ.tolist()] == brute_pairs(pats, big)
    m2, t2, cnt = oracle.scan(pats, big, counts=True, threads=3)
    assert m2.tolist() == bm and t2 == bt
    assert cnt.tolist() == np.bincount(occ[:, 0], minlength=len(big)).tolist() if len(occ) else \
        not cnt.any()


def test_random_tiny_cases():
    g = W.rng(12345)
    alphabet = np.frombuffer(b"ACGTACGTACGTNacgt\n", dtype=np.uint8)
    for case in range(400):
        P = int(g.integers(1, 13))
        pats = []
        for _ in range(P):
            if pats and g.random() < 0.25:
                src = pats[int(g.integers(0, len(pats)))]
                cut = int(g.integers(1, len(src) + 1))
                pats.append(src[:cut] if g.random() < 0.5 else src)   # prefix or duplicate
            else:
                L = int(g.integers(1, 9))
                pats.append(W.uniform_ascii(L, g).tobytes())
        n = int(g.integers(0, 80))
        text = alphabet[g.integers(0, alphabet.size, size=n)].tobytes()
        if n and g.random() < 0.5:          # plant a pattern
            p = pats[int(g.integers(0, P))]
            o = int(g.integers(0, n))
            text = (text[:o] + p + text[o:])[:max(n, len(p))]
        m, total = oracle.scan(pats, text)
        bm, bt = brute(pats, text)
        assert m.tolist() == bm, (case, pats, text)
        assert total == bt, (case, pats, text)
        mt, tt = oracle.scan(pats, text, threads=3)
        assert mt.tolist() == bm and tt == bt
        occ = oracle.occurrences(pats, text)
        assert [tuple(r) for r in occ.tolist()] == brute_pairs(pats, text), (case, pats, text)


# ---------------------------------------------------------------- special cases

def test_single_pattern_counts_overlapping_occurrences():
    g = W.rng(7)
    text = W.uniform_ascii(200_000, g).tobytes()
    for p in [b"A", b"ACA", b"AAAA", b"GATTACA", b"ACGTACGTAC"]:
        cnt = 0
        i = text.find(p)
        while i >= 0:
            cnt += 1
            i = text.find(p, i + 1)
        m, total = oracle.scan([p], text)
        assert total == cnt
        assert int((m == 1).sum()) == cnt


def test_equal_length_patterns_are_a_dictionary_lookup():
    g = W.rng(8)
    k = 6
    pats = W.random_patterns(300, k, k, g)
    text = W.uniform_ascii(50_000, g).tobytes()
    first = {}
    for i, p in enumerate(pats, start=1):
        first.setdefault(p, i)
    m, _ = oracle.scan(pats, text)
    exp = [first.get(text[i:i + k], 0) if i + k <= len(text) else 0 for i in range(len(text))]
    assert m.tolist() == exp


def test_pattern_longer_than_text_never_matches():
    m, total = oracle.scan([b"ACGTACGT"], b"ACGTACG")
    assert total == 0 and not m.any()
    m, total = oracle.scan([b"ACGT"], b"")
    assert total == 0 and m.size == 0


def test_invalid_patterns_rejected():
    with pytest.raises(oracle.OracleError) as e:
        oracle.scan([b"ACGT", b"ACNT"], b"ACGT")
    assert e.value.bad_index == 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.scan([b"", b"A"], b"ACGT")
    assert e.value.bad_index == 0
    with pytest.raises(oracle.OracleError):
        oracle.scan([b"acgt"], b"ACGT")


def test_non_acgt_text_bytes_stop_walks():
    m, total = oracle.scan([b"ACGT", b"CG"], b"ACNGTACgTACGT\nACGT")
    bm, bt = brute([b"ACGT", b"CG"], b"ACNGTACgTACGT\nACGT")
    assert m.tolist() == bm and total == bt == 4


# ---------------------------------------------------------------- independent checker

def test_kmer_checker_agrees_on_tiny_workload():
    w = W.plain_workload(0)
    m, total = oracle.scan(w.patterns, w.text)
    km, kt = kmer_check(w.patterns, w.text)
    assert np.array_equal(m, km) and total == kt


def test_kmer_checker_agrees_on_markov_workload():
    w = W.plain_workload(1, n=1 << 19, num_patterns=3000)
    m, total = oracle.scan(w.patterns, w.text, threads=4)
    km, kt = kmer_check(w.patterns, w.text)
    assert np.array_equal(m, km) and total == kt


def test_kmer_checker_agrees_on_short_dense_patterns():
    g = W.rng(99)
    pats = W.random_patterns(2000, 3, 9, g) + W.random_patterns(20, 33, 40, g)
    text = W.uniform_ascii(100_000, g)
    pats += W.cut_patterns(text, 30, 33, 45, g)
    m, total = oracle.scan(pats, text)
    km, kt = kmer_check(pats, text)
    assert np.array_equal(m, km) and total == kt


def test_pointwise_oracle_agrees():
    w = W.plain_workload(0)
    m, total = oracle.scan(w.patterns, w.text)
    po = PointOracle(w.patterns)
    g = W.rng(5)
    hits = np.nonzero(m)[0]
    pos = np.concatenate([hits, g.integers(0, w.n, size=2000), [0, w.n - 1]])
    pm, pc = po.many(w.text, pos)
    assert np.array_equal(pm, m[pos])
    for ex in ["ex1_fig1_text.txt", "ex2_table1_text.txt"]:
        e = read_golden(ex)
        pats = _pats(e["patterns"])
        po = PointOracle(pats)
        text = e["text"].encode()
        pm, pc = po.many(text, range(len(text)))
        assert pm.tolist() == [int(x) for x in e["match"].split()]
        assert int(pc.sum()) == int(e["total"])


# ---------------------------------------------------------------- invariants

def test_invariants_on_tiny_workload():
    w = W.plain_workload(0)
    m, total = oracle.scan(w.patterns, w.text)
    text = w.text.tobytes()
    lens = np.array([len(p) for p in w.patterns])
    hits = np.nonzero(m)[0]
    assert total >= hits.size > 0
    for i in hits:
        k = int(m[i])
        assert text[i:i + lens[k - 1]] == w.patterns[k - 1]
        # no longer pattern starts here
        for q, p in enumerate(w.patterns, start=1):
            if len(p) > lens[k - 1]:
                assert text[i:i + len(p)] != p
    # every planted pattern (the first half) is reported with at least its length
    for p in w.patterns[:50]:
        o = text.find(p)
        assert o >= 0 and m[o] != 0 and lens[m[o] - 1] >= len(p)


def test_multithreaded_scan_is_identical():
    w = W.plain_workload(1, n=1 << 20, num_patterns=2000)
    m1, t1 = oracle.scan(w.patterns, w.text)
    for th in (2, 7, 16):
        m2, t2 = oracle.scan(w.patterns, w.text, threads=th)
        assert np.array_equal(m1, m2) and t1 == t2


def test_markov_generator_is_stationary_and_seeded():
    g = W.rng(1)
    P = W.markov_matrix(g)
    pi = np.array([0.295, 0.205, 0.205, 0.295])
    assert np.allclose(pi @ P, pi, atol=1e-12)
    a = W.plain_workload(1, n=100_000, num_patterns=10).text
    b = W.plain_workload(1, n=100_000, num_patterns=10).text
    assert np.array_equal(a, b)
    codes = W.ascii_to_codes(W.plain_workload(1, n=1 << 20, num_patterns=10).text)
    gc = float(np.isin(codes, [1, 2]).mean())
    assert abs(gc - 0.41) < 0.02


def test_markov_blocked_sampler_equals_sequential_chain():
    """The blocked sampler is the sequential chain for the same random bytes."""
    g = W.rng(3)
    P = W.markov_matrix(g)
    out = W.markov_codes(10_000, W.rng(77), P, block=64)
    # replay sequentially with the same byte stream
    g2 = W.rng(77)
    pi = np.linalg.eig(P.T)
    cum = np.cumsum(P, axis=1)
    u_mid = (np.arange(256) + 0.5) / 256.0
    step = np.stack([np.minimum(np.searchsorted(cum[s], u_mid, side="right"), 3) for s in range(4)])
    w, v = pi
    st = np.real(v[:, np.argmin(np.abs(w - 1))])
    st = st / st.sum()
    x = min(int(np.searchsorted(np.cumsum(st), g2.random(), side="right")), 3)
    nb = (10_000 + 63) // 64
    u = g2.integers(0, 256, size=(64, nb), dtype=np.uint8)
    seq = []
    for b in range(nb):
        for t in range(64):
            x = int(step[x, u[t, b]])
            seq.append(x)
    assert np.array_equal(out, np.array(seq[:10_000], dtype=np.uint8))


def test_pack2bit_layout():
    codes = np.array([0, 1, 2, 3, 3, 2], dtype=np.uint8)   # A C G T T G
    p = W.pack2bit(codes)
    assert p.tolist() == [0b11100100, 0b1011]
    assert W.unpack2bit_ascii(p, 0, 6).tobytes() == b"ACGTTG"
    assert W.unpack2bit_ascii(p, 3, 2).tobytes() == b"TT"


# ---------------------------------------------------------------- byte alphabet

def test_byte_alphabet_worked_example():
    ex = read_golden("bytes_ushers.txt")
    pats = _pats(ex["patterns"])
    m, total = oracle.scan_bytes(pats, ex["text"].encode())
    assert m.tolist() == [int(x) for x in ex["match"].split()]
    assert total == int(ex["total"])
    occ = oracle.occurrences(pats, ex["text"].encode(), alphabet="bytes")
    want = [tuple(int(x) for x in c.split(",")) for c in ex["occurrences"].split()]
    assert [tuple(r) for r in occ.tolist()] == want


def test_byte_alphabet_against_brute_force():
    """Random byte patterns (any of 256 values, small alphabets for many
    matches, nested prefixes and duplicates) over random byte texts."""
    g = W.rng(4321)
    for case in range(300):
        k = int(g.integers(2, 257)) if case % 3 else 3
        symbols = g.choice(256, size=min(k, 256), replace=False).astype(np.uint8)
        P = int(g.integers(1, 15))
        pats = []
        for _ in range(P):
            if pats and g.random() < 0.3:
                src = pats[int(g.integers(0, len(pats)))]
                pats.append(src[:int(g.integers(1, len(src) + 1))])
            else:
                pats.append(symbols[g.integers(0, symbols.size, size=int(g.integers(1, 7)))]
                            .tobytes())
        n = int(g.integers(0, 120))
        text = symbols[g.integers(0, symbols.size, size=n)].tobytes()
        m, total = oracle.scan_bytes(pats, text, threads=1 + case % 3)
        bm, bt = brute(pats, text)
        assert m.tolist() == bm and total == bt, (case, pats, text)
        occ = oracle.occurrences(pats, text, alphabet="bytes")
        assert [tuple(r) for r in occ.tolist()] == brute_pairs(pats, text), case


def test_byte_alphabet_agrees_with_dna_oracle_on_dna():
    """On A, C, G, T only (no other byte in text or patterns) the two
    alphabets define the same thing."""
    w = W.plain_workload(0, n=100_000)
    m1, t1 = oracle.scan(w.patterns, w.text)
    m2, t2 = oracle.scan_bytes(w.patterns, w.text, threads=4)
    assert np.array_equal(m1, m2) and t1 == t2
    with pytest.raises(oracle.OracleError):
        oracle.scan_bytes([b"AC", b""], b"ACGT")          # empty pattern
