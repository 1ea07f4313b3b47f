"""CPU tests of the library's host side: the C ABI loads and exports every
declared symbol, and the host-built table (breadth-first numbering, packed
edges, root jump tables) reproduces the oracle when walked."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W
from _checkers import read_golden

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FINAL = 0x80000000
MASK = 0x7FFFFFFF


def _lib():
    from paper_1811_10498_amd import _lib as L
    return L.lib()


def test_library_exports_every_declared_symbol():
    lib = _lib()
    declared = set()
    inc = os.path.join(ROOT, "include")
    for name in os.listdir(inc):
        if name.endswith(".h"):
            src = open(os.path.join(inc, name)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            declared |= set(re.findall(r"^\s*(?:const\s+)?[\w ]+\*?\s*\b(pfac_\w+)\s*\(", src,
                                       flags=re.M))
    assert {"pfac_build_table", "pfac_match", "pfac_match_batch", "pfac_batch_create",
            "pfac_batch_launch", "pfac_batch_free"} <= declared
    for sym in sorted(declared):
        assert hasattr(lib, sym), sym
    assert lib.pfac_version().decode().startswith("pfac")
    assert lib.pfac_strerror(-2).decode()


def host_table(patterns, K=None):
    lib = _lib()
    pats = [bytes(p) for p in patterns]
    bufs = [ctypes.create_string_buffer(p, max(1, len(p))) for p in pats]
    arr = (ctypes.c_void_p * len(pats))(*[ctypes.addressof(b) for b in bufs])
    lens = (ctypes.c_uint32 * len(pats))(*[len(p) for p in pats])
    S = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    rc = lib.pfac_build_host(ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(lens, ctypes.c_void_p),
                             len(pats), None, None, None, 0, 0, None, None, None,
                             ctypes.byref(S), ctypes.byref(bad))
    if rc != 0:
        return rc, bad.value, None
    cap = S.value
    nxt = np.zeros(4 * cap, dtype=np.uint32)
    pid = np.zeros(cap, dtype=np.int32)
    mult = np.zeros(cap, dtype=np.uint32)
    jump = jpid = jcnt = None
    if K:
        jump = np.zeros(4 ** K, dtype=np.uint32)
        jpid = np.zeros(4 ** K, dtype=np.int32)
        jcnt = np.zeros(4 ** K, dtype=np.uint32)
    rc = lib.pfac_build_host(ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(lens, ctypes.c_void_p),
                             len(pats), nxt.ctypes.data, pid.ctypes.data, mult.ctypes.data, cap,
                             K or 0, jump.ctypes.data if K else None,
                             jpid.ctypes.data if K else None, jcnt.ctypes.data if K else None,
                             ctypes.byref(S), ctypes.byref(bad))
    assert rc == 0
    return 0, -1, dict(next=nxt.reshape(-1, 4), pid=pid, mult=mult, jump=jump, jpid=jpid,
                       jcnt=jcnt, S=cap)


CODE = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}


def _pattern_arrays(patterns):
    pats = [bytes(p) for p in patterns]
    bufs = [ctypes.create_string_buffer(p, max(1, len(p))) for p in pats]
    arr = (ctypes.c_void_p * len(pats))(*[ctypes.addressof(b) for b in bufs])
    lens = (ctypes.c_uint32 * len(pats))(*[len(p) for p in pats])
    return ctypes.cast(arr, ctypes.c_void_p), ctypes.cast(lens, ctypes.c_void_p), bufs


def walk_all(t, text):
    """PFAC walk (paper Sec. IV) over the host table, every start position."""
    text = bytes(text)
    n = len(text)
    m = np.zeros(n, dtype=np.int32)
    total = 0
    nxt, pid, mult = t["next"], t["pid"], t["mult"]
    for i in range(n):
        s = 0
        for q in range(i, n):
            c = CODE.get(text[q])
            if c is None:
                break
            e = int(nxt[s, c])
            if e == 0:
                break
            s = e & MASK
            if e & FINAL:
                m[i] = pid[s]
                total += int(mult[s])
    return m, total


def test_fig1_breadth_first_numbering():
    g = read_golden("fig1_goto.txt")
    pats = [p.encode() for p in g["patterns"].split()]
    rc, _, t = host_table(pats)
    assert rc == 0 and t["S"] == 10
    # breadth-first: depth 1 = A, C, T; depth 2 = AC, CT, TG; depth 3 = ACG, CTG; depth 4 = CTGT
    finals = {int(t["pid"][s]): s for s in range(t["S"]) if t["pid"][s]}
    assert finals == {1: 4, 2: 7, 3: 9, 4: 6}
    # every edge points to a larger state number and the state depth never decreases
    depth = np.zeros(t["S"], dtype=int)
    for s in range(t["S"]):
        for a in range(4):
            e = int(t["next"][s, a])
            if e:
                assert (e & MASK) > s
                depth[e & MASK] = depth[s] + 1
                assert bool(e & FINAL) == bool(t["pid"][e & MASK])
    assert np.all(np.diff(depth) >= 0)


def test_walking_host_table_reproduces_oracle_small():
    g = W.rng(41)
    for case in range(60):
        pats = W.random_patterns(int(g.integers(1, 20)), 1, 7, g)
        if case % 3 == 0:
            pats += pats[: 3]          # duplicates
        text = W.uniform_ascii(int(g.integers(0, 400)), g)
        if text.size > 10:
            text[int(g.integers(0, text.size))] = ord("N")
        rc, _, t = host_table(pats)
        assert rc == 0
        m, total = walk_all(t, text)
        mr, tr = oracle.scan(pats, text)
        assert np.array_equal(m, mr) and total == tr


def test_walking_host_table_reproduces_oracle_workload():
    w = W.plain_workload(0, n=20_000)
    rc, _, t = host_table(w.patterns)
    m, total = walk_all(t, w.text)
    mr, tr = oracle.scan(w.patterns, w.text)
    assert np.array_equal(m, mr) and total == tr


@pytest.mark.parametrize("K", [6, 7, 8])
def test_root_jump_table_is_the_k_step_walk(K):
    g = W.rng(50 + K)
    pats = W.random_patterns(300, 1, 12, g) + [b"A" * 3, b"ACG", b"ACG"]
    rc, _, t = host_table(pats, K=K)
    nxt, pid, mult = t["next"], t["pid"], t["mult"]
    for x in range(4 ** K):
        s, best, cnt, alive, fin = 0, 0, 0, True, False
        for d in range(K):
            e = int(nxt[s, (x >> (2 * (K - 1 - d))) & 3])
            if e == 0:
                alive = False
                break
            s = e & MASK
            if e & FINAL:
                fin = True
                best = int(pid[s])
                cnt += int(mult[s])
        j = int(t["jump"][x])
        assert (j & MASK) == (s if alive else 0)
        assert bool(j & FINAL) == fin
        if fin:
            assert t["jpid"][x] == best and t["jcnt"][x] == cnt


def test_host_build_rejects_bad_patterns():
    rc, bad, _ = host_table([b"ACGT", b"AC-T"])
    assert rc == -2 and bad == 1
    rc, bad, _ = host_table([b"ACGT", b""])
    assert rc == -2 and bad == 1
    rc, bad, _ = host_table([b"acgt"])
    assert rc == -2 and bad == 0


def test_state_counts_of_workload_tries():
    """Trie sizes of the benchmark pattern sets (recorded in the design notes)."""
    w = W.plain_workload(0)
    rc, _, t = host_table(w.patterns)
    assert 2000 < t["S"] < 3500


def host_image(patterns, D):
    lib = _lib()
    pats = [bytes(p) for p in patterns]
    bufs = [ctypes.create_string_buffer(p, max(1, len(p))) for p in pats]
    arr = (ctypes.c_void_p * len(pats))(*[ctypes.addressof(b) for b in bufs])
    lens = (ctypes.c_uint32 * len(pats))(*[len(p) for p in pats])
    nw = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    rc = lib.pfac_build_host_image(ctypes.cast(arr, ctypes.c_void_p),
                                   ctypes.cast(lens, ctypes.c_void_p), len(pats), D, None, 0,
                                   None, ctypes.byref(nw), ctypes.byref(bad))
    assert rc == 0
    words = np.zeros(nw.value, dtype=np.uint32)
    meta = np.zeros(1 + 3 * 8, dtype=np.uint32)
    rc = lib.pfac_build_host_image(ctypes.cast(arr, ctypes.c_void_p),
                                   ctypes.cast(lens, ctypes.c_void_p), len(pats), D,
                                   words.ctypes.data, nw.value, meta.ctypes.data,
                                   ctypes.byref(nw), ctypes.byref(bad))
    assert rc == 0
    return words, meta


@pytest.mark.parametrize("D,npat,lmin,lmax", [(6, 400, 8, 20), (7, 3000, 9, 16), (8, 5000, 10, 24)])
def test_lds_image_navigation_matches_next_table(D, npat, lmin, lmax):
    """Rank-based navigation of the LDS image (filter bitmap rank -> level-D
    node, child-bit counts -> deeper nodes) reaches exactly the states of the
    breadth-first next-state table."""
    g = W.rng(60 + D)
    text = W.uniform_ascii(50_000, g)
    pats = W.cut_patterns(text, npat // 2, lmin, lmax, g) + W.random_patterns(npat // 2, lmin, lmax, g)
    _, _, t = host_table(pats)
    words, meta = host_image(pats, D)
    levels = int(meta[0])
    assert levels >= 1
    nxt = t["next"]
    bm = words[:4 ** D // 32]
    pre = words[4 ** D // 32: 4 ** D // 32 + 4 ** D // 128]
    # depth of every state and the first state of each level (breadth-first)
    depth = np.zeros(t["S"], dtype=np.int64)
    for s in range(t["S"]):
        for a in range(4):
            e = int(nxt[s, a])
            if e:
                depth[e & MASK] = depth[s] + 1
    first = {int(d): int(np.nonzero(depth == d)[0][0]) for d in np.unique(depth)}

    def byte_of(k, j):
        w = int(words[int(meta[1 + 3 * k]) + (j >> 2)])
        return (w >> (8 * (j & 3))) & 0xFF

    def child_index(k, j, c):
        b = byte_of(k, j)
        cnt = int(words[int(meta[2 + 3 * k]) + (j >> 4)])
        for jj in range(j & ~15, j):
            cnt += bin(byte_of(k, jj) & 15).count("1")
        return cnt + bin(b & ((1 << c) - 1)).count("1")

    checked = 0
    for start in range(0, text.size - D - levels, 7):
        win = text[start:start + D + levels]
        codes = [b"ACGT".index(bytes([x])) for x in win]
        x = 0
        for c in codes[:D]:
            x = (x << 2) | c
        # reference: walk the next table
        s = 0
        ok = True
        for c in codes[:D]:
            e = int(nxt[s, c])
            if e == 0:
                ok = False
                break
            s = e & MASK
        bit = (int(bm[x >> 5]) >> (x & 31)) & 1
        assert bit == int(ok)
        if not ok:
            continue
        j = int(pre[x >> 7]) + sum(bin(int(bm[(x >> 5) & ~3 | w])).count("1") for w in range((x >> 5) & 3))
        j += bin(int(bm[x >> 5]) & ((1 << (x & 31)) - 1)).count("1")
        assert first[D] + j == s
        for k in range(levels - 1):
            c = codes[D + k]
            b = byte_of(k, j)
            assert bool(b & 16) == bool(t["pid"][s])
            e = int(nxt[s, c])
            assert bool((b >> c) & 1) == bool(e)
            if not e:
                break
            s = e & MASK
            j = child_index(k, j, c)
            assert first[D + k + 1] + j == s
            checked += 1
    assert checked > 50


@pytest.mark.parametrize("bits", [12, 14, 18, 19, 20])
def test_second_filter_bitmap_holds_every_pattern_prefix(bits):
    """The hash bitmap (its definition is part of the public header) has the
    two bits of the first K bases of every pattern; smaller bitmaps are the
    OR-fold of the largest; random windows pass at about the square of the
    fraction of set bits."""
    import ctypes
    from paper_1811_10498_amd import _lib as L
    lib = L.lib()
    g = W.rng(81)
    pats = W.random_patterns(3000, 16, 40, g) + [b"ACGTACGTACGTACGTA"]
    arr, lens, keep = _pattern_arrays(pats)
    def get(b):
        words = np.zeros((1 << b) // 32, dtype=np.uint32)
        k = ctypes.c_uint32(0)
        bad = ctypes.c_int64(-1)
        rc = lib.pfac_build_host_hash(arr, lens, len(pats), b, words.ctypes.data,
                                      ctypes.byref(k), ctypes.byref(bad))
        assert rc == 0
        return words, k.value
    words, K = get(bits)
    assert K == 16
    def h(key, b, mul=0x9E3779B1):
        return ((key * mul) & 0xFFFFFFFF) >> (32 - b)
    code = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}
    for p in pats:
        key = 0
        for i in range(K):
            key |= code[p[i]] << (30 - 2 * i)
        for mul in (0x9E3779B1, 0x85EBCA77):
            x = h(key, bits, mul)
            assert (words[x >> 5] >> (x & 31)) & 1
    big, _ = get(20)
    bigbits = np.unpackbits(big.view(np.uint8), bitorder="little").astype(bool)
    folded = bigbits.reshape(1 << bits, 1 << (20 - bits)).any(axis=1)
    mine = np.unpackbits(words.view(np.uint8), bitorder="little").astype(bool)
    assert np.array_equal(folded, mine)
    keys = g.integers(0, 1 << 32, size=20000, dtype=np.uint64)
    def hv(mul):
        x = ((keys * np.uint64(mul)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - bits)
        return mine[x.astype(np.int64)]
    rate = (hv(0x9E3779B1) & hv(0x85EBCA77)).mean()      # both bits: about f^2
    assert abs(rate - mine.mean() ** 2) < 0.03


def test_one_hash_second_filter_bits_and_folds():
    """The one-hash form (K <= 12): every pattern's bit is set, smaller sizes
    are the OR-fold of the largest, random keys pass at about its fill, and a
    set whose shortest pattern is longer than 12 bases has no such bitmap."""
    import ctypes
    from paper_1811_10498_amd import _lib as L
    lib = L.lib()
    g = W.rng(83)
    pats = W.random_patterns(5000, 12, 30, g)
    arr, lens, keep = _pattern_arrays(pats)
    def get(b, ps=None):
        a, l, kp = (arr, lens, keep) if ps is None else _pattern_arrays(ps)
        n = len(pats) if ps is None else len(ps)
        words = np.zeros((1 << b) // 32, dtype=np.uint32)
        k = ctypes.c_uint32(0)
        bad = ctypes.c_int64(-1)
        rc = lib.pfac_build_host_hash1(a, l, n, b, words.ctypes.data, ctypes.byref(k),
                                       ctypes.byref(bad))
        del kp
        return rc, words, k.value
    rc, words, K = get(16)
    assert rc == 0 and K == 12
    code = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}
    for p in pats:
        key = 0
        for i in range(K):
            key = (key << 2) | code[p[i]]
        x = ((key * 0xC6A4A7) & 0xFFFFFFFF) >> (32 - 16)
        assert (words[x >> 5] >> (x & 31)) & 1
    _, big, _ = get(20)
    bigbits = np.unpackbits(big.view(np.uint8), bitorder="little").astype(bool)
    folded = bigbits.reshape(1 << 16, 1 << 4).any(axis=1)
    mine = np.unpackbits(words.view(np.uint8), bitorder="little").astype(bool)
    assert np.array_equal(folded, mine)
    keys = g.integers(0, 1 << 24, size=20000, dtype=np.uint64)
    x = ((keys * np.uint64(0xC6A4A7)) & np.uint64(0xFFFFFFFF)) >> np.uint64(16)
    assert abs(mine[x.astype(np.int64)].mean() - mine.mean()) < 0.03
    rc, w13, K13 = get(16, [b"ACGTACGTACGTA", b"CCCCCCCCCCCCCCCCCC"])
    assert K13 == 13 and rc != 0 and not w13.any()


def test_second_filter_k_is_shortest_pattern_capped_at_16():
    import ctypes
    from paper_1811_10498_amd import _lib as L
    lib = L.lib()
    for pats, want in [([b"ACGTACGTACGT", b"ACGTACGTACGTACGTACGT"], 12),
                       ([b"A" * 30, b"C" * 20], 16)]:
        arr, lens, keep = _pattern_arrays(pats)
        k = ctypes.c_uint32(0)
        bad = ctypes.c_int64(-1)
        assert lib.pfac_build_host_hash(arr, lens, len(pats), 12, None, ctypes.byref(k),
                                        ctypes.byref(bad)) == 0
        assert k.value == want


def host_chain(patterns):
    lib = _lib()
    arr, lens, keep = _pattern_arrays(patterns)
    S = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    assert lib.pfac_build_host_chain(arr, lens, len(patterns), None, 0, ctypes.byref(S),
                                     ctypes.byref(bad)) == 0
    chain = np.zeros(2 * S.value, dtype=np.uint32)
    assert lib.pfac_build_host_chain(arr, lens, len(patterns), chain.ctypes.data, S.value,
                                     ctypes.byref(S), ctypes.byref(bad)) == 0
    return chain.reshape(-1, 2)


def walk_all_with_runs(t, chain, text):
    """Walk every start position taking runs of single-child steps at once
    (the kernel's deep walk), on the host tables."""
    codes = [CODE.get(int(b), -1) for b in text]
    n = len(codes)
    out = np.zeros(n, dtype=np.int32)
    total = 0
    for i in range(n):
        s, q, best = 0, i, 0
        while True:
            cx, cy = int(chain[s, 0]), int(chain[s, 1])
            L = cx & 15
            if L >= 2:
                ok = q + L <= n and all(codes[q + k] == (cx >> (30 - 2 * k)) & 3
                                        for k in range(L))
                if not ok:
                    break
                s = cy & 0x7FFFFFFF
                q += L
                if cy >> 31:
                    best = int(t["pid"][s])
                    total += int(t["mult"][s])
                continue
            if q >= n or codes[q] < 0:
                break
            e = int(t["next"][s, codes[q]])
            if e == 0:
                break
            s = e & 0x7FFFFFFF
            if e >> 31:
                best = int(t["pid"][s])
                total += int(t["mult"][s])
            q += 1
        out[i] = best
    return out, total


def test_runs_of_single_child_steps_are_well_formed():
    """Every run record: its bases follow single-child edges of the next
    table, every state strictly inside is non-final with one child, it ends
    where the record says, with the right final bit."""
    g = W.rng(91)
    pats = W.random_patterns(200, 10, 60, g) + [b"A" * 50, b"A" * 20, b"ACGT" * 10]
    rc, _, t = host_table(pats)
    chain = host_chain(pats)
    nxt = t["next"]
    runs = 0
    for s in range(t["S"]):
        cx, cy = int(chain[s, 0]), int(chain[s, 1])
        L = cx & 15
        if L < 2:
            continue
        runs += 1
        assert L <= 14
        cur = s
        for k in range(L):
            kids = [a for a in range(4) if nxt[cur, a]]
            assert len(kids) == 1, (s, k)
            a = (cx >> (30 - 2 * k)) & 3
            assert kids == [a]
            e = int(nxt[cur, a])
            cur = e & 0x7FFFFFFF
            fin = bool(e >> 31)
            if k < L - 1:
                assert not fin and bin(int(sum(1 for b in range(4) if nxt[cur, b]))).count("1")
        assert cur == (cy & 0x7FFFFFFF) and fin == bool(cy >> 31)
    assert runs > 100


def test_walking_with_runs_reproduces_oracle():
    g = W.rng(92)
    text = W.uniform_ascii(4000, g)
    pats = (W.cut_patterns(text, 60, 12, 60, g) + W.random_patterns(40, 5, 30, g)
            + [bytes(text[100:160]), bytes(text[100:130]), bytes(text[100:116])])
    text[700] = ord("N")
    rc, _, t = host_table(pats)
    chain = host_chain(pats)
    m, total = walk_all_with_runs(t, chain, text)
    m_ref, total_ref = oracle.scan(pats, text)
    assert np.array_equal(m, m_ref) and total == total_ref


@pytest.mark.parametrize("lmin,want_k", [(12, 12), (9, 9), (20, 12), (6, 0)])
def test_prefix_filter_bitmap_is_the_set_of_pattern_prefixes(lmin, want_k):
    """The prefix bitmap has exactly the bits of the patterns' first K2 bases
    (K2 = min(shortest pattern, 12), none below 7 bases)."""
    import ctypes
    from paper_1811_10498_amd import _lib as L
    lib = L.lib()
    g = W.rng(90 + lmin)
    pats = W.random_patterns(5000, lmin, lmin + 20, g) + [b"A" * lmin, b"T" * (lmin + 3)]
    arr, lens, keep = _pattern_arrays(pats)
    k = ctypes.c_uint32(0)
    nk = ctypes.c_uint64(0)
    bad = ctypes.c_int64(-1)
    words = np.zeros(1 << 19, dtype=np.uint32)
    rc = lib.pfac_build_host_prefix(arr, lens, len(pats), words.ctypes.data, words.size,
                                    ctypes.byref(k), ctypes.byref(nk), ctypes.byref(bad))
    assert rc == 0 and k.value == want_k
    if want_k == 0:
        assert nk.value == 0
        return
    K = want_k
    code = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}
    keys = set()
    for p in pats:
        x = 0
        for i in range(K):
            x = (x << 2) | code[p[i]]
        keys.add(x)
    bits = np.unpackbits(words[:(1 << (2 * K)) // 32].view(np.uint8), bitorder="little")
    assert set(np.nonzero(bits)[0].tolist()) == keys
    assert nk.value == len(keys)
