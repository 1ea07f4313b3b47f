"""Seeded synthetic DNA texts, pattern sets and request streams.

The paper's pattern files (about 100-base lines, 1000-5000 of them) and input
files (0.75 M - 3.75 M lines of about 100 bases) are not public (Sec. VI,
Tables II and III); everything here is a synthetic stand-in with the shapes,
sizes and value distributions of the workloads named in ``CONFIGS``.

Encodings produced here (input formats, not matching logic):
  * ASCII: one byte per base, b'A', b'C', b'G', b'T';
  * 2-bit packed: A=0, C=1, G=2, T=3, base 4k+j in bits 2j..2j+1 of byte k.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ACGT", "rng", "uniform_codes", "uniform_ascii", "markov_matrix", "markov_codes",
    "codes_to_ascii", "ascii_to_codes", "pack2bit", "unpack2bit_ascii", "random_packed",
    "cut_patterns", "random_patterns", "PlainWorkload", "plain_workload", "BatchWorkload",
    "batch_workload", "served_tries", "ServedRequest", "served_requests", "CONFIG_NAMES",
    "lognormal_lengths", "ReadsWorkload", "reads_workload",
]

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
_CODE_OF = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _CODE_OF[_c] = _i

CONFIG_NAMES = ("c0_tiny", "c1_large_markov", "c2_packed_big_trie", "c3_batched", "c4_served")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_codes(n: int, g: np.random.Generator) -> np.ndarray:
    return g.integers(0, 4, size=int(n), dtype=np.uint8)


def codes_to_ascii(codes: np.ndarray) -> np.ndarray:
    return ACGT[codes]


def ascii_to_codes(text: np.ndarray) -> np.ndarray:
    c = _CODE_OF[np.asarray(text, dtype=np.uint8)]
    if c.size and c.max() == 255:
        raise ValueError("text holds bytes other than A, C, G, T")
    return c


def uniform_ascii(n: int, g: np.random.Generator) -> np.ndarray:
    return codes_to_ascii(uniform_codes(n, g))


def markov_matrix(g: np.random.Generator, pi=(0.295, 0.205, 0.205, 0.295),
                  concentration: float = 40.0) -> np.ndarray:
    """Random first-order transition matrix whose stationary law is ``pi``.

    Proposal rows are Dirichlet(concentration * pi), i.e. random rows centred
    on pi; a Metropolis correction P[i,j] = min(Q[i,j], pi[j] Q[j,i] / pi[i])
    (j != i) makes the chain reversible with respect to pi, so pi is exactly
    stationary (GC content pi[C] + pi[G] = 0.41 for the default).  With the
    default concentration the entropy rate is about 1.9 bits per base, close
    to that of first-order models of real genomes; flat Dirichlet(1,1,1,1)
    rows would instead pile mass on the diagonal (about 1 bit per base, long
    single-base runs).
    """
    pi = np.asarray(pi, dtype=np.float64)
    Q = g.dirichlet(concentration * pi, size=4)
    P = np.zeros((4, 4))
    for i in range(4):
        for j in range(4):
            if i != j:
                P[i, j] = min(Q[i, j], pi[j] * Q[j, i] / pi[i])
        P[i, i] = 1.0 - P[i].sum()
    return P


def markov_codes(n: int, g: np.random.Generator, P: np.ndarray, pi=None,
                 block: int = 4096) -> np.ndarray:
    """Sample n steps of the chain P (codes 0..3) with x0 ~ pi.

    Transition probabilities are quantised to multiples of 1/256 and driven by
    one uniform byte per step.  The chain is cut into ``block``-long pieces;
    the end state of every piece is first computed for all four possible
    entry states (vectorised over pieces), the entry states are then chained
    piece by piece, and each piece is finally replayed from its true entry
    state.  The result is exactly the sequential chain for the same bytes.
    """
    n = int(n)
    if n == 0:
        return np.zeros(0, dtype=np.uint8)
    if pi is None:
        w, v = np.linalg.eig(P.T)
        pi = np.real(v[:, np.argmin(np.abs(w - 1))])
        pi = pi / pi.sum()
    cum = np.cumsum(P, axis=1)
    # step table: next state for (state, byte)
    u_mid = (np.arange(256) + 0.5) / 256.0
    step = np.zeros((4, 256), dtype=np.uint8)
    for s in range(4):
        step[s] = np.minimum(np.searchsorted(cum[s], u_mid, side="right"), 3)
    step_flat = step.reshape(-1)
    x0 = int(np.searchsorted(np.cumsum(pi), g.random(), side="right"))
    x0 = min(x0, 3)
    nb = (n + block - 1) // block
    u = g.integers(0, 256, size=(block, nb), dtype=np.uint8)  # u[t, b] drives step t of piece b
    # pass 1: end state of each piece for every entry state
    st = np.repeat(np.arange(4, dtype=np.uint16)[:, None], nb, axis=1)  # (4, nb)
    for t in range(block):
        st = step_flat[(st << 8) | u[t][None, :]].astype(np.uint16)
    ends = st.astype(np.uint8)  # ends[s0, b]
    # chain entry states piece by piece
    entry = np.zeros(nb, dtype=np.uint8)
    cur = x0
    for b in range(nb):
        entry[b] = cur
        cur = int(ends[cur, b])
    # pass 2: replay every piece from its entry state
    out = np.empty((block, nb), dtype=np.uint8)
    st1 = entry.astype(np.uint16)
    for t in range(block):
        st1 = step_flat[(st1 << 8) | u[t]].astype(np.uint16)
        out[t] = st1
    return np.ascontiguousarray(out.T).reshape(-1)[:n]


def pack2bit(codes: np.ndarray) -> np.ndarray:
    """Pack codes 0..3 four per byte, base 4k+j in bits 2j..2j+1 of byte k."""
    c = np.asarray(codes, dtype=np.uint8)
    n = c.size
    pad = (-n) % 4
    if pad:
        c = np.concatenate([c, np.zeros(pad, dtype=np.uint8)])
    c = c.reshape(-1, 4)
    return (c[:, 0] | (c[:, 1] << 2) | (c[:, 2] << 4) | (c[:, 3] << 6)).astype(np.uint8)


def unpack2bit_ascii(packed: np.ndarray, start: int, length: int) -> np.ndarray:
    """ASCII bases [start, start+length) of a 2-bit packed text."""
    if length <= 0:
        return np.zeros(0, dtype=np.uint8)
    b0 = start // 4
    b1 = (start + length + 3) // 4
    p = np.asarray(packed[b0:b1], dtype=np.uint8)
    codes = np.stack([(p >> (2 * j)) & 3 for j in range(4)], axis=1).reshape(-1)
    off = start - 4 * b0
    return ACGT[codes[off:off + length]]


def random_packed(n: int, g: np.random.Generator) -> np.ndarray:
    """Uniform ACGT text of n bases, directly in 2-bit packed form."""
    nbytes = (int(n) + 3) // 4
    p = g.integers(0, 256, size=nbytes, dtype=np.uint8)
    rem = int(n) % 4
    if rem and nbytes:
        p[-1] &= np.uint8((1 << (2 * rem)) - 1)
    return p


def cut_patterns(source, count: int, lmin: int, lmax: int, g: np.random.Generator,
                 n: int | None = None, packed: bool = False):
    """``count`` patterns cut at uniform random offsets of a text.

    ``source`` is an ASCII uint8 array, or a 2-bit packed array when
    ``packed`` (then ``n`` gives its base count).
    """
    if n is None:
        n = int(np.asarray(source).size)
    lens = g.integers(lmin, lmax + 1, size=count)
    out = []
    for L in lens:
        L = int(min(L, n))
        off = int(g.integers(0, n - L + 1))
        if packed:
            out.append(unpack2bit_ascii(source, off, L).tobytes())
        else:
            out.append(np.asarray(source[off:off + L], dtype=np.uint8).tobytes())
    return out


def random_patterns(count: int, lmin: int, lmax: int, g: np.random.Generator):
    lens = g.integers(lmin, lmax + 1, size=count)
    return [uniform_ascii(int(L), g).tobytes() for L in lens]


@dataclass
class PlainWorkload:
    name: str
    n: int
    enc: str                      # "ascii" or "2bit"
    text: np.ndarray              # ASCII uint8[n] or packed uint8[ceil(n/4)]
    patterns: list
    lmin: int
    lmax: int
    recipe: str

    def ascii(self, start: int = 0, length: int | None = None) -> np.ndarray:
        if length is None:
            length = self.n - start
        if self.enc == "ascii":
            return self.text[start:start + length]
        return unpack2bit_ascii(self.text, start, length)


def plain_workload(idx: int, n: int | None = None, num_patterns: int | None = None,
                   seed: int | None = None) -> PlainWorkload:
    """Plain single-text workloads.

    idx 0: uniform ASCII, 1 Mbase; 100 patterns, lengths U[20,40], 50 cut
           from the text then 50 uniform random.
    idx 1: first-order Markov ASCII (stationary GC 0.41), 256 Mbase; 10,000
           patterns, lengths U[16,64], 70 % cut from the text then 30 % random.
    idx 2: uniform 2-bit packed, 1 Gbase; 200,000 patterns, lengths U[12,32],
           50 % cut from the text then 50 % random.
    ``n`` / ``num_patterns`` shrink a workload for tests (same distributions).
    """
    s = idx if seed is None else seed
    g = rng(s)
    if idx == 0:
        n = 1 << 20 if n is None else n
        P = 100 if num_patterns is None else num_patterns
        text = uniform_ascii(n, g)
        planted = P // 2
        pats = cut_patterns(text, planted, 20, 40, g) + random_patterns(P - planted, 20, 40, g)
        return PlainWorkload(CONFIG_NAMES[0], n, "ascii", text, pats, 20, 40,
                             "uniform ACGT ASCII; 50%% patterns cut from the text, 50%% random; "
                             "lengths U[20,40]; PCG64 seed %d" % s)
    if idx == 1:
        n = 256 << 20 if n is None else n
        P = 10000 if num_patterns is None else num_patterns
        Pm = markov_matrix(g)
        text = codes_to_ascii(markov_codes(n, g, Pm, pi=np.array([0.295, 0.205, 0.205, 0.295])))
        planted = (P * 7) // 10
        pats = cut_patterns(text, planted, 16, 64, g) + random_patterns(P - planted, 16, 64, g)
        return PlainWorkload(CONFIG_NAMES[1], n, "ascii", text, pats, 16, 64,
                             "first-order Markov ACGT ASCII (stationary GC 0.41, Metropolis-"
                             "corrected Dirichlet rows); 70%% patterns cut from the text, 30%% "
                             "random; lengths U[16,64]; PCG64 seed %d" % s)
    if idx == 2:
        n = 1 << 30 if n is None else n
        P = 200000 if num_patterns is None else num_patterns
        text = random_packed(n, g)
        planted = P // 2
        pats = (cut_patterns(text, planted, 12, 32, g, n=n, packed=True)
                + random_patterns(P - planted, 12, 32, g))
        return PlainWorkload(CONFIG_NAMES[2], n, "2bit", text, pats, 12, 32,
                             "uniform ACGT, 2-bit packed; 50%% patterns cut from the text, 50%% "
                             "random; lengths U[12,32]; PCG64 seed %d" % s)
    raise ValueError("plain workloads are 0, 1 and 2")


def lognormal_lengths(count: int, g: np.random.Generator, median: float = 20000.0,
                      sigma: float = 1.336, lo: int = 150, hi: int = 2_000_000) -> np.ndarray:
    L = np.exp(math.log(median) + sigma * g.standard_normal(count))
    return np.clip(np.rint(L), lo, hi).astype(np.int64)


@dataclass
class BatchWorkload:
    name: str
    lengths: np.ndarray           # int64[T]
    offsets: np.ndarray           # int64[T], byte offsets into ``buffer`` (16-byte aligned)
    buffer: np.ndarray            # uint8 ASCII, texts at ``offsets`` (gaps hold b'N')
    patterns: list
    recipe: str

    def text(self, t: int) -> np.ndarray:
        o = int(self.offsets[t])
        return self.buffer[o:o + int(self.lengths[t])]

    @property
    def total_bases(self) -> int:
        return int(self.lengths.sum())


def batch_workload(num_texts: int = 4096, num_patterns: int = 50000, seed: int = 3,
                   median: float = 20000.0, hi: int = 2_000_000, lmin: int = 16,
                   lmax: int = 48) -> BatchWorkload:
    """Many independent uniform ASCII texts, lognormal lengths (median 20 kbase,
    sigma 1.336 so the mean is about 48.8 kbase), clipped to [150, 2 M]; one
    pattern set, lengths U[16,48], half cut from the batch (text chosen with
    probability proportional to its length), half random."""
    g = rng(seed)
    lengths = lognormal_lengths(num_texts, g, median=median, hi=hi)
    padded = (lengths + 15) // 16 * 16
    offsets = np.concatenate([[0], np.cumsum(padded)[:-1]]).astype(np.int64)
    total = int(padded.sum())
    buf = np.full(total, ord("N"), dtype=np.uint8)
    allcodes = uniform_codes(int(lengths.sum()), g)
    src = 0
    for t in range(num_texts):
        L = int(lengths[t])
        buf[offsets[t]:offsets[t] + L] = ACGT[allcodes[src:src + L]]
        src += L
    planted = num_patterns // 2
    lens = g.integers(lmin, lmax + 1, size=planted)
    prob = lengths / lengths.sum()
    which = g.choice(num_texts, size=planted, p=prob)
    pats = []
    for L, t in zip(lens, which):
        L = int(min(L, lengths[t]))
        off = int(g.integers(0, int(lengths[t]) - L + 1))
        o = int(offsets[t]) + off
        pats.append(buf[o:o + L].tobytes())
    pats += random_patterns(num_patterns - planted, lmin, lmax, g)
    return BatchWorkload(CONFIG_NAMES[3], lengths, offsets, buf, pats,
                         "%d uniform ASCII texts, lognormal lengths (median %g, sigma 1.336) "
                         "clipped to [150, %d]; %d patterns U[%d,%d], half cut from the batch; "
                         "PCG64 seed %d" % (num_texts, median, hi, num_patterns, lmin, lmax, seed))


def served_tries(seed: int = 4, sizes=None, lmin: int = 12, lmax: int = 64,
                 pool_bases: int = 50_000_000):
    """Eight pattern sets with geometric sizes 1,000 .. 200,000, lengths
    U[12,64], half cut from a seeded uniform pool, half random."""
    if sizes is None:
        sizes = [int(round(1000 * (200.0 ** (k / 7.0)))) for k in range(8)]
    g = rng(seed)
    pool = uniform_ascii(pool_bases, g)
    tries = []
    for P in sizes:
        planted = P // 2
        tries.append(cut_patterns(pool, planted, lmin, lmax, g)
                     + random_patterns(P - planted, lmin, lmax, g))
    return tries


@dataclass
class ServedRequest:
    rid: int
    kind: str           # "reads", "contig" or "chromosome"
    trie: int
    lengths: np.ndarray  # bases per text of the request
    seed: int
    arrival: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def bases(self) -> int:
        return int(self.lengths.sum())

    def texts(self) -> list:
        g = rng(self.seed)
        return [uniform_ascii(int(L), g) for L in self.lengths]


REQUEST_KINDS = {
    "reads": (10000, 150),
    "contig": (1, 1_000_000),
    "chromosome": (1, 50_000_000),
}


def served_requests(count: int, rate_bases_per_s: float, seed: int = 4, num_tries: int = 8,
                    scale: float = 1.0) -> list:
    """Request stream: kind equiprobable among reads (10,000 x 150 b), contig
    (1 Mbase) and chromosome (50 Mbase); trie uniform; Poisson arrivals whose
    mean offered load is ``rate_bases_per_s``.  ``scale`` shrinks every text
    length for tests."""
    g = rng(1000 + seed)
    kinds = list(REQUEST_KINDS)
    mean_bases = np.mean([REQUEST_KINDS[k][0] * max(1, int(REQUEST_KINDS[k][1] * scale))
                          for k in kinds])
    lam = rate_bases_per_s / mean_bases  # requests per second
    t = 0.0
    out = []
    for r in range(count):
        t += float(g.exponential(1.0 / lam))
        k = kinds[int(g.integers(0, 3))]
        cnt, L = REQUEST_KINDS[k]
        L = max(1, int(L * scale))
        out.append(ServedRequest(r, k, int(g.integers(0, num_tries)),
                                 np.full(cnt, L, dtype=np.int64), int(g.integers(0, 2**62)), t))
    return out


@dataclass
class ReadsWorkload:
    """A pattern set and a reads file in the shape of the paper's experiments
    (Tables II and III): ``num_patterns`` patterns of 100 bases, and
    ``num_reads`` reads of 95..105 bases, one per line (each read followed by
    a newline byte, which no walk crosses)."""
    name: str
    text: np.ndarray              # ASCII uint8, reads joined by b"\n"
    patterns: list
    num_reads: int
    recipe: str

    @property
    def n(self) -> int:
        return int(self.text.size)


def reads_workload(pattern_set: int, data_set: int, seed: int = 5,
                   num_reads: int | None = None) -> ReadsWorkload:
    """Paper-shaped stand-in: pattern set k has 1000*k patterns of 100 bases
    (the 101.1 KB per 1000 lines of Table II); data set k has 750,000*k reads
    of U[95,105] uniform-random bases, newline-terminated (about 101 bytes a
    line, as in Table III).  Half of the patterns are cut from reads of at
    least 100 bases (so they occur), the other half are uniform random."""
    if not (1 <= pattern_set <= 5 and 1 <= data_set <= 5):
        raise ValueError("pattern and data sets are numbered 1..5")
    g = rng(seed * 100 + pattern_set * 10 + data_set)
    R = 750_000 * data_set if num_reads is None else int(num_reads)
    lens = g.integers(95, 106, size=R)
    ends = np.cumsum(lens + 1)
    total = int(ends[-1]) if R else 0
    text = uniform_ascii(total, g)
    text[ends - 1] = ord("\n")
    starts = ends - 1 - lens
    P = 1000 * pattern_set
    long_reads = np.nonzero(lens >= 100)[0]
    planted = P // 2
    pats = []
    for r in g.choice(long_reads, size=planted, replace=True):
        off = int(starts[r]) + int(g.integers(0, int(lens[r]) - 100 + 1))
        pats.append(text[off:off + 100].tobytes())
    pats += random_patterns(P - planted, 100, 100, g)
    return ReadsWorkload("paper_p%d_d%d" % (pattern_set, data_set), text, pats, R,
                         "%d reads of U[95,105] uniform ACGT bases, newline-terminated; "
                         "%d patterns of 100 bases, half cut from reads, half random; "
                         "PCG64 seed %d" % (R, P, seed * 100 + pattern_set * 10 + data_set))
