"""Shape of the paper-shaped reads workload (Tables II and III): reads of
95..105 bases, each followed by a newline; patterns of 100 bases, the first
half cut from reads."""
import numpy as np

import workloads as W


def test_reads_workload_shape():
    w = W.reads_workload(3, 2, num_reads=5000)
    assert w.num_reads == 5000 and len(w.patterns) == 3000
    nl = np.nonzero(w.text == ord("\n"))[0]
    assert nl.size == 5000 and nl[-1] == w.n - 1
    lens = np.diff(np.concatenate([[-1], nl])) - 1
    assert lens.min() >= 95 and lens.max() <= 105
    body = np.delete(w.text, nl)
    assert np.isin(body, np.frombuffer(b"ACGT", dtype=np.uint8)).all()
    assert all(len(p) == 100 for p in w.patterns)
    raw = w.text.tobytes()
    assert all(p in raw for p in w.patterns[:1500])


def test_reads_workload_full_size_matches_the_paper_files():
    # file sizes of Table III: 76 MB for 750,000 reads .. 380.2 MB for 3.75 M
    # (about 101 bytes a line); computed from the read lengths alone
    g = W.rng(0)
    lens = g.integers(95, 106, size=750_000)
    assert abs((lens + 1).sum() / 1e6 - 76.0) < 1.0
