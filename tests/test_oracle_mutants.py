"""The oracle's pins catch plausible mistakes: each planted mistake (compiled
into a separate build of the oracle source, on the CPU) makes at least one
pin fail."""
import ctypes
import itertools
import os

import numpy as np
import pytest

import oracle
import workloads as W
from _checkers import brute, brute_pairs, read_golden

MUTANTS = {
    1: "no dictionary links",
    2: "ties go to the larger ID",
    3: "start position off by one",
    4: "non-bases read as A",
    5: "shortest pattern wins",
    6: "failure links never followed",
}

PATTERN_SETS = [
    [b"AC", b"ACG", b"CTGT", b"TG"],
    [b"CG", b"ACGT", b"G", b"GT", b"TACG"],
    [b"ACG", b"ACG", b"CG", b"CG", b"G"],
    [b"AT", b"TA", b"ATA", b"TAT", b"ATAT", b"TATA"],
]


def _pins_pass(lib) -> bool:
    """The brute-force and worked-example pins, run against one build."""
    for name in ("ex1_fig1_text.txt", "ex2_table1_text.txt"):
        ex = read_golden(name)
        pats = [p.encode() for p in ex["patterns"].split()]
        m, t = oracle.scan(pats, ex["text"].encode(), lib=lib)
        if m.tolist() != [int(x) for x in ex["match"].split()] or t != int(ex["total"]):
            return False
    texts = []
    for L in range(0, 6):
        texts += ["".join(x) for x in itertools.product("ACGT", repeat=L)]
    big = ("N".join(texts) + "NACGTnacgtACGT").encode()
    for pats in PATTERN_SETS:
        m, t = oracle.scan(pats, big, lib=lib)
        bm, bt = brute(pats, big)
        if m.tolist() != bm or t != bt:
            return False
    return True


def test_reference_build_passes_the_pins():
    assert _pins_pass(None)


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_planted_mistake_is_caught(k, tmp_path):
    path = oracle.build_mutant(k, str(tmp_path))
    lib = oracle._declare(ctypes.CDLL(path))
    assert not _pins_pass(lib), "mutant %d (%s) passed every pin" % (k, MUTANTS[k])


def _occurrence_pins_pass(lib) -> bool:
    """The all-occurrence list against brute force, on its own."""
    texts = []
    for L in range(0, 6):
        texts += ["".join(x) for x in itertools.product("ACGT", repeat=L)]
    big = ("N".join(texts) + "NACGTnacgtACGT").encode()
    for pats in PATTERN_SETS:
        occ = oracle.occurrences(pats, big, lib=lib)
        if [tuple(r) for r in occ.tolist()] != brute_pairs(pats, big):
            return False
    return True


def test_reference_build_passes_the_occurrence_pins():
    assert _occurrence_pins_pass(None)


@pytest.mark.parametrize("k", [1, 3, 4, 6])
def test_planted_mistake_in_the_scan_breaks_the_occurrence_list(k, tmp_path):
    """Mistakes in the scan itself (not in the longest-wins rule) show in the
    list of every occurrence."""
    path = oracle.build_mutant(k, str(tmp_path))
    lib = oracle._declare(ctypes.CDLL(path))
    assert not _occurrence_pins_pass(lib), "mutant %d (%s) passed" % (k, MUTANTS[k])
