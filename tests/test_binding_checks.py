"""Argument checks of the Python binding, on the CPU: every call whose
buffers are too small for what the kernels would read or write is refused
before anything reaches the library."""
import numpy as np
import pytest
import torch

from paper_1811_10498_amd import matcher as M


def _out(n_match, hits_shape=(8, 2), counters=2):
    return M.MatchResult(torch.empty(n_match, dtype=torch.int32) if n_match is not None else None,
                         torch.empty(hits_shape, dtype=torch.int32) if hits_shape else None,
                         torch.empty(counters, dtype=torch.int64))


def test_one_text_checks():
    M.check_match_args(100, 100, "ascii")
    M.check_match_args(100, 25, "2bit")
    with pytest.raises(ValueError):
        M.check_match_args(101, 100, "ascii")
    with pytest.raises(ValueError):
        M.check_match_args(101, 25, "2bit")
    with pytest.raises(ValueError):
        M.check_match_args(1 << 32, 1 << 33, "ascii")
    with pytest.raises(ValueError):
        M.check_match_args(10, 10, "utf8")
    M.check_match_args(100, 100, "ascii", _out(100))
    with pytest.raises(ValueError):
        M.check_match_args(100, 100, "ascii", _out(99))
    with pytest.raises(ValueError):
        M.check_match_args(100, 100, "ascii", _out(100, hits_shape=(8, 3)))
    with pytest.raises(ValueError):
        M.check_match_args(100, 100, "ascii", _out(100, counters=1))
    M.check_match_args(100, 100, "ascii", _out(None, hits_shape=None))


def _descs(offsets, lengths, enc="ascii", match_offsets=None):
    d, T, _, _ = M._descriptors(offsets, lengths, None, enc, match_offsets)
    return d, T


def test_batch_extent_checks():
    d, T = _descs([0, 160, 320], [150, 150, 150])
    M.check_batch_extents(d, T, 470, 454)
    with pytest.raises(ValueError):
        M.check_batch_extents(d, T, 469, 454)          # last text runs past the base
    with pytest.raises(ValueError):
        M.check_batch_extents(d, T, 470, 453)          # outputs run past match_out
    M.check_batch_extents(d, T, 470, None)             # no dense output
    d2, T2 = _descs([0, 64], [100, 100], enc="2bit")
    M.check_batch_extents(d2, T2, 89, 200)
    with pytest.raises(ValueError):
        M.check_batch_extents(d2, T2, 88, 200)
    d3, T3 = _descs([0, 1000], [10, 0])                # empty texts reach nothing
    M.check_batch_extents(d3, T3, 10, 10)
    with pytest.raises(ValueError):
        M.check_batch_extents(d, T, 470, 454, hits_shape=(16, 2))
    with pytest.raises(ValueError):
        M.check_batch_extents(d, T, 470, 454, counters_numel=7)
    assert M._extents(d, T) == (470, 454)
    d4, T4 = _descs([0, 16], [5, 5], match_offsets=np.array([100, 0]))
    assert M._extents(d4, T4) == (21, 105)


def test_default_match_layout_is_aligned_and_disjoint():
    L = np.array([150, 1, 0, 7, 4, 2049, 3], dtype=np.int64)
    o = M.match_layout(L).astype(np.int64)
    assert o.dtype == np.int64 and o.size == L.size
    assert (o % 4 == 0).all()
    assert (o[1:] >= o[:-1] + L[:-1]).all()             # runs do not overlap
    assert (o[1:] - (o[:-1] + L[:-1]) <= 3).all()       # at most 3 elements of padding
    d, T = _descs(np.arange(L.size) * 4096, L)
    assert (d["match_offset"][:T] == o).all()
    assert M._extents(d, T)[1] == int(o[-1] + L[-1])
    assert M.match_layout([]).size == 0
