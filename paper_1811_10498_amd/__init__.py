"""PFAC DNA matching on AMD Instinct MI355X (gfx950).

Parallel Failure-less Aho-Corasick (Lin et al.; the DNA-specific variant of
Thambawita, Ragel and Elkaduwe, arXiv:1811.10498): every text position walks
a failure-link-free goto trie over {A,C,G,T} and reports the longest pattern
starting there.  The matching runs in hand-written HIP kernels behind the C
ABI of include/pfac.h (libpfac.so); this package is the Python binding.
"""
from ._lib import (PFAC_HASH_NONE, PFAC_LEVELS_NONE, PFAC_VARIANT_GLOBAL,
                   PFAC_VARIANT_GLOBAL_MERGED, PFAC_VARIANT_GLOBAL_TWO_ARRAYS, PFAC_VARIANT_TILED,
                   PFAC_PREFIX_NONE, PFAC_PAIR_NONE, PFAC_WALKS_DEFERRED, PFAC_WALKS_INLINE, PfacError, lib)
from .matcher import (AllResult, Batch, BatchResult, MatchResult, Table, match, match_all,
                      match_batch, match_layout, n_bases)

__all__ = [
    "Table", "match", "match_all", "AllResult", "match_batch", "Batch", "MatchResult",
    "BatchResult", "PfacError", "lib", "n_bases", "match_layout", "PFAC_VARIANT_TILED", "PFAC_VARIANT_GLOBAL",
    "PFAC_VARIANT_GLOBAL_TWO_ARRAYS", "PFAC_VARIANT_GLOBAL_MERGED", "PFAC_LEVELS_NONE", "PFAC_HASH_NONE",
    "PFAC_WALKS_INLINE", "PFAC_WALKS_DEFERRED", "PFAC_PREFIX_NONE", "PFAC_PAIR_NONE",
]
