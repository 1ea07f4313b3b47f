"""Seeded synthetic inputs for PFAC DNA matching.

This package produces texts, pattern sets and request streams only.  It holds
none of the matching arithmetic: both the GPU library's tests/benchmarks and
the CPU oracle's tests consume what it generates.
"""
from .synth import *  # noqa: F401,F403
