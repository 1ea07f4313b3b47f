"""Build libpfac.so (HIP for gfx950) in-tree with hipcc.

The scan kernel is instantiated for every workgroup size and launch kind in
its own translation unit (``scan_inst.hip`` compiled once per combination),
so the units compile in parallel; the host API unit, the host trie builder
and the units are then linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpfac.so")
PROBE_SRC = os.path.join(CSRC, "probe", "stream_probe.hip")
PROBE_LIB = os.path.join(HERE, "libpfac_probe.so")

BLOCKS = (256, 512, 768, 1024)

# Packed-FP32 instructions are disabled for every HIP object (the matcher has
# no floating point, the flag keeps the compiler from emitting them anyway).
HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _units():
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    units = []
    for b in BLOCKS:
        for single in (1, 0):
            obj = os.path.join(OBJ, "scan_b%d_%s.o" % (b, "single" if single else "batch"))
            units.append(([hipcc(), *HIPCC_FLAGS, *inc, "-DPFAC_BLOCK=%d" % b,
                           "-DPFAC_SINGLE=%d" % single, "-c",
                           os.path.join(CSRC, "scan_inst.hip"), "-o", obj], obj))
    # every other HIP unit (host API, allocation-free entry point, ...)
    for src in sorted(os.listdir(CSRC)):
        if src.endswith(".hip") and src != "scan_inst.hip":
            obj = os.path.join(OBJ, src[:-4] + ".o")
            units.append(([hipcc(), *HIPCC_FLAGS, *inc, "-c", os.path.join(CSRC, src),
                           "-o", obj], obj))
    obj = os.path.join(OBJ, "builder.o")
    units.append((["g++", *CXX_FLAGS, *inc, "-c", os.path.join(CSRC, "builder.cpp"), "-o", obj],
                  obj))
    return units


def _clean(out: str) -> str:
    return "\n".join(l for l in out.splitlines()
                     if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)


def _run(cmd):
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return res.returncode, _clean(res.stdout)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), max(1, min(16, os.cpu_count() or 1)))
    if verbose:
        print("compiling %d units with %d jobs" % (len(units), jobs), flush=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _run(u[0]), units))
    errors = [(u, r) for u, r in zip(units, results) if r[0] != 0]
    if errors:
        (cmd, _), (_, out) = errors[0]
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), out))
    if verbose:
        for (cmd, _), (_, out) in zip(units, results):
            if out.strip():
                print(out, flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    rc, out = _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC",
                    *[o for _, o in units], "-o", tmp])
    if rc != 0:
        raise RuntimeError("link failed:\n" + out)
    os.replace(tmp, LIB)
    build_probe()
    return LIB


def build_probe() -> str:
    """The bandwidth reference kernels of the benchmark's roofline
    (measurement only, a library of their own)."""
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    rc, out = _run([hipcc(), *HIPCC_FLAGS, "-shared", PROBE_SRC, "-o", tmp])
    if rc != 0:
        raise RuntimeError("probe build failed:\n" + out)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
