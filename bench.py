#!/usr/bin/env python3
"""PFAC benchmark on one MI355X.

One step = one pfac_match call over the whole text of the plain large-text
workload (256 Mbase first-order Markov ASCII text, 10,000 patterns of 16-64
bases, 70 % cut from the text): text ingest, per-position walks, dense int32
match array, ordered hit list and occurrence count.  The text and the table
are resident in HBM before the timed region; untimed calls for 50 ms (the
GPU raises its clocks under load) and W warm-up steps come first, then K
steps back to back between two synchronisations, with two HIP events on the
launching stream around them.  Prints one JSON line (with --paper-ladder
instead the paper's placement ladder, one line per case and a table).

Beside the primary figure the line carries every other workload, each timed
the same way: the 1 Mbase tiny case, the 1 Gbase 2-bit text against 200,000
patterns (dense output and hit list only), the 4,096-text batch (prepared
launch, one-shot batched call, the one-text kernel over the same bases, one
call per text), the served request mix (capacity, latency at 0.7 load, the
one-launch-per-request baseline), the bandwidth of plain fills and copies
and of a probe kernel with the scan's exact access shape, and the oracle on
the host's cores.  --only picks one of them (for profiling runs).
"""
import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CSRC = os.path.join(ROOT, "paper_1811_10498_amd", "csrc")
KERNEL_SRCS = ("scan_device.h", "scan_inst.hip", "pfac_api.hip", "pfac_internal.h")
PROFILES = os.path.join(ROOT, "profiles")
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, 8 TB/s
PARTS = ("c0", "c1", "c2", "c3", "c4", "floor")


def kernel_sha() -> str:
    """Hash of the kernel sources (device code, instantiations, host launch code)."""
    h = hashlib.sha256()
    for name in KERNEL_SRCS:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counters(workload: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    or None if it is missing or was taken on another kernel source."""
    path = os.path.join(PROFILES, "pfac_kernel_%s_counters.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("kernel_sha256") != kernel_sha():
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * 1024
        write = float(kv["write_kib_per_dispatch"]) * 1024
        return (fetch * float(kv["fetch_factor"]) + write * float(kv["write_factor"]))
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def warm_clock(torch, fn, seconds=0.05):
    """Untimed calls for `seconds` (the GPU raises its clocks under load)."""
    t = time.perf_counter()
    while time.perf_counter() - t < seconds:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def region_ms(torch, fn, reps):
    """Average ms of `reps` back-to-back calls: two events on the current
    stream around them."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def per_call_ms(torch, fn, reps):
    """Median and min of `reps` calls, each between its own two events."""
    import numpy as np
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return float(np.median(t)), float(t.min())


def alg_bytes_one(n, enc, hits, states, dense=True):
    """Algorithmic bytes of a one-text call: the text, the dense int32 output
    (when written), 8 bytes per hit, the counters and the next-state table
    read once (16 bytes per state)."""
    text = n if enc == "ascii" else (n + 3) // 4
    return text + (4 * n if dense else 0) + 8 * hits + 16 + 16 * states


def roofline(bytes_, ms, traffic=None, bound="hbm"):
    gbs = bytes_ / (ms / 1e3) / 1e9
    return {"bound": bound, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else int(traffic),
            "algorithmic_bytes_per_launch": int(bytes_), "avg_launch_ms": round(ms, 4)}


def oracle_baseline(w, sample_mbases, seconds):
    """The oracle (classic Aho-Corasick, plain C) on the host's cores: all
    threads on a bounded sample for about `seconds`, then one thread on a
    smaller sample for half as long."""
    import oracle
    threads = os.cpu_count() or 1
    sample = min(w.n, sample_mbases << 20)
    host_text = w.ascii(0, sample)
    reps = 0
    t1 = time.perf_counter()
    while True:
        oracle.scan(w.patterns, host_text, threads=threads)
        reps += 1
        dt = time.perf_counter() - t1
        if dt >= seconds or reps >= 1000:
            break
    out = {"value": round(sample * reps / dt / 1e9, 4), "unit": "Gbases/s", "cores": threads,
           "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model(),
           "sample": "first %d Mbase of the same text, all %d patterns, classic Aho-Corasick "
                     "scan split over %d threads (all of os.cpu_count()), %d passes (wall %.2f s, "
                     "about %.0f core-seconds)" % (sample >> 20, len(w.patterns), threads, reps,
                                                   dt, dt * threads)}
    sample1 = min(w.n, 8 << 20)
    text1 = w.ascii(0, sample1)
    reps1 = 0
    t1 = time.perf_counter()
    while True:
        oracle.scan(w.patterns, text1, threads=1)
        reps1 += 1
        dt1 = time.perf_counter() - t1
        if dt1 >= seconds / 2 or reps1 >= 1000:
            break
    out["one_thread_value"] = round(sample1 * reps1 / dt1 / 1e9, 4)
    out["one_thread_sample"] = "first %d Mbase, %d passes on one thread (wall %.2f s)" % (
        sample1 >> 20, reps1, dt1)
    return out


def filter_rates(pf, table_patterns, plan, codes_sample):
    """Fractions of the positions of a text sample that pass each filter
    stage of `plan` (the depth-D LDS bitmap, the hashed bitmap, the prefix
    bitmap), from the library's own host-built bitmaps; walks per base is
    the last.  `codes_sample`: 2-bit codes of the sample (uint8 0..3)."""
    import numpy as np
    from paper_1811_10498_amd import _lib as L
    lib = L.lib()
    pats = [bytes(p) for p in table_patterns]
    bufs = [ctypes.create_string_buffer(p, len(p)) for p in pats]
    arr = (ctypes.c_void_p * len(pats))(*[ctypes.addressof(b) for b in bufs])
    lens = (ctypes.c_uint32 * len(pats))(*[len(p) for p in pats])
    bad = ctypes.c_int64(-1)
    c = np.asarray(codes_sample, dtype=np.uint64)
    n = c.size - 16
    key16 = np.zeros(n, dtype=np.uint64)
    for k in range(16):
        key16 = (key16 << np.uint64(2)) | c[k:k + n]
    D = plan["depth"]
    words = np.zeros((1 << (2 * D)) // 32 + (1 << (2 * D)) // 128 + (1 << 20), dtype=np.uint32)
    nw = ctypes.c_uint64(0)
    meta = (ctypes.c_uint32 * 25)()
    lib.pfac_build_host_image(arr, lens, len(pats), D, words.ctypes.data, words.size, meta,
                              ctypes.byref(nw), ctypes.byref(bad))
    bits = np.unpackbits(words[:(1 << (2 * D)) // 32].view(np.uint8), bitorder="little")
    xD = (key16 >> np.uint64(32 - 2 * D)).astype(np.int64)
    passD = bits[xD].astype(bool)
    out = {"depth_filter": float(passD.mean())}
    passH = passD
    if plan.get("hash_bits", 0xFFFFFFFF) != 0xFFFFFFFF:
        b = plan["hash_bits"]
        hw = np.zeros((1 << b) // 32, dtype=np.uint32)
        K = ctypes.c_uint32(0)
        lib.pfac_build_host_hash(arr, lens, len(pats), b, hw.ctypes.data, ctypes.byref(K),
                                 ctypes.byref(bad))
        hb = np.unpackbits(hw.view(np.uint8), bitorder="little").astype(bool)
        key = (key16 & np.uint64(((1 << (2 * K.value)) - 1) << (32 - 2 * K.value)))
        if K.value <= 12 and bits.mean() > 0.3:
            # large sets: the one-hash form (first K bases right-aligned, 24-bit multiplier)
            lib.pfac_build_host_hash1(arr, lens, len(pats), b, hw.ctypes.data, ctypes.byref(K),
                                      ctypes.byref(bad))
            hb = np.unpackbits(hw.view(np.uint8), bitorder="little").astype(bool)
            k24 = key >> np.uint64(32 - 2 * K.value)
            h1 = ((k24 * np.uint64(0xC6A4A7)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - b)
            passH = passD & hb[h1.astype(np.int64)]
            out["hash_form"] = "one 24-bit multiplicative hash"
        else:
            h1 = ((key * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - b)
            h2 = ((key * np.uint64(0x85EBCA77)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - b)
            passH = passD & hb[h1.astype(np.int64)] & hb[h2.astype(np.int64)]
        out["hash_filter"] = float(passH.mean())
    passP = passH
    if plan.get("prefix", 0xFFFFFFFF) == 1:
        pw = np.zeros(1 << 19, dtype=np.uint32)
        K2 = ctypes.c_uint32(0)
        nk = ctypes.c_uint64(0)
        lib.pfac_build_host_prefix(arr, lens, len(pats), pw.ctypes.data, pw.size,
                                   ctypes.byref(K2), ctypes.byref(nk), ctypes.byref(bad))
        pb = np.unpackbits(pw[:(1 << (2 * K2.value)) // 32].view(np.uint8),
                           bitorder="little").astype(bool)
        x2 = (key16 >> np.uint64(32 - 2 * K2.value)).astype(np.int64)
        passP = passH & pb[x2]
        out["global_prefix_reads_per_base"] = float(passH.mean())
        out["prefix_filter"] = float(passP.mean())
    out["lds_bitmap_lookups_per_base"] = round(1.0 + (2.0 * float(passD.mean())
                                                      if "hash_filter" in out else 0.0), 4)
    out["walks_per_base"] = float(passP.mean())
    out["sample_bases"] = int(n)
    return out


def bench_one(pf, torch, w, plan, steps, warmup, dense=True):
    """K back-to-back calls of one workload: whole-job rate, event-timed
    average, per-call median/min.  Returns (stats, result of the last call)."""
    dev = torch.device("cuda:0")
    table = pf.Table(w.patterns)
    text = torch.from_numpy(w.text).to(dev)
    n = w.n
    res = pf.match(table, text, n=n, enc=w.enc, plan=plan, dense=dense, hit_cap=n // 64 + 1024)
    torch.cuda.synchronize()
    num_hits, total = res.num_hits(), res.total()
    if num_hits > res.hits.shape[0]:
        res = pf.match(table, text, n=n, enc=w.enc, plan=plan, dense=dense,
                       hit_cap=num_hits + 1024)
    call = lambda: pf.match(table, text, n=n, enc=w.enc, plan=plan, out=res)
    warm_clock(torch, call)
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = e0.elapsed_time(e1) / steps
    assert res.num_hits() == num_hits and res.total() == total
    med, mn = per_call_ms(torch, call, max(steps, 20))
    st = {"n": n, "ms_per_step": wall * 1e3 / steps, "avg_launch_ms": avg_ms,
          "median_ms": med, "min_ms": mn, "hits": num_hits, "occurrences": total,
          "trie_states": table.num_states,
          "plan": plan or table.default_plan(n, w.enc)}
    return st, table, text, res


def part_c1(pf, torch, args, plan):
    import workloads as W
    t_gen = time.time()
    w = W.plain_workload(1)
    t_gen = time.time() - t_gen
    st, table, text, res = bench_one(pf, torch, w, plan, args.steps, args.warmup)
    n = w.n
    alg = alg_bytes_one(n, w.enc, st["hits"], table.num_states)
    # end to end: the text from pinned host memory, the call, the hit list back
    host = torch.from_numpy(w.text).pin_memory()
    dtext = torch.empty_like(text)
    hits_host = torch.empty((res.hits.shape[0], 2), dtype=torch.int32).pin_memory()

    def e2e():
        dtext.copy_(host, non_blocking=True)
        pf.match(table, dtext, n=n, enc=w.enc, plan=plan, out=res)
        hits_host[:st["hits"]].copy_(res.hits[:st["hits"]], non_blocking=True)
    warm_clock(torch, e2e)
    e2e_ms = region_ms(torch, e2e, 10)
    out = {
        "workload": w.name, "description": w.recipe, "n_bases": n, "encoding": w.enc,
        "patterns": len(w.patterns), "trie_states": table.num_states,
        "outputs": "dense int32 match per position + position-ordered hit list + counts",
        "hits": st["hits"], "occurrences": st["occurrences"], "plan": st["plan"],
        "gbases_per_s": n * args.steps / (st["ms_per_step"] * args.steps / 1e3) / 1e9,
        "ms_per_step": st["ms_per_step"], "median_ms": st["median_ms"], "min_ms": st["min_ms"],
        "roofline": roofline(alg, st["avg_launch_ms"], read_counters(w.name)),
        "end_to_end": {"ms": round(e2e_ms, 4), "gbases_per_s": round(n / e2e_ms / 1e6, 2),
                       "what": "host-to-device copy of the text from pinned memory + the call "
                               "+ the hit list back to pinned host memory (table resident)"},
        "workload_generation_s": round(t_gen, 2),
    }
    return out, w


def part_c0(pf, torch, args, plan):
    import workloads as W
    w = W.plain_workload(0)
    st, table, _, _ = bench_one(pf, torch, w, plan, max(args.steps, 50), args.warmup)
    alg = alg_bytes_one(w.n, w.enc, st["hits"], table.num_states)
    return {"workload": w.name, "n_bases": w.n, "patterns": len(w.patterns),
            "trie_states": table.num_states, "plan": st["plan"],
            "median_ms": round(st["median_ms"], 4), "min_ms": round(st["min_ms"], 4),
            "avg_ms": round(st["avg_launch_ms"], 4),
            "gbases_per_s": round(w.n / st["avg_launch_ms"] / 1e6, 2),
            "roofline": roofline(alg, st["avg_launch_ms"]),
            "note": "launch-bound: two kernels for 1 Mbase"}


def part_c2(pf, torch, args, plan, tune=False):
    import numpy as np
    import workloads as W
    w = W.plain_workload(2)
    out = {"workload": w.name, "n_bases": w.n, "encoding": w.enc, "patterns": len(w.patterns)}
    tuned = None
    if tune and plan is None:
        from paper_1811_10498_amd.autotune import Autotuner
        tab0 = pf.Table(w.patterns)
        text0 = torch.from_numpy(w.text).to(torch.device("cuda:0"))
        tr = Autotuner(reps=2, sample_bases=256 << 20).tune(tab0, text0, n=w.n, enc=w.enc)
        tuned = tr.plan
        out["autotune"] = {"plan": tr.plan, "ms_on_sample": round(tr.ms, 4),
                           "candidates": len(tr.tried)}
        del tab0, text0
    use = tuned if tuned is not None else plan
    kinds = {"both": (True, False), "dense": (True,), "hits": (False,)}[args.c2_output]
    for dense in kinds:
        st, table, _, _ = bench_one(pf, torch, w, use, args.steps, args.warmup, dense=dense)
        alg = alg_bytes_one(w.n, w.enc, st["hits"], table.num_states, dense=dense)
        key = "dense" if dense else "hits_only"
        out[key] = {"ms": round(st["avg_launch_ms"], 4), "median_ms": round(st["median_ms"], 4),
                    "min_ms": round(st["min_ms"], 4),
                    "gbases_per_s": round(w.n / st["avg_launch_ms"] / 1e6, 2),
                    "roofline": roofline(alg, st["avg_launch_ms"],
                                         read_counters(w.name + ("" if dense else "_hits"))),
                    "hits": st["hits"], "occurrences": st["occurrences"]}
        out["plan"] = st["plan"]
        out["trie_states"] = table.num_states
    # how many positions reach each filter stage, on a 32 Mbase sample
    codes = np.stack([(w.text[:8 << 20] >> (2 * j)) & 3 for j in range(4)], axis=1).reshape(-1)
    out["filter_rates"] = filter_rates(pf, w.patterns, out["plan"], codes)
    out["lookups"] = ("per base: 1 LDS bitmap lookup; walks per base = the fraction passing "
                      "every filter; each walk reads the jump table and 1-3 next-state rows")
    return out


def part_c3(pf, torch, args, plan, tune=False):
    import numpy as np
    import workloads as W
    dev = torch.device("cuda:0")
    wb = W.batch_workload()
    tab = pf.Table(wb.patterns)
    base = torch.from_numpy(wb.buffer).to(dev)
    total = wb.total_bases
    cap = total // 16
    out = {"workload": wb.name, "texts": int(wb.lengths.size), "bases": int(total),
           "patterns": len(wb.patterns), "trie_states": tab.num_states}
    use = plan
    if tune and plan is None:
        from paper_1811_10498_amd.autotune import Autotuner
        tr = Autotuner(reps=2).tune_batch([tab], base, wb.offsets, wb.lengths)
        use = tr.plan
        out["autotune"] = {"plan": tr.plan, "ms": round(tr.ms, 4), "candidates": len(tr.tried)}
    # prepared batch: the launch enqueues kernels only (graph-capturable)
    b = pf.Batch([tab], wb.offsets, wb.lengths, plan=use, device=dev, hit_cap=cap)
    call = lambda: b.launch(base)
    call()
    torch.cuda.synchronize()
    nh = int(b.counters[0])
    warm_clock(torch, call)
    ms = region_ms(torch, call, max(args.steps, 10))
    med, mn = per_call_ms(torch, call, 20)
    alg = total + 4 * total + 8 * nh + 16 * tab.num_states + 16 * (2 + 2 * wb.lengths.size)
    out["prepared"] = {"ms": round(ms, 4), "median_ms": round(med, 4), "min_ms": round(mn, 4),
                       "gbases_per_s": round(total / ms / 1e6, 2),
                       "roofline": roofline(alg, ms, read_counters(wb.name)), "hits": nh}
    # graph of the prepared launch, replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.launch(base, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.launch(base, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    gms = region_ms(torch, g.replay, max(args.steps, 10))
    out["graph_replay"] = {"ms": round(gms, 4), "gbases_per_s": round(total / gms / 1e6, 2)}
    # one-shot batched call (host layout, descriptor upload, work items, kernels)
    res = pf.match_batch([tab], base, wb.offsets, wb.lengths, plan=use, hit_cap=cap)
    one = lambda: pf.match_batch([tab], base, wb.offsets, wb.lengths, plan=use, hit_cap=cap,
                                 match_out=res.match)
    warm_clock(torch, one)
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        one()
    torch.cuda.synchronize()
    t_call = (time.perf_counter() - t0) / reps
    out["one_shot_call"] = {"ms": round(t_call * 1e3, 4),
                            "gbases_per_s": round(total / t_call / 1e9, 2)}
    # the one-text kernel over the same bases: the texts joined by one
    # non-base byte (walks stop there), one pfac_match call
    sep = np.frombuffer(b"N", dtype=np.uint8)
    parts = []
    for t in range(wb.lengths.size):
        parts.append(wb.text(t))
        parts.append(sep)
    joined = torch.from_numpy(np.concatenate(parts)).to(dev)
    jr = pf.match(tab, joined, plan=plan, hit_cap=cap)
    jcall = lambda: pf.match(tab, joined, plan=plan, out=jr)
    warm_clock(torch, jcall)
    jms = region_ms(torch, jcall, max(args.steps, 10))
    out["one_text_kernel_joined"] = {"ms": round(jms, 4),
                                     "gbases_per_s": round(total / jms / 1e6, 2),
                                     "n": int(joined.numel()),
                                     "plan": tab.default_plan(int(joined.numel()))}
    # one plain pfac_match call per text (launch-bound), for reference
    views = [base[int(o):int(o) + int(L)] for o, L in zip(wb.offsets, wb.lengths)]
    outs = [pf.match(tab, v, hit_cap=int(v.numel()) // 16 + 64) for v in views]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v, o in zip(views, outs):
        pf.match(tab, v, out=o)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    out["per_text_calls"] = {"ms": round(t_plain * 1e3, 3),
                             "gbases_per_s": round(total / t_plain / 1e9, 2)}
    out["speedup_vs_per_text_calls"] = round(t_plain / (ms / 1e3), 2)
    out["vs_one_text_kernel"] = round(jms / ms, 3)
    out["plan"] = use if use is not None else (
        "library choice (2048-position tiles; 256 for texts up to 512 bases when a table "
        "has 4096 or more of them)")
    b.close()
    return out


def part_c4(pf, torch, args, plan, num_requests=2000, load=0.7, plain_requests=None):
    """Served workload: 8 resident tries (1,000 .. 200,000 patterns), requests
    equiprobable among a batch of 10,000 150-base reads, a 1 Mbase contig and
    a 50 Mbase chromosome-like text, texts already in device memory.  Closed
    loop first (capacity), then Poisson arrivals at `load` x capacity for
    latency; the baseline handles requests one after another, one launch per
    request, on the same request stream."""
    import numpy as np
    import workloads as W
    from paper_1811_10498_amd.serve import Request, Server, TextBatch, plain_per_request
    tries = W.served_tries(seed=4)
    tables = [pf.Table(t) for t in tries]
    g = W.rng(44)
    pool_long = torch.from_numpy(W.uniform_ascii(256 << 20, g)).cuda()
    slot = 160                                 # 150-base reads in 16-byte aligned slots
    pool_reads = torch.from_numpy(W.uniform_ascii(slot * 10000 * 8, g)).cuda()
    specs = W.served_requests(num_requests, rate_bases_per_s=1.0, seed=4)

    def make(arrivals, specs=specs):
        out = []
        for r, a in zip(specs, arrivals):
            if r.kind == "reads":
                k = int(W.rng(r.seed).integers(0, 8))
                n = int(r.lengths.size)
                offs = (k * 10000 + np.arange(n)) * slot
                out.append(Request(r.rid, r.trie, TextBatch(pool_reads, offs, r.lengths), a))
            else:
                L = int(r.lengths[0])
                o = int(W.rng(r.seed).integers(0, pool_long.numel() - L)) // 16 * 16
                out.append(Request(r.rid, r.trie, [pool_long[o:o + L]], a))
        return out

    kw = dict(budget_bytes=32 << 30, keep_results=False, plan=plan)
    srv = Server(tables, trace=True, **kw)
    warm = max(60, num_requests // 10)                 # the first tenth warms up
    srv.run(make([0.0] * num_requests)[:warm])        # warm-up (and prepared batches)
    srv.done.clear()
    srv.trace.clear()
    closed = srv.run(make([0.0] * num_requests))
    iv = srv.device_intervals()
    busy = 0.0
    if iv:
        ev = sorted([(a, 1) for _, a, _, _ in iv] + [(b, -1) for _, _, b, _ in iv])
        depth, last = 0, None
        for t, d in ev:
            if depth > 0 and last is not None:
                busy += t - last
            depth += d
            last = t
    cap = closed["gbases_per_s"] * 1e9
    bases = sum(int(r.bases) for r in make([0.0] * num_requests))
    rate = load * cap / (bases / num_requests)
    arr = np.cumsum(W.rng(45).exponential(1.0 / rate, size=num_requests))
    srv2 = Server(tables, **kw)
    srv2.run(make(arr[:warm] - arr[0]))               # warm the prepared batches of this server
    srv2.done.clear()
    opened = srv2.run(make(arr))
    # the baseline on the same requests as the closed loop (a sample would
    # hold another mix of kinds, and the kinds' rates differ by 80x)
    plain_requests = num_requests if plain_requests is None else plain_requests
    plain_per_request(tables, make([0.0] * 4, specs[:4]), plan=plan)      # warm-up
    plain = plain_per_request(tables, make([0.0] * plain_requests, specs[:plain_requests]),
                              plan=plan)
    # each request kind alone, closed loop: the server against one launch per
    # request on the same requests (the long texts get one-text launches in
    # both, so only the short kinds can gain from coalescing)
    per_kind = {}
    for kind in ("reads", "contig", "chromosome"):
        ks = [r for r in specs if r.kind == kind][:40]
        if not ks:
            continue
        reqs = lambda: make([0.0] * len(ks), ks)
        sv = Server(tables, **kw)
        sv.run(reqs())                                  # warm-up: scratch, prepared batches
        sv.done.clear()
        sk = sv.run(reqs())
        plain_per_request(tables, reqs()[:4], plan=plan)   # warm-up
        pk = plain_per_request(tables, reqs(), plan=plan)
        per_kind[kind] = {"requests": len(ks),
                          "served_gbases_per_s": round(sk["gbases_per_s"], 2),
                          "plain_gbases_per_s": round(pk["gbases_per_s"], 2),
                          "served_vs_plain": round(sk["gbases_per_s"] / pk["gbases_per_s"], 2),
                          "served_p50_ms": round(sk["p50_ms"], 3),
                          "plain_p50_ms": round(pk["p50_ms"], 3)}
    served_bytes = 5.0 * closed["gbases_per_s"] * 1e9
    return {
        "tries": [len(t) for t in tries], "requests": num_requests,
        "bases": closed.get("bases"),
        "capacity_gbases_per_s": round(closed["gbases_per_s"], 2),
        "capacity_dispatches": len(srv.dispatch_sizes),
        "prepared_batch_dispatches": srv.prepared_hits,
        "device_busy_fraction": round(busy / (iv[-1][2] - iv[0][1]), 3) if len(iv) > 1 else None,
        "max_overlapping_dispatches": srv.max_seen_inflight,
        "offered_load": load,
        "served_gbases_per_s": round(opened["gbases_per_s"], 2),
        "p50_ms": round(opened["p50_ms"], 3), "p99_ms": round(opened["p99_ms"], 3),
        "plain_per_request_gbases_per_s": round(plain["gbases_per_s"], 2),
        "plain_per_request_p50_ms": round(plain["p50_ms"], 3),
        "plain_requests_timed": plain_requests,
        "capacity_vs_plain": round(closed["gbases_per_s"] / plain["gbases_per_s"], 2),
        "served_at_load_vs_plain_capacity": round(opened["gbases_per_s"] / plain["gbases_per_s"],
                                                  2),
        "per_kind_closed_loop": per_kind,
        "roofline": {"bound": "hbm", "achieved": round(served_bytes / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(served_bytes / 1e9 / HBM_PEAK_GBS, 4),
                     "what": "5 bytes per base (text + int32 output) at closed-loop capacity"},
        "texts": "device-resident (host-to-device copies not in the timed path); a reads "
                 "request is 10,000 texts of 150 bases in 160-byte slots",
        "baseline": "requests one after another, one launch per request (pfac_match for one "
                    "text, one pfac_match_batch over a request's reads), synchronised per "
                    "request, one stream",
    }


def part_floor(pf, torch, args):
    """What the memory system gives for this traffic: plain fills and copies
    of 1 GiB by the runtime, and the probe kernel with the scan's exact
    access shape (a wave per 2048-position tile, 2 KB read, 8 KB written,
    16-byte non-temporal accesses, 1024-thread workgroups, one per CU); the
    last case issues each tile's loads before the previous tile's stores, so
    the wait for them does not drain those stores."""
    from paper_1811_10498_amd import build as B
    dev = torch.device("cuda:0")
    a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    out = {}
    for name, fn, bytes_ in (("torch_fill_1GiB", lambda: a.fill_(7), 1 << 30),
                             ("torch_zero_1GiB", lambda: a.zero_(), 1 << 30),
                             ("torch_copy_1GiB", lambda: b.copy_(a), 2 << 30)):
        warm_clock(torch, fn)
        ms = region_ms(torch, fn, 10)
        out[name] = {"ms": round(ms, 4), "gb_per_s": round(bytes_ / ms / 1e6, 1)}
    del b
    lib = ctypes.CDLL(B.PROBE_LIB)
    lib.pfac_probe_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p]
    lib.pfac_probe_stream.restype = ctypes.c_int
    n = 256 << 20                              # the large-text scan's shape: 256 Mbase
    src = a[:n]
    dst = torch.empty(n, dtype=torch.int32, device=dev)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    tiles = n // 2048
    cases = [(0, 0, 0, "scan_shape_read_256MB_write_1GiB", 5 * n),
             (1, 0, 0, "scan_shape_read_only_256MB", n),
             (2, 0, 0, "scan_shape_write_only_1GiB", 4 * n),
             (0, 1, 0, "scan_shape_plain_stores", 5 * n),
             (0, 2, 0, "scan_shape_plain_loads", 5 * n),
             (0, 0, 512, "scan_shape_2_workgroups_per_cu", 5 * n),
             (3, 0, 0, "scan_shape_stores_left_in_flight", 5 * n)]
    for mode, flags, grid, name, bytes_ in cases:
        fn = lambda: lib.pfac_probe_stream(src.data_ptr(), dst.data_ptr(), tiles, mode, flags,
                                           grid, sink.data_ptr(),
                                           torch.cuda.current_stream().cuda_stream)
        assert fn() == 0
        warm_clock(torch, fn)
        ms = region_ms(torch, fn, 20)
        out[name] = {"ms": round(ms, 4), "gb_per_s": round(bytes_ / ms / 1e6, 1),
                     "frac_of_peak": round(bytes_ / ms / 1e6 / HBM_PEAK_GBS, 4)}
    return out


# ---------------------------------------------------------------- paper ladder
# The paper times its kernel on five pattern sets (1000..5000 patterns of
# about 100 bases) against five read files (0.75 M..3.75 M reads), adding one
# memory placement at a time: global memory only, then the text in shared
# memory, then the table through the texture cache, each with the table as
# two arrays or one merged array (Sec. VI, Tables II and III; Sec. VII).
# --paper-ladder runs that structure with paper-shaped synthetic inputs over
# the placements this library has (no texture path on this GPU: loads of any
# array go through the same caches), every plan checked bit for bit against
# the first:
#   global-2arr every position walks from the root, text and table in global
#               memory (the paper's one-thread-per-character kernel), the table
#               as the paper's two arrays (next state, matched pattern ID);
#   global-merged  the same with the two merged into one array of cells;
#   global      the same with this library's edge words (child + final bit,
#               pattern IDs per state);
#   lds-d6      text tile and a depth-6 window bitmap in LDS, deep walks in
#               the global table;
#   lds-d9      the same with a depth-9 bitmap;
#   lds-levels  depth-8 bitmap and the trie levels below it in LDS, the rest
#               in the global table (the hot-prefix-in-LDS split);
#   d9-hash     depth-9 bitmap and the 2^18-bit hashed second filter, walks
#               at once;
#   default     the library's plan (the same filters, walks deferred to the
#               end of each wave).

LADDER_NAMES = ("global-2arr", "global-merged", "global", "lds-d6", "lds-d9", "lds-levels",
                "d9-hash", "default")


def ladder_plans(pf):
    return (
        ("global-2arr", dict(variant=pf.PFAC_VARIANT_GLOBAL_TWO_ARRAYS)),
        ("global-merged", dict(variant=pf.PFAC_VARIANT_GLOBAL_MERGED)),
        ("global", dict(variant=pf.PFAC_VARIANT_GLOBAL)),
        ("lds-d6", dict(depth=6, levels=pf.PFAC_LEVELS_NONE, hash_bits=pf.PFAC_HASH_NONE,
                        walks=pf.PFAC_WALKS_INLINE)),
        ("lds-d9", dict(depth=9, levels=pf.PFAC_LEVELS_NONE, hash_bits=pf.PFAC_HASH_NONE,
                        walks=pf.PFAC_WALKS_INLINE)),
        ("lds-levels", dict(depth=8, levels=0, hash_bits=pf.PFAC_HASH_NONE,
                            walks=pf.PFAC_WALKS_INLINE)),
        ("d9-hash", dict(depth=9, levels=pf.PFAC_LEVELS_NONE, hash_bits=18,
                         walks=pf.PFAC_WALKS_INLINE)),
        ("default", None),
    )


def run_ladder(pf, torch, pattern_sets=(1, 2, 3, 4, 5), data_sets=(1, 5), reps=10, num_reads=None,
               seed=5):
    import workloads as W

    dev = torch.device("cuda:0")
    rows = []
    for d in data_sets:
        for k in pattern_sets:
            w = W.reads_workload(k, d, seed=seed, num_reads=num_reads)
            tab = pf.Table(w.patterns)
            text = torch.from_numpy(w.text).to(dev)
            ref = None
            for name, plan in ladder_plans(pf):
                res = pf.match(tab, text, plan=plan, hit_cap=w.n // 8 + 1024)
                torch.cuda.synchronize()
                if ref is None:
                    ref = (res.match.clone(), res.num_hits(), res.total())
                else:
                    same = (torch.equal(res.match, ref[0]) and res.num_hits() == ref[1]
                            and res.total() == ref[2])
                    if not same:
                        raise RuntimeError("plan %s differs from plan %s on %s"
                                           % (name, ladder_plans(pf)[0][0], w.name))
                for _ in range(2):
                    pf.match(tab, text, plan=plan, out=res)
                s = torch.cuda.Event(enable_timing=True)
                e = torch.cuda.Event(enable_timing=True)
                s.record()
                for _ in range(reps):
                    pf.match(tab, text, plan=plan, out=res)
                e.record()
                torch.cuda.synchronize()
                ms = s.elapsed_time(e) / reps
                resolved = tab.default_plan(w.n, "ascii") if plan is None else plan
                row = dict(pattern_set=k, data_set=d, patterns=len(w.patterns),
                           reads=w.num_reads, bytes=w.n, plan=name, resolved=resolved,
                           ms=round(ms, 4), gbases_per_s=round(w.n / ms / 1e6, 1),
                           hits=ref[1], total=ref[2])
                rows.append(row)
                print(json.dumps(row), flush=True)
            del text, tab
    return rows


def ladder_table(rows):
    names = LADDER_NAMES
    keys = sorted({(r["data_set"], r["pattern_set"]) for r in rows})
    out = ["| data set | pattern set | " + " | ".join(names) + " |",
           "|---|---|" + "---|" * len(names)]
    for d, k in keys:
        ms = {r["plan"]: r["ms"] for r in rows if r["data_set"] == d and r["pattern_set"] == k}
        out.append("| %d | %d | " % (d, k) + " | ".join("%.3f" % ms[n] for n in names) + " |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", default=None, choices=PARTS,
                    help="run one part only (c1 prints the full contract line)")
    ap.add_argument("--plan", default=None, help="JSON launch plan (default: library choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-mbases", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall seconds of oracle passes for the CPU baseline")
    ap.add_argument("--autotune", action="store_true",
                    help="let the autotuner pick the plans of the packed and batched workloads")
    ap.add_argument("--requests", type=int, default=2000, help="served requests")
    ap.add_argument("--c2-output", default="both", choices=("both", "dense", "hits"),
                    help="outputs timed on the packed workload (profiling runs take one)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (the reference of the HBM "
                         "traffic counters)")
    ap.add_argument("--paper-ladder", action="store_true",
                    help="instead: the paper's placement ladder on paper-shaped pattern and "
                         "read sets (prints one JSON line per case and a table)")
    ap.add_argument("--ladder-pattern-sets", default="1,2,3,4,5")
    ap.add_argument("--ladder-data-sets", default="1,5")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the scan would shard by contiguous start-position ranges with a read-only halo; "
              "see the design notes).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1811_10498_amd as pf

    if args.paper_ladder:
        t0 = time.time()
        rows = run_ladder(pf, torch,
                          tuple(int(x) for x in args.ladder_pattern_sets.split(",")),
                          tuple(int(x) for x in args.ladder_data_sets.split(",")))
        print("milliseconds per call (reads file resident in HBM, dense output + hit list):")
        print(ladder_table(rows))
        print("total %.1f s" % (time.time() - t0))
        return

    torch.cuda.set_device(torch.device("cuda:0"))
    if args.calibrate_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    plan = json.loads(args.plan) if args.plan else None
    parts = PARTS if args.only is None else (args.only,)
    extra = {}
    for part in ("floor", "c0", "c2", "c3", "c4"):
        if part in parts:
            t = time.time()
            print("bench: %s ..." % part, file=sys.stderr, flush=True)
            fn = {"floor": lambda: part_floor(pf, torch, args),
                  "c0": lambda: part_c0(pf, torch, args, plan),
                  "c2": lambda: part_c2(pf, torch, args, plan, tune=args.autotune),
                  "c3": lambda: part_c3(pf, torch, args, plan, tune=args.autotune),
                  "c4": lambda: part_c4(pf, torch, args, plan, num_requests=args.requests)}[part]
            extra[part] = fn()
            extra[part]["bench_s"] = round(time.time() - t, 1)
            torch.cuda.empty_cache()
    if "c1" not in parts:
        print(json.dumps({"parts": extra}), flush=True)
        return
    print("bench: c1 ...", file=sys.stderr, flush=True)
    c1, w = part_c1(pf, torch, args, plan)
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline ...", file=sys.stderr, flush=True)
        cpu = oracle_baseline(w, args.cpu_sample_mbases, args.cpu_seconds)
    names = {"c0": "tiny", "c2": "packed", "c3": "batched", "c4": "served", "floor": "floor"}
    out = {
        "metric": "Gbases/s scanned (plain large-text PFAC scan)",
        "value": round(c1["gbases_per_s"], 2),
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(c1["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": c1["workload"],
            "description": c1["description"],
            "n_bases": c1["n_bases"],
            "encoding": c1["encoding"],
            "patterns": c1["patterns"],
            "trie_states": c1["trie_states"],
            "outputs": c1["outputs"],
            "hits": c1["hits"],
            "occurrences": c1["occurrences"],
            "plan": c1["plan"],
            "parallelism": "single GPU",
        },
        "roofline": c1["roofline"],
        "cpu_baseline": cpu,
        "timing": {"median_ms": round(c1["median_ms"], 4), "min_ms": round(c1["min_ms"], 4),
                   "calls_timed_each": max(args.steps, 20)},
        "end_to_end": c1["end_to_end"],
        "workload_generation_s": c1["workload_generation_s"],
    }
    for k, v in extra.items():
        out[names[k]] = v
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
