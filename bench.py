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
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KERNEL_SRC = os.path.join(ROOT, "paper_1811_10498_amd", "csrc", "pfac_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, 8 TB/s


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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


def make_workload(name: str):
    import workloads as W
    idx = {"c0": 0, "c1": 1, "c2": 2}[name]
    return W.plain_workload(idx)


def bench_batched(pf, torch, reps=5):
    """Batched workload: 4,096 lognormal texts (~200 Mbase) against one
    50,000-pattern trie in one pfac_match_batch call, against the same texts
    matched one plain pfac_match call each."""
    import numpy as np
    import workloads as W
    wb = W.batch_workload()
    tab = pf.Table(wb.patterns)
    base = torch.from_numpy(wb.buffer).cuda()
    total = wb.total_bases
    cap = total // 16
    res = pf.match_batch([tab], base, wb.offsets, wb.lengths, hit_cap=cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pf.match_batch([tab], base, wb.offsets, wb.lengths, hit_cap=cap,
                       match_out=res.match)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    views = [base[int(o):int(o) + int(L)] for o, L in zip(wb.offsets, wb.lengths)]
    outs = [None] * len(views)
    for i, v in enumerate(views):            # warm and allocate outputs
        outs[i] = pf.match(tab, v, hit_cap=int(v.numel()) // 16 + 64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for v, o in zip(views, outs):
        pf.match(tab, v, out=o)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    return {
        "workload": wb.name, "texts": int(wb.lengths.size), "bases": int(total),
        "patterns": len(wb.patterns), "trie_states": tab.num_states,
        "batched_gbases_per_s": round(total / t_batch / 1e9, 2),
        "batched_ms": round(t_batch * 1e3, 3),
        "plain_per_text_gbases_per_s": round(total / t_plain / 1e9, 2),
        "plain_per_text_ms": round(t_plain * 1e3, 3),
        "speedup_vs_plain": round(t_plain / t_batch, 2),
        "plan": tab.default_plan(),
    }


def bench_served(pf, torch, num_requests=600, load=0.7, plain_requests=60):
    """Served workload: 8 resident tries (1,000 .. 200,000 patterns), requests
    equiprobable among a batch of 10,000 separate 150-base reads, a 1 Mbase
    contig and a 50 Mbase chromosome-like text, texts already in device
    memory.  Closed loop first (capacity), then Poisson arrivals at `load` x
    capacity for latency, and the plain per-request path (one pfac_match call
    per text, synchronised per request) on the first `plain_requests`
    requests of the same stream."""
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

    # closed loop: every request waiting at t=0
    srv = Server(tables, budget_bytes=32 << 30, max_inflight=2)
    srv.run(make([0.0] * num_requests)[:40])          # warm-up
    srv = Server(tables, budget_bytes=32 << 30, max_inflight=2)
    closed = srv.run(make([0.0] * num_requests))
    cap = closed["gbases_per_s"] * 1e9
    # open loop: Poisson arrivals at load x capacity
    bases = sum(int(r.bases) for r in make([0.0] * num_requests))
    rate = load * cap / (bases / num_requests)
    arr = np.cumsum(W.rng(45).exponential(1.0 / rate, size=num_requests))
    srv = Server(tables, budget_bytes=32 << 30, max_inflight=2)
    opened = srv.run(make(arr))
    plain = plain_per_request(tables, make([0.0] * plain_requests, specs[:plain_requests]))
    return {
        "tries": [len(t) for t in tries], "requests": num_requests,
        "bases": closed.get("bases"),
        "capacity_gbases_per_s": round(closed["gbases_per_s"], 2),
        "offered_load": load,
        "served_gbases_per_s": round(opened["gbases_per_s"], 2),
        "p50_ms": round(opened["p50_ms"], 3), "p99_ms": round(opened["p99_ms"], 3),
        "plain_per_request_gbases_per_s": round(plain["gbases_per_s"], 2),
        "plain_requests_timed": plain_requests,
        "speedup_vs_plain": round(closed["gbases_per_s"] / plain["gbases_per_s"], 2),
        "texts": "device-resident (host-to-device copies not in the timed path); reads are "
                 "10,000 separate texts per request",
    }


# ---------------------------------------------------------------- paper ladder
# The paper times its kernel on five pattern sets (1000..5000 patterns of
# about 100 bases) against five read files (0.75 M..3.75 M reads), adding one
# memory placement at a time: global memory only, then the text in shared
# memory, then the table through the texture cache, each with the table as
# two arrays or one merged array (Sec. VI, Tables II and III; Sec. VII).
# --paper-ladder runs that structure with paper-shaped synthetic inputs over
# the placements this library has (merged table throughout; no texture path
# on this GPU), every plan checked bit for bit against the first:
#   global      every position walks from the root, text and table in global
#               memory (the paper's one-thread-per-character kernel);
#   lds-d6      text tile and a depth-6 window bitmap in LDS, deep walks in
#               the global table;
#   lds-d9      the same with a depth-9 bitmap;
#   lds-levels  depth-8 bitmap and the trie levels below it in LDS, the rest
#               in the global table (the hot-prefix-in-LDS split);
#   d9-hash     depth-9 bitmap and the 2^18-bit hashed second filter, walks
#               at once;
#   default     the library's plan (the same filters, walks deferred to the
#               end of each wave).

LADDER_NAMES = ("global", "lds-d6", "lds-d9", "lds-levels", "d9-hash", "default")


def ladder_plans(pf):
    return (
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
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c2"])
    ap.add_argument("--plan", default=None, help="JSON launch plan (default: library choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-mbases", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall seconds of oracle passes for the CPU baseline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-served", action="store_true", help="skip the served workload")
    ap.add_argument("--paper-ladder", action="store_true",
                    help="instead: the paper's placement ladder on paper-shaped pattern and "
                         "read sets (prints one JSON line per case and a table)")
    ap.add_argument("--ladder-pattern-sets", default="1,2,3,4,5")
    ap.add_argument("--ladder-data-sets", default="1,5")
    ap.add_argument("--autotune", action="store_true",
                    help="also time the autotuner's plan (reported beside the default plan)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the scan would shard by contiguous start-position ranges with a read-only halo; "
              "see the design notes).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.time()
    w = make_workload(args.workload)
    t_gen = time.time() - t_gen
    table = pf.Table(w.patterns)
    text = torch.from_numpy(w.text).to(dev)
    plan = json.loads(args.plan) if args.plan else None
    n = w.n
    res = pf.match(table, text, n=n, enc=w.enc, plan=plan)
    torch.cuda.synchronize()
    num_hits, total = res.num_hits(), res.total()
    if num_hits > res.hits.shape[0]:
        res = pf.match(table, text, n=n, enc=w.enc, plan=plan, hit_cap=num_hits + 1024)
    # the GPU raises its clocks only after some milliseconds of work: untimed
    # calls for at least 50 ms first, then the W warm-up steps
    t_warm = time.perf_counter()
    while time.perf_counter() - t_warm < 0.05:
        for _ in range(10):
            pf.match(table, text, n=n, enc=w.enc, plan=plan, out=res)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        pf.match(table, text, n=n, enc=w.enc, plan=plan, out=res)
    torch.cuda.synchronize()

    # the K calls back to back, as a caller issues them; HIP events on the
    # launching stream around the whole timed region give the average
    # duration of one call (events between the calls would add their own
    # gaps to every call)
    K = args.steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for k in range(K):
        pf.match(table, text, n=n, enc=w.enc, plan=plan, out=res)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region_ms = ev0.elapsed_time(ev1)
    assert res.num_hits() == num_hits and res.total() == total

    if args.calibrate_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    ms_per_step = wall * 1e3 / K
    gbases = n * K / wall / 1e9
    avg_launch_s = region_ms / K / 1e3
    text_bytes = n if w.enc == "ascii" else (n + 3) // 4
    alg_bytes = text_bytes + 4 * n + 8 * num_hits + 16 + 16 * table.num_states
    achieved = alg_bytes / avg_launch_s / 1e9
    traffic = read_counters(w.name)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        sample = min(n, args.cpu_sample_mbases << 20)
        host_text = w.ascii(0, sample)
        # repeat the bounded sample for about args.cpu_seconds of wall time
        reps = 0
        t1 = time.perf_counter()
        while True:
            oracle.scan(w.patterns, host_text, threads=threads)
            reps += 1
            dt = time.perf_counter() - t1
            if dt >= args.cpu_seconds or reps >= 1000:
                break
        cpu = {"value": round(sample * reps / dt / 1e9, 4), "unit": "Gbases/s",
               "cores": threads, "kind": "oracle",
               "sample": "first %d Mbase of the same text, all %d patterns, classic "
                         "Aho-Corasick scan split over %d threads, %d passes "
                         "(wall %.2f s, about %.0f core-seconds)"
                         % (sample >> 20, len(w.patterns), threads, reps, dt, dt * threads)}
        # the same oracle on one thread, a smaller sample for about half the time
        sample1 = min(n, 8 << 20)
        text1 = w.ascii(0, sample1)
        reps1 = 0
        t1 = time.perf_counter()
        while True:
            oracle.scan(w.patterns, text1, threads=1)
            reps1 += 1
            dt1 = time.perf_counter() - t1
            if dt1 >= args.cpu_seconds / 2 or reps1 >= 1000:
                break
        cpu["one_thread_value"] = round(sample1 * reps1 / dt1 / 1e9, 4)
        cpu["one_thread_sample"] = ("first %d Mbase, %d passes on one thread (wall %.2f s)"
                                    % (sample1 >> 20, reps1, dt1))

    tuned = None
    if args.autotune:
        # the autotuner's choice on a 128 Mbase sample, timed like the default
        from paper_1811_10498_amd.autotune import Autotuner
        tr = Autotuner(reps=3).tune(table, text, n=n, enc=w.enc)
        s_ev = torch.cuda.Event(enable_timing=True)
        e_ev = torch.cuda.Event(enable_timing=True)
        rt = pf.match(table, text, n=n, enc=w.enc, plan=tr.plan, hit_cap=num_hits + 1024)
        torch.cuda.synchronize()
        assert rt.num_hits() == num_hits and rt.total() == total
        s_ev.record()
        for _ in range(K):
            pf.match(table, text, n=n, enc=w.enc, plan=tr.plan, out=rt)
        e_ev.record()
        torch.cuda.synchronize()
        tms = s_ev.elapsed_time(e_ev) / K
        tuned = {"plan": tr.plan, "candidates_tried": len(tr.tried), "ms_per_step": round(tms, 4),
                 "gbases_per_s": round(n / tms / 1e6, 2)}

    batched = None if args.no_batched else bench_batched(pf, torch)
    served = None if args.no_served else bench_served(pf, torch)

    out = {
        "metric": "Gbases/s scanned (plain large-text PFAC scan)",
        "value": round(gbases, 2),
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "description": w.recipe,
            "n_bases": n,
            "encoding": w.enc,
            "patterns": len(w.patterns),
            "trie_states": table.num_states,
            "outputs": "dense int32 match per position + position-ordered hit list + counts",
            "hits": num_hits,
            "occurrences": total,
            "plan": plan or table.default_plan(n, w.enc),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else int(traffic),
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "avg_launch_ms": round(avg_launch_s * 1e3, 4),
        },
        "cpu_baseline": cpu,
        "autotuned": tuned,
        "batched": batched,
        "served": served,
        "hbm_fraction_of_peak": round(achieved / HBM_PEAK_GBS, 4),
        "workload_generation_s": round(t_gen, 2),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
