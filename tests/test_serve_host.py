"""CPU tests of the serving layer's admission bookkeeping."""
import numpy as np
import pytest

from paper_1811_10498_amd.serve import Admission, Request, summarize


def _req(rid, n, arrival=0.0):
    return Request(rid, 0, [np.zeros(n, dtype=np.uint8)], arrival)


def test_budget_is_never_exceeded_and_order_is_fifo():
    budget = 10 * _req(0, 1000).device_bytes()
    gate = Admission(budget)
    reqs = [_req(i, 1000 * (1 + i % 3)) for i in range(20)]
    for r in reqs:
        gate.offer(r)
    served = []
    live = []
    while len(served) < len(reqs):
        adm = gate.admit()
        assert gate.reserved <= budget
        live += adm
        served += adm
        if live:                          # finish the oldest running request
            gate.release(live.pop(0))
    assert [r.rid for r in served] == list(range(20))   # first come, first served
    for r in live:
        gate.release(r)
    assert gate.reserved == 0


def test_request_larger_than_budget_is_rejected():
    gate = Admission(1000)
    with pytest.raises(ValueError):
        gate.offer(_req(0, 10_000))


def test_head_of_line_request_waits_for_memory():
    big = _req(0, 8000)
    small = _req(1, 10)
    gate = Admission(big.device_bytes() + small.device_bytes() - 1)
    first = _req(2, 10)
    gate.offer(first)
    gate.offer(big)
    gate.offer(small)
    adm = gate.admit()
    assert [r.rid for r in adm] == [2]      # big does not fit next to first; small waits behind it
    gate.release(first)
    assert [r.rid for r in gate.admit()] == [0]


def test_summary_percentiles():
    done = []
    for i in range(100):
        r = _req(i, 100, arrival=i * 0.01)
        r.completed = r.arrival + (i + 1) * 1e-3
        done.append(r)
    s = summarize(done)
    assert s["requests"] == 100 and s["bases"] == 100 * 100
    assert abs(s["p50_ms"] - 50.5) < 1.0 and s["p99_ms"] > 98.0


def test_reservation_covers_what_a_dispatch_allocates():
    """A multi-text request reserves its copied host texts, its int32
    outputs, 12 bytes per hit slot (the rule the dispatch sizes its hit
    buffer with) and its counters."""
    from paper_1811_10498_amd.serve import TextBatch, hit_cap_of
    buf = np.zeros(10_000 * 160, dtype=np.uint8)
    r = Request(0, 0, TextBatch(buf, 160 * np.arange(10_000), np.full(10_000, 150)), 0.0)
    bases = 150 * 10_000
    cap = hit_cap_of(r.lengths)
    assert cap == bases // 16 + 64 * 10_000
    text = (10_000 * 160 - 10 + 15) // 16 * 16
    dispatch = text + 4 * bases + 12 * cap + 8 * (2 + 2 * 10_000)
    assert r.device_bytes() >= dispatch
    assert r.host_text_bytes() == text
