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
