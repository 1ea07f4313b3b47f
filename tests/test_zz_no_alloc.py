"""GPU test of the allocation-free entry point (pfac_match_noalloc): its
scratch is a fixed device array inside the library, so it must give what
pfac_match gives on the same input, call after call, also when a later call
is smaller than an earlier one (the array keeps the earlier call's contents)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_10498_amd as pf  # noqa: E402

DEV = torch.device("cuda:0")


def _outputs(n, cap):
    return pf.MatchResult(torch.full((n,), -7, dtype=torch.int32, device=DEV),
                          torch.full((cap, 2), -7, dtype=torch.int32, device=DEV),
                          torch.full((2,), -7, dtype=torch.int64, device=DEV))


def _same(a, b):
    assert np.array_equal(a.match.cpu().numpy(), b.match.cpu().numpy())
    ca, cb = a.counters.cpu().numpy(), b.counters.cpu().numpy()
    assert np.array_equal(ca, cb), (ca, cb)
    k = int(min(ca[0], a.hits.shape[0]))
    assert np.array_equal(a.hits[:k].cpu().numpy(), b.hits[:k].cpu().numpy())


def _pair(table, text, n, enc="ascii", plan=None):
    cap = n // 8 + 64
    ref = pf.match(table, text, n=n, enc=enc, plan=plan, hit_cap=cap)
    out = _outputs(n, cap)
    got = pf.match(table, text, n=n, enc=enc, plan=plan, out=out, noalloc=True)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("enc", ["ascii", "2bit"])
def test_noalloc_matches_pfac_match_two_calls(enc):
    w = W.plain_workload(1, n=24_000_017, num_patterns=10_000)
    table = pf.Table(w.patterns)
    host = w.text if enc == "ascii" else W.pack2bit(W.ascii_to_codes(w.text))
    text = torch.from_numpy(np.ascontiguousarray(host)).to(DEV)
    print("noalloc: enc=%s n=%d then smaller" % (enc, w.n), flush=True)
    for n in (w.n, 3_000_011):
        if enc == "2bit":
            n -= n % 4
        ref, got = _pair(table, text, n, enc)
        _same(ref, got)


def test_noalloc_plans_and_tiny():
    w = W.plain_workload(0, n=1_000_003)
    table = pf.Table(w.patterns)
    text = torch.from_numpy(w.text).to(DEV)
    for plan in (None, {"walks": pf.PFAC_WALKS_INLINE}, {"variant": pf.PFAC_VARIANT_GLOBAL}):
        for n in (w.n, 4097, 1):
            ref, got = _pair(table, text, n, plan=plan)
            _same(ref, got)


def test_noalloc_rejects_too_large():
    w = W.plain_workload(0, n=1_000)
    table = pf.Table(w.patterns)
    limit = int(table._lib.pfac_noalloc_scratch_bytes())
    assert limit == 64 << 20
    # a real text of 10^9 non-base bytes: needs more scratch than the fixed
    # area holds, so the call is refused on the host before any launch
    n = 1_000_000_000
    text = torch.zeros(n, dtype=torch.uint8, device=DEV)
    out = pf.MatchResult(None, None, torch.zeros(2, dtype=torch.int64, device=DEV))
    with pytest.raises(pf.PfacError) as e:
        pf.match(table, text, n=n, out=out, noalloc=True)
    assert e.value.code == -7
    del text
