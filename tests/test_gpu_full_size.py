"""GPU parity at the full sizes of the plain workloads (256 Mbase Markov ASCII
against 10,000 patterns; 1 Gbase 2-bit packed text against 200,000
patterns), in the launch configuration the benchmark times: the library's
default plan, dense output and hit list, a first call and then a call that
reuses its outputs.  Every position, the total occurrence count and the whole
hit list are compared with the oracle."""
import time

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_10498_amd as pf  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("idx", [1, 2])
def test_full_size_plain_workload_matches_oracle(idx):
    t0 = time.time()
    w = W.plain_workload(idx)
    print("workload %d: n=%d enc=%s patterns=%d (%.1f s)" % (idx, w.n, w.enc, len(w.patterns),
                                                            time.time() - t0), flush=True)
    tab = pf.Table(w.patterns)
    plan = tab.default_plan(w.n, w.enc)
    print("default plan", plan, flush=True)
    dt = torch.from_numpy(w.text).to(DEV)
    res = pf.match(tab, dt, n=w.n, enc=w.enc)
    torch.cuda.synchronize()
    nh = res.num_hits()
    if nh > res.hits.shape[0]:
        res = pf.match(tab, dt, n=w.n, enc=w.enc, hit_cap=nh + 1024)
    # the timed calls write into the outputs of the first one
    res.match.fill_(-1)
    pf.match(tab, dt, n=w.n, enc=w.enc, out=res)
    torch.cuda.synchronize()
    m = res.match.cpu().numpy()
    hits = res.hit_list()
    total = res.total()
    print("gpu done: hits %d total %d (%.1f s)" % (res.num_hits(), total, time.time() - t0),
          flush=True)
    text_ascii = w.text if w.enc == "ascii" else w.ascii()
    m_ref, total_ref = oracle.scan(w.patterns, text_ascii, threads=16)
    print("oracle done (%.1f s)" % (time.time() - t0), flush=True)
    bad = np.nonzero(m != m_ref)[0]
    assert bad.size == 0, "first mismatch at %d: gpu %d oracle %d (%d mismatches)" % (
        bad[0], m[bad[0]], m_ref[bad[0]], bad.size)
    assert total == total_ref
    pos, ids = oracle.hits_of(m_ref)
    assert res.num_hits() == pos.size
    assert np.array_equal(hits[:, 0], pos) and np.array_equal(hits[:, 1], ids)
