"""GPU tests of the launch-plan autotuner: every candidate plan it accepts
gives the oracle's result, the plan it keeps is one of them, and its cache
answers a second call without timing again."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1811_10498_amd as pf  # noqa: E402
from paper_1811_10498_amd.autotune import Autotuner, candidate_plans  # noqa: E402

DEV = torch.device("cuda:0")


def test_tuned_plan_is_a_candidate_and_gives_the_oracle_result(tmp_path):
    w = W.plain_workload(1, n=3_000_001, num_patterns=2000)
    tab = pf.Table(w.patterns)
    text = torch.from_numpy(w.text).to(DEV)
    cands = candidate_plans(blocks=(512, 1024), depths=(8, 9))
    tuner = Autotuner(cache_path=str(tmp_path / "tune.json"), reps=2, sample_bases=1 << 20)
    res = tuner.tune(tab, text, candidates=cands)
    print("tuned", res.plan, "%.3f ms" % res.ms, "tried", len(res.tried), flush=True)
    assert res.plan in cands and len(res.tried) >= 4
    m_ref, total_ref = oracle.scan(w.patterns, w.text, threads=8)
    for plan, _ in res.tried[:6] + [(res.plan, 0)]:
        r = pf.match(tab, text, plan=plan, hit_cap=w.n // 8)
        torch.cuda.synchronize()
        assert np.array_equal(r.match.cpu().numpy(), m_ref), plan
        assert r.total() == total_ref
    again = Autotuner(cache_path=str(tmp_path / "tune.json"))
    assert again.tune(tab, text, candidates=cands).plan == res.plan   # from the file cache
