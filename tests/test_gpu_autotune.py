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
from paper_1811_10498_amd.autotune import Autotuner, candidate_plans, focused_plans  # noqa: E402
from _gpu_common import check_batch, joined_oracle  # noqa: E402

DEV = torch.device("cuda:0")


def test_tuned_plan_is_a_candidate_and_gives_the_oracle_result(tmp_path):
    w = W.plain_workload(1, n=3_000_001, num_patterns=2000)
    tab = pf.Table(w.patterns)
    text = torch.from_numpy(w.text).to(DEV)
    cands = candidate_plans(blocks=(512, 1024), depths=(8, 9),
                            hashes=(0, pf.PFAC_HASH_NONE), prefixes=(0,), tiles=(2048, 1024))
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


def test_batch_tuning_keeps_a_plan_that_gives_the_oracle_result(tmp_path):
    wb = W.batch_workload(num_texts=400, num_patterns=20000, median=4000.0, hi=200_000, seed=61)
    tab = pf.Table(wb.patterns)
    base = torch.from_numpy(wb.buffer).to(DEV)
    tuner = Autotuner(cache_path=str(tmp_path / "tune.json"), reps=2)
    cands = focused_plans(tab, batch=True)
    res = tuner.tune_batch([tab], base, wb.offsets, wb.lengths, candidates=cands)
    print("batch tuned", res.plan, "%.3f ms" % res.ms, "tried", len(res.tried), flush=True)
    assert res.plan in cands and len(res.tried) >= 8
    texts = [wb.text(t) for t in range(wb.lengths.size)]
    refs = joined_oracle(wb.patterns, texts)
    for plan, _ in [(res.plan, 0)] + res.tried[:4]:
        r = pf.match_batch([tab], base, wb.offsets, wb.lengths, plan=plan,
                           hit_cap=wb.total_bases // 8)
        torch.cuda.synchronize()
        check_batch(r, refs, wb.lengths)
    again = Autotuner(cache_path=str(tmp_path / "tune.json"))
    assert again.tune_batch([tab], base, wb.offsets, wb.lengths).plan == res.plan
