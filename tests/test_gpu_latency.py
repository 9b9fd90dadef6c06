"""GPU: iteration budgets and plain-BP LLR export.

* Latency tail (paper Sec. 7.2): with one solution per decode, the failures of
  a run with iteration budget T (max_total_iters) equal those derived from one
  unbounded run, failed-within-T plus every shot needing more than T.
* Plain BP (paper Sec. 7.1: 25 rounds of standard BP produce the LLRs handed
  to the next stage when memory BP fails; gamma = 0 in Sec. 2.3): the GPU's
  marginals after 25 rounds equal the oracle's bit for bit.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import RELAY_DEFAULT, logical_failures_np
from workloads import codes, sampling

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2511_21660_amd import relaybp

    relaybp.load_library()
    return relaybp


def _decode(rb, prob, prm, syn, want_llr=False):
    dec = rb.Decoder.from_problem(prob, **prm)
    out = dec.decode(torch.from_numpy(np.ascontiguousarray(syn)).cuda(), want_llr=want_llr)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    dec.close()
    return res


def test_budget_ler_from_one_run(rb):
    from paper_2511_21660_amd import latency

    prob = codes.bb_problem("bb144", 0.06)
    faults, syn = sampling.sample_batch(prob, 0x7A11, 0, 20000)
    prm = dict(RELAY_DEFAULT)
    full = _decode(rb, prob, prm, syn)
    fail = logical_failures_np(prob, faults, full["corr"], full["conv"])
    budgets = [1, 20, 60, 150, 400]
    derived = latency.ler_vs_budget(full["iters"], fail, budgets)
    print(f"[latency] bb144 p=0.06 B=20000 derived LER {derived}", flush=True)
    for t, ler in zip(budgets, derived):
        cut = _decode(rb, prob, dict(prm, max_total_iters=t), syn)
        cfail = logical_failures_np(prob, faults, cut["corr"], cut["conv"])
        assert cfail.mean() == ler, t
        keep = full["iters"] <= t
        for k in ("corr", "conv", "legs", "iters"):
            assert np.array_equal(cut[k][keep], full[k][keep]), (t, k)
        assert (cut["iters"][~keep] == t).all() and (cut["conv"][~keep] == 0).all()


def test_plain_bp_llr_export_matches_oracle(rb):
    prob = codes.dem_problem()
    # a tenfold prior makes many syndromes that plain BP does not settle in 25 rounds
    dense = codes.Problem(prob.name, prob.m, prob.n, prob.rows, prob.cols,
                          np.minimum(prob.prior * 10.0, 0.2), prob.logical)
    _, syn = sampling.sample_batch(dense, 0xB925, 0, 600)
    prm = rb.bp_params(25)
    gpu = _decode(rb, dense, prm, syn, want_llr=True)
    ref = oracle.decode(dense.m, dense.n, dense.rows, dense.cols, dense.prior, prm, syn, want_llr=True)
    print(f"[bp-llr] dem B=600 unconverged {int((gpu['conv'] == 0).sum())}", flush=True)
    assert (gpu["conv"] == 0).sum() > 100
    assert np.array_equal(gpu["iters"][gpu["conv"] == 0], np.full((gpu["conv"] == 0).sum(), 25))
    for k in ("corr", "conv", "legs", "iters", "weight", "llr"):
        assert np.array_equal(gpu[k], ref[k]), k
    assert (gpu["legs"] == 1).all()
