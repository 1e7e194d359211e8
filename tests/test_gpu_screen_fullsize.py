"""Screening passes at the full workload sizes against the oracle.

A pass creates every candidate of a workload (each binary operator over
every child pair, 2,497,500 candidates), applies the value rules, scores
them against ten residuals (sisso_sis_score_op, the launches bench.py
times) and selects the m best (sisso_topm).  The selection is compared with
the stored oracle result (tests/golden/oracle_sis_<workload>.json, written
by tests/golden/make_golden_sis.py from the CPU oracle only): the same
candidates except those tied with the m-th score within 1e-12, scores to
1e-12.  A seeded sample of candidates is also created and scored by the
oracle one by one, and the stored form (values written out, then
sisso_sis_score) must score them as the fused form does."""
import json
import math
import os

import numpy as np
import pytest

from oracle import sisso_ref as R
from synth import make_screen_workload, screen_digest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WORKLOADS = ["sis_s1000_n2000", "sis_t2_s1000_n156"]


def _say(msg):
    print(f"[screen] {msg}", flush=True)


def _pass(w):
    import torch
    from paper_2502_20072_amd import _binding as B
    dev = "cuda:0"
    X = torch.from_numpy(w.X).to(dev)
    pairs = torch.from_numpy(w.pairs).to(dev)
    h = B.SisScreen(torch.from_numpy(w.R).to(dev), w.task_offsets)
    scores = torch.empty(w.candidates, dtype=torch.float64, device=dev)
    for o, op in enumerate(w.ops):
        h.score_op(op, X, pairs, w.lower, w.upper, scores[o * w.P:(o + 1) * w.P])
    idx = torch.empty(w.m, dtype=torch.int64, device=dev)
    sc = torch.empty(w.m, dtype=torch.float64, device=dev)
    cnt = B.sisso_topm(scores, w.m, idx, sc)
    return h, X, pairs, scores, idx[:cnt].cpu().numpy(), sc[:cnt].cpu().numpy()


@pytest.mark.parametrize("name", WORKLOADS)
def test_screening_pass_against_stored_oracle(name):
    path = os.path.join(GOLDEN, f"oracle_sis_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle result {os.path.basename(path)} not generated")
    g = json.load(open(path))
    w = make_screen_workload(name)
    assert screen_digest(w) == g["input_sha256"], "regenerated inputs differ from the stored result's"
    _say(f"{name}: n={w.n} T={len(w.task_offsets) - 1} children={w.X.shape[0]} candidates={w.candidates} m={w.m}")
    h, X, pairs, scores, gi, gs = _pass(w)
    allsc = scores.cpu().numpy()
    h.close()
    assert int(np.isfinite(allsc).sum()) == g["n_valid"]
    oi, osc = np.array(g["idx"]), np.array(g["score"])
    assert len(gi) == len(oi)
    np.testing.assert_allclose(gs, osc, rtol=0, atol=1e-12)
    sm = osc[-1]
    gset, oset = set(gi.tolist()), set(oi.tolist())
    stray = [c for c in gset ^ oset if abs(allsc[c] - sm) > 1e-12]
    assert not stray, stray[:10]


@pytest.mark.parametrize("name", WORKLOADS)
def test_screening_sampled_candidates_and_stored_form(name):
    import torch
    from paper_2502_20072_amd import _binding as B
    w = make_screen_workload(name)
    h, X, pairs, scores, gi, gs = _pass(w)
    rng = np.random.default_rng(11)
    sample = np.unique(np.concatenate([rng.choice(w.candidates, size=120, replace=False), gi[:8],
                                       [0, w.P - 1, w.P, w.candidates - 1]]))
    got = scores.cpu().numpy()
    _say(f"{name}: {len(sample)} sampled candidates against the oracle")
    res = list(w.R)
    for c in sample:
        o, p = divmod(int(c), w.P)
        vals, ok = R.create(w.ops[o], w.X, w.pairs[p:p + 1], w.lower, w.upper)
        ref = R.sis_score(vals[0], res, w.task_offsets) if ok[0] else float("nan")
        if math.isnan(ref):
            assert math.isnan(got[c]), (c, got[c])
        else:
            assert abs(got[c] - ref) <= 1e-12, (c, got[c], ref)
    # the stored form: the sampled candidates written out, then scored
    Xs = torch.empty((len(sample), w.n), dtype=torch.float64, device="cuda:0")
    v = torch.empty(len(sample), dtype=torch.uint8, device="cuda:0")
    for o, op in enumerate(w.ops):
        sel = np.flatnonzero(sample // w.P == o)
        if len(sel):
            pv = torch.from_numpy(np.ascontiguousarray(w.pairs[sample[sel] % w.P])).to("cuda:0")
            tmp = torch.empty((len(sel), w.n), dtype=torch.float64, device="cuda:0")
            B.sisso_fc_eval(op, X, pv, w.lower, w.upper, tmp, v[:len(sel)])
            Xs[torch.from_numpy(sel).to("cuda:0")] = tmp
    ss = torch.empty(len(sample), dtype=torch.float64, device="cuda:0")
    h.score(Xs, ss)
    st = ss.cpu().numpy()
    h.close()
    fused = got[sample]
    live = np.isfinite(fused)
    np.testing.assert_allclose(st[live], fused[live], rtol=0, atol=1e-13)
