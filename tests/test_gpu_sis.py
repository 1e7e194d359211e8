"""Screening, feature creation, residuals, top-m and the dimension loop on the
GPU (through the C ABI of include/sisso_sis.h) against oracle/sisso_ref.py."""
import math

import numpy as np
import pytest

from oracle import sisso_ref as R
from synth import make_problem, tiny_problem

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[sis] {msg}", flush=True)


def _d(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))
    return torch.from_numpy(a).to("cuda:0")


def _problem(seed, S, n, T):
    sizes = None if T == 1 else [n // T + (7 * t) for t in range(T)]
    return tiny_problem(seed, S=S, n=n, T=T, D=2, sigma=0.5, task_sizes=sizes)


@pytest.mark.parametrize("T,nres", [(1, 1), (1, 4), (3, 1), (3, 3), (1, 5), (2, 10), (1, 16)])
def test_sis_scores_match_oracle(T, nres):
    import torch
    from paper_2502_20072_amd import _binding as B
    p = _problem(100 + 10 * T + nres, S=70, n=150, T=T)
    F = p.F.copy()
    F[3, p.task_offsets[-2]:p.task_offsets[-1]] = 1.25     # constant on the last task
    rng = np.random.default_rng(nres)
    res = [p.y] + [p.y - F[j] * rng.uniform(0.5, 1.5) for j in rng.choice(p.S, size=nres - 1, replace=False)]
    _say(f"scores T={T} nres={nres} S={p.S} n={p.n}")
    h = B.SisScreen(_d(np.array(res)), p.task_offsets)
    out = torch.empty(p.S, dtype=torch.float64, device="cuda:0")
    h.score(_d(F), out)
    got = out.cpu().numpy()
    h.close()
    ref = R.sis_scores(F, res, p.task_offsets)
    assert np.array_equal(np.isnan(got), np.isnan(ref)) and np.isnan(got[3])
    live = ~np.isnan(ref)
    np.testing.assert_allclose(got[live], ref[live], rtol=0, atol=1e-12)


@pytest.mark.parametrize("T", [1, 2])
def test_sis_scores_shift_and_cancellation_edges(T):
    """Features whose shifted sums cancel heavily (a spike on the first
    sample of a task with n_t > 1024, a large offset), constant and
    non-finite stored features, and a partial last group of candidates."""
    import torch
    from paper_2502_20072_amd import _binding as B
    n = 3000
    offs = np.array([0, n], dtype=np.int64) if T == 1 else np.array([0, 1300, n], dtype=np.int64)
    rng = np.random.default_rng(40 + T)
    F = rng.normal(size=(70, n))
    for t in range(T):
        a, b = offs[t], offs[t + 1]
        F[0, a:b] = 0.0
        F[0, a] = 1.0                                   # one-hot spike on the task's first sample
        F[1, a:b] = rng.normal(0, 1e-3, b - a)
        F[1, a] = 5.0                                   # spike over small noise
    F[2] = 1e6 + rng.normal(size=n)                     # large offset, unit spread
    F[3] = 1e6 * rng.normal(size=n) + 3e9               # large values, large offset
    F[4] = -2.5                                         # constant everywhere
    F[5, offs[-2]:] = 0.125                             # constant on the last task
    F[6, 11] = np.inf                                   # non-finite values
    F[7, n - 1] = np.nan
    F[8] = rng.normal(size=n) * 1e-150                  # tiny but not constant
    res = [rng.normal(size=n) + F[9] * 0.5, F[10] - 0.3 * F[0], rng.normal(size=n)]
    _say(f"shift/cancellation edges T={T} n={n} M={F.shape[0]}")
    h = B.SisScreen(_d(np.array(res)), offs)
    out = torch.empty(F.shape[0], dtype=torch.float64, device="cuda:0")
    h.score(_d(F), out)
    got = out.cpu().numpy()
    h.close()
    ref = R.sis_scores(F, res, offs)
    assert np.array_equal(np.isnan(got), np.isnan(ref)), (np.flatnonzero(np.isnan(got)), np.flatnonzero(np.isnan(ref)))
    assert all(np.isnan(got[[4, 5, 6, 7]]))
    live = ~np.isnan(ref)
    np.testing.assert_allclose(got[live], ref[live], rtol=0, atol=1e-12)


@pytest.mark.parametrize("M,m", [(1, 1), (1000, 37), (5000, 5000), (3_000_001, 4096)])
def test_topm_matches_oracle_with_ties(M, m):
    import torch
    from paper_2502_20072_amd import _binding as B
    rng = np.random.default_rng(M)
    sc = rng.uniform(0, 1, size=M)
    if M > 10:
        sc[rng.choice(M, size=M // 10, replace=False)] = 0.75         # many exact ties
        sc[rng.choice(M, size=M // 50, replace=False)] = np.nan
        sc[rng.choice(M, size=3, replace=False)] = np.inf              # never selected
        sc[rng.choice(M, size=3, replace=False)] = -0.0
    _say(f"top-m M={M} m={m}")
    out = torch.full((m,), -1, dtype=torch.int64, device="cuda:0")
    osc = torch.empty(m, dtype=torch.float64, device="cuda:0")
    cnt = B.sisso_topm(_d(sc), m, out, osc)
    if M > 100_000:
        # the oracle's sort on the finite scores; same (score desc, index asc) rule
        fin = np.flatnonzero(np.isfinite(sc))
        order = fin[np.lexsort((fin, -sc[fin]))][:m].tolist()
    else:
        order = R.top_m(sc, m)
    assert cnt == len(order)
    assert out[:cnt].cpu().numpy().tolist() == order
    np.testing.assert_array_equal(osc[:cnt].cpu().numpy(), sc[order] + 0.0)


def test_topm_fewer_finite_than_m():
    import torch
    from paper_2502_20072_amd import _binding as B
    sc = np.full(100, np.nan)
    sc[[5, 17, 40]] = [0.1, 0.3, 0.3]
    out = torch.full((10,), -1, dtype=torch.int64, device="cuda:0")
    assert B.sisso_topm(_d(sc), 10, out) == 3
    assert out[:3].cpu().numpy().tolist() == [17, 40, 5]
    assert B.sisso_topm(_d(np.full(8, np.nan)), 4, out) == 0


def _children(seed, n, Mc):
    rng = np.random.default_rng(seed)
    X = rng.lognormal(0, 0.5, size=(Mc, n))
    X[1] = rng.normal(size=n)                 # negative values
    X[2, 3] = 0.0                             # a zero divisor / log(0)
    X[3] = 1.5                                # constant
    X[4] = X[0] * 1e-7                        # tiny values
    X[5] = X[0] * 1e6                         # large values
    return X


@pytest.mark.parametrize("op", list(R.OPS))
def test_fc_eval_matches_oracle(op):
    import torch
    from paper_2502_20072_amd import _binding as B
    n, Mc = 203, 9
    X = _children(7, n, Mc)
    pairs = np.array([(i, j) for i in range(Mc) for j in range(Mc) if i != j or op not in R.BINARY], dtype=np.int32)
    if op not in R.BINARY:
        pairs = np.array([(i, 0) for i in range(Mc)], dtype=np.int32)
    _say(f"feature creation op={op} pairs={len(pairs)}")
    lo, hi = 1e-5, 1e8
    vals, ok = R.create(op, X, pairs, lo, hi)
    out = torch.empty((len(pairs), n), dtype=torch.float64, device="cuda:0")
    valid = torch.empty(len(pairs), dtype=torch.uint8, device="cuda:0")
    B.sisso_fc_eval(op, _d(X), _d(pairs), lo, hi, out, valid)
    gv, gok = out.cpu().numpy(), valid.cpu().numpy().astype(bool)
    assert gok.tolist() == ok.tolist()
    exact = op in ("add", "sub", "mul", "div", "abs_diff", "abs", "sq", "cb", "six_pow", "inv")
    for p in np.flatnonzero(ok):
        if exact:
            np.testing.assert_array_equal(gv[p], vals[p])
        else:
            np.testing.assert_allclose(gv[p], vals[p], rtol=4e-16 * 8, atol=0)
    # the fused screening of the same candidates scores what the oracle scores
    # on the oracle's values
    y = X[0] * 0.7 - 0.2 * X[6] + np.random.default_rng(1).normal(0, 0.1, n)
    h = B.SisScreen(_d(y[None, :]))
    sc = torch.empty(len(pairs), dtype=torch.float64, device="cuda:0")
    v2 = torch.empty(len(pairs), dtype=torch.uint8, device="cuda:0")
    h.score_op(op, _d(X), _d(pairs), lo, hi, sc, v2)
    gs = sc.cpu().numpy()
    h.close()
    assert v2.cpu().numpy().astype(bool).tolist() == ok.tolist()
    for p in range(len(pairs)):
        ref = R.sis_score(vals[p], [y]) if ok[p] else float("nan")
        if math.isnan(ref):
            assert math.isnan(gs[p]), (p, gs[p])
        else:
            assert abs(gs[p] - ref) <= 1e-12, (p, gs[p], ref)


def test_fc_eval_out_of_range_index_is_invalid():
    import torch
    from paper_2502_20072_amd import _binding as B
    X = _children(3, 64, 6)
    pairs = np.array([[0, 1], [0, 6], [-1, 2], [2, 5]], dtype=np.int32)
    valid = torch.full((4,), 7, dtype=torch.uint8, device="cuda:0")
    B.sisso_fc_eval("add", _d(X), _d(pairs), 1e-5, 1e8, None, valid)
    assert valid.cpu().numpy().tolist() == [1, 0, 0, 1]


def test_residuals_match_oracle():
    import torch
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd import _binding as B
    p = _problem(41, S=30, n=120, T=3)
    s = L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=6)
    s.gram().search(3, 6)
    idx, sse, coef = s.topk()
    s.close()
    _say("residuals of 6 models, T=3")
    R_out = torch.empty((6, p.n), dtype=torch.float64, device="cuda:0")
    B.sisso_residuals(_d(p.F), _d(p.y), _d(p.task_offsets), _d(idx.astype(np.int32)), _d(coef), R_out)
    got = R_out.cpu().numpy()
    scale = float(np.abs(p.y).max())
    for q in range(6):
        ref, _ = R.model_residual(p.F, p.y, tuple(int(v) for v in idx[q]), p.task_offsets)
        np.testing.assert_allclose(got[q], ref, rtol=0, atol=1e-11 * scale)
        assert abs(float(got[q] @ got[q]) - sse[q]) <= 1e-9 * sse[q]


@pytest.mark.parametrize("T", [1, 3])
def test_dimension_loop_matches_oracle(T):
    from paper_2502_20072_amd import _binding as B
    tasks = dict(T=T, lo=120, hi=260) if T > 1 else None
    p = make_problem(n=400, S=80, D=3, k=5, seed=900 + T, beta=(1.5, -0.8, 0.6), sigma=0.05, tasks=tasks)
    _say(f"dimension loop T={T} S={p.S} n={p.n}")
    D_max, m_sis, n_res, k = 3, 8, 4, 6
    got = B.sisso_fit(_d(p.F), _d(p.y), p.task_offsets, D_max, m_sis, n_res, k)
    ref = R.sisso(p.F, p.y, p.task_offsets, D_max, m_sis, n_res, k)
    for D in range(1, D_max + 1):
        r = ref[D - 1]
        assert got["subspace"][:D * m_sis].tolist() == r["subspace"], D
        gm = [tuple(int(v) for v in row[:D]) for row in got["models"][D - 1]]
        assert gm == r["models"], (D, gm, r["models"])
        np.testing.assert_allclose(got["sse"][D - 1], r["sse"], rtol=1e-10)
    assert gm[0] == tuple(p.planted)
