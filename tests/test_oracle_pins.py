"""Pins of the CPU oracle to things other than itself.

Each test checks the oracle (``oracle/oracle_l0.c``) against a fact fixed by
the paper or by mathematics, never against a retyped copy of its own formula:

* library routine: every tuple's SSE and coefficients vs numpy.linalg.lstsq
  (LAPACK's SVD-based solver, a different algorithm from Householder QR);
* exact arithmetic: normal equations solved in fractions.Fraction on
  small-integer data give the exact SSE;
* closed forms: D=1 uses the Pearson coefficient of eq. (1) (SSE = c(1-r^2));
  D=2 the two-predictor R^2 formula; the paper's statement that the 1-D SISSO
  model is the exact l0 one (section "SISSO") means the D=1 ranking is the
  |r| ranking;
* planted targets: exact (SSE ~ 0, rank 1) and noisy (chi-square band);
* invariances: feature/sample permutations, affine rescaling of a feature;
* structure: nesting monotonicity, multi-task = sum of single-task fits,
  range-split merge = whole, number of scored tuples = C(S, D) (the paper's
  printed model counts are exactly binomials, tests/golden).
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import make_config, make_problem, tiny_problem, integer_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lstsq_sse(F, y, tup, offsets=None):
    """Reference: numpy lstsq per task with an explicit ones column."""
    n = F.shape[1]
    offsets = [0, n] if offsets is None else list(offsets)
    total, coefs = 0.0, []
    for t in range(len(offsets) - 1):
        a, b = offsets[t], offsets[t + 1]
        X = np.column_stack([np.ones(b - a)] + [F[j, a:b] for j in tup])
        beta, *_ = np.linalg.lstsq(X, y[a:b], rcond=None)
        r = y[a:b] - X @ beta
        total += float(r @ r)
        coefs.append(beta)
    return total, np.array(coefs)


def centered_ss(v):
    v = np.asarray(v, dtype=np.float64)
    d = v - v.mean()
    return float(d @ d)


@pytest.mark.parametrize("seed,S,n,D,T", [
    (1, 7, 12, 1, 1), (2, 7, 12, 2, 1), (3, 8, 15, 3, 1), (4, 6, 30, 2, 3),
    (5, 8, 40, 3, 2), (6, 9, 25, 4, 1), (7, 5, 50, 5, 1),
])
def test_every_tuple_matches_lstsq(seed, S, n, D, T):
    p = tiny_problem(seed, S=S, n=n, T=T, D=D, sigma=0.3)
    got = oracle.all_sse(p.F, p.y, D, p.task_offsets)
    tuples = list(itertools.combinations(range(S), D))
    assert len(got) == len(tuples)
    c = sum(centered_ss(p.y[p.task_offsets[t]:p.task_offsets[t + 1]]) for t in range(p.T))
    for s, tup in zip(got, tuples):
        ref, _ = lstsq_sse(p.F, p.y, tup, p.task_offsets)
        assert abs(s - ref) <= 1e-12 * max(ref, 1e-3 * c), (tup, s, ref)


def test_coefficients_match_lstsq():
    p = tiny_problem(11, S=6, n=40, T=2, D=3, sigma=0.2)
    for tup in [(0, 1, 2), (1, 3, 5), (0, 4, 5)]:
        s, coef = oracle.tuple_sse(p.F, p.y, tup, p.task_offsets, with_coef=True)
        ref_s, ref_c = lstsq_sse(p.F, p.y, tup, p.task_offsets)
        assert coef.shape == (2, 4)
        np.testing.assert_allclose(coef, ref_c, rtol=1e-10, atol=1e-12)
        assert abs(s - ref_s) <= 1e-12 * ref_s


def _exact_sse(F, y, tup):
    """Exact SSE from the normal equations in rational arithmetic (or None if singular)."""
    n = len(y)
    cols = [[Fraction(1)] * n] + [[Fraction(int(v)) for v in F[j]] for j in tup]
    yy = [Fraction(int(v)) for v in y]
    m = len(cols)
    M = [[sum(a * b for a, b in zip(cols[i], cols[j])) for j in range(m)] for i in range(m)]
    v = [sum(a * b for a, b in zip(cols[i], yy)) for i in range(m)]
    # Gauss-Jordan on [M | v]
    A = [row[:] + [v[i]] for i, row in enumerate(M)]
    for c in range(m):
        piv = next((r for r in range(c, m) if A[r][c] != 0), None)
        if piv is None:
            return None
        A[c], A[piv] = A[piv], A[c]
        for r in range(m):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * z for x, z in zip(A[r], A[c])]
    beta = [A[i][m] / A[i][i] for i in range(m)]
    yty = sum(a * a for a in yy)
    return yty - sum(b * vi for b, vi in zip(beta, v))


@pytest.mark.parametrize("seed,D", [(21, 1), (22, 2), (23, 3)])
def test_exact_rational_sse(seed, D):
    p = integer_problem(seed, S=7, n=14)
    got = oracle.all_sse(p.F, p.y, D)
    c = centered_ss(p.y)
    for s, tup in zip(got, itertools.combinations(range(7), D)):
        ex = _exact_sse(p.F, p.y, tup)
        if ex is None:
            assert s == math.inf
            continue
        ex = float(ex)
        assert abs(s - ex) <= 1e-12 * max(ex, 1e-6 * c), (tup, s, ex)


def _pearson(x, y):
    """Eq. (1) of the paper, written out."""
    xm, ym = x.mean(), y.mean()
    return float(np.sum((x - xm) * (y - ym)) / math.sqrt(np.sum((x - xm) ** 2) * np.sum((y - ym) ** 2)))


def test_d1_is_pearson_closed_form_and_ranking():
    p = make_config("plain_s200_d2")
    c = centered_ss(p.y)
    got = oracle.all_sse(p.F, p.y, 1)
    r = np.array([_pearson(p.F[j], p.y) for j in range(p.S)])
    np.testing.assert_allclose(got, c * (1.0 - r ** 2), rtol=1e-9, atol=1e-11 * c)
    idx, sse, _ = oracle.topk(p.F, p.y, 1, 20)
    by_r = np.argsort(-np.abs(r), kind="stable")[:20]
    assert list(idx[:, 0]) == list(by_r)


def test_d2_two_predictor_r2():
    p = make_config("plain_s200_d2")
    c = centered_ss(p.y)
    rng = np.random.default_rng(0)
    for _ in range(40):
        i, j = sorted(rng.choice(p.S, 2, replace=False))
        r1, r2, r12 = _pearson(p.F[i], p.y), _pearson(p.F[j], p.y), _pearson(p.F[i], p.F[j])
        R2 = (r1 ** 2 + r2 ** 2 - 2 * r1 * r2 * r12) / (1 - r12 ** 2)
        s = oracle.tuple_sse(p.F, p.y, (int(i), int(j)))
        assert abs(s - c * (1 - R2)) <= 1e-9 * c


@pytest.mark.parametrize("D", [1, 2, 3])
def test_planted_exact_target(D):
    p = make_problem(n=60, S=30, D=D, k=5, seed=31 + D, beta=(1.5, -0.8, 0.6)[:D], sigma=0.0)
    c = centered_ss(p.y)
    idx, sse, cnt = oracle.topk(p.F, p.y, D, 5)
    assert cnt == math.comb(30, D)
    assert list(idx[0]) == p.planted
    assert sse[0] <= 1e-20 * c
    assert sse[1] > 1e-8 * c


def test_planted_noisy_chi_square():
    p = make_config("plain_s1000_d3")
    sigma = p.meta["sigma"]
    s = oracle.tuple_sse(p.F, p.y, p.planted)
    dof = p.n - p.D - 1
    z = (s / sigma ** 2 - dof) / math.sqrt(2 * dof)
    assert abs(z) < 5.0


def test_feature_permutation_invariance():
    p = tiny_problem(41, S=12, n=30, D=3, sigma=0.5)
    perm = np.random.default_rng(1).permutation(p.S)
    idx, sse, _ = oracle.topk(p.F, p.y, 3, 15)
    idx2, sse2, _ = oracle.topk(p.F[perm], p.y, 3, 15)
    mapped = [tuple(sorted(perm[list(t)])) for t in idx2]
    np.testing.assert_allclose(sse2, sse, rtol=1e-12)
    # equal SSE sets up to ordering among exact ties
    assert sorted(map(tuple, idx)) == sorted(mapped)


def test_sample_permutation_invariance_per_task():
    p = tiny_problem(42, S=8, n=45, T=3, D=2, sigma=0.5)
    rng = np.random.default_rng(2)
    order = np.concatenate([rng.permutation(np.arange(p.task_offsets[t], p.task_offsets[t + 1]))
                            for t in range(p.T)])
    a = oracle.all_sse(p.F, p.y, 2, p.task_offsets)
    b = oracle.all_sse(p.F[:, order], p.y[order], 2, p.task_offsets)
    np.testing.assert_allclose(a, b, rtol=1e-11)


def test_affine_rescaling_invariance():
    p = tiny_problem(43, S=7, n=25, D=3, sigma=0.4)
    G = p.F.copy()
    G[2] = 37.5 * G[2] - 11.0
    G[5] = -0.01 * G[5] + 3.0
    np.testing.assert_allclose(oracle.all_sse(G, p.y, 3), oracle.all_sse(p.F, p.y, 3), rtol=1e-10)


def test_nesting_monotonicity():
    p = tiny_problem(44, S=10, n=30, D=3, sigma=0.5)
    for tup in itertools.combinations(range(10), 2):
        base = oracle.tuple_sse(p.F, p.y, tup)
        for k in range(10):
            if k in tup:
                continue
            bigger = tuple(sorted(tup + (k,)))
            assert oracle.tuple_sse(p.F, p.y, bigger) <= base * (1 + 1e-12)


def test_multitask_is_sum_of_single_tasks():
    p = tiny_problem(45, S=9, n=70, T=4, D=3, sigma=0.3, task_sizes=[5, 11, 30, 24])
    got = oracle.all_sse(p.F, p.y, 3, p.task_offsets)
    parts = []
    for t in range(p.T):
        a, b = p.task_offsets[t], p.task_offsets[t + 1]
        parts.append(oracle.all_sse(p.F[:, a:b], p.y[a:b], 3))
    np.testing.assert_allclose(got, np.sum(parts, axis=0), rtol=1e-12)


def test_range_split_merge_equals_whole():
    p = tiny_problem(46, S=25, n=40, D=3, sigma=0.5)
    k = 30
    idx, sse, n_all = oracle.topk(p.F, p.y, 3, k)
    pieces = []
    total = 0
    for lo, hi in [(0, 2), (2, 7), (7, 25)]:
        i2, s2, c2 = oracle.topk(p.F, p.y, 3, k, i1_range=(lo, hi))
        total += c2
        pieces += [(s, tuple(t)) for s, t in zip(s2, i2) if np.isfinite(s)]
    pieces.sort()
    assert total == n_all == math.comb(25, 3)
    assert [t for _, t in pieces[:k]] == [tuple(t) for t in idx]
    np.testing.assert_array_equal([s for s, _ in pieces[:k]], sse)


def test_topk_order_and_ties():
    # duplicated column: tuples using column 0 or its copy 5 tie exactly
    p = tiny_problem(47, S=6, n=20, D=2, sigma=0.5)
    F = p.F.copy()
    F[5] = F[0]
    idx, sse, _ = oracle.topk(F, p.y, 2, 15)
    keys = [(s, tuple(t)) for s, t in zip(sse, idx) if np.isfinite(s)]
    assert keys == sorted(keys)
    assert all(tuple(t) != (0, 5) for t in idx)      # (0,5) is rank-deficient


def test_rank_deficient_tuples_are_excluded():
    p = tiny_problem(48, S=6, n=20, D=3, sigma=0.5)
    F = p.F.copy()
    F[2] = 2.0 * F[0] - 0.5 * F[1] + 3.0     # exact linear combination
    F[4] = 7.0                                 # constant column
    assert oracle.tuple_sse(F, p.y, (0, 1, 2)) == math.inf
    assert oracle.tuple_sse(F, p.y, (0, 2, 3)) < math.inf
    assert oracle.tuple_sse(F, p.y, (1, 3, 4)) == math.inf
    assert oracle.tuple_sse(F, p.y, (0, 4)) == math.inf
    idx, sse, _ = oracle.topk(F, p.y, 3, math.comb(6, 3))
    finite = {tuple(t) for t, s in zip(idx, sse) if np.isfinite(s)}
    assert (0, 1, 2) not in finite and all(4 not in t for t in finite)


def test_column_constant_on_a_task_up_to_rounding_is_excluded():
    """A column constant on one task up to a relative 1e-13 has 1 - R^2 on the
    intercept alone (uncentred: |x - mean|^2 / |x|^2) of ~1e-26 there, so every
    tuple using it is rank-deficient; a relative spread of 1e-3 (ratio ~1e-6)
    is kept, and tuples without the column keep their lstsq SSE."""
    p = tiny_problem(53, S=6, n=40, T=2, D=2, task_sizes=[20, 20], sigma=0.5)
    F = p.F.copy()
    rng = np.random.default_rng(5)
    F[3, 20:] = 5.0 * (1.0 + 1e-13 * rng.standard_normal(20))    # task 1: constant up to rounding
    F[4, 20:] = 5.0 * (1.0 + 1e-3 * rng.standard_normal(20))     # task 1: small but real spread
    x3 = F[3, 20:]
    assert np.sum((x3 - x3.mean()) ** 2) / np.sum(x3 ** 2) <= 1e-10
    for t in [(0, 3), (3, 5), (1, 3)]:
        assert oracle.tuple_sse(F, p.y, t, p.task_offsets) == math.inf
    for t in [(0, 4), (4, 5), (0, 1)]:
        s = oracle.tuple_sse(F, p.y, t, p.task_offsets)
        assert abs(s - lstsq_sse(F, p.y, t, p.task_offsets)[0]) <= 1e-9 * s
    idx, sse, _ = oracle.topk(F, p.y, 2, math.comb(6, 2), p.task_offsets)
    finite = {tuple(t) for t, v in zip(idx, sse) if np.isfinite(v)}
    assert all(3 not in t for t in finite) and len(finite) == math.comb(5, 2)


def test_task_row_limits():
    p = tiny_problem(49, S=5, n=6, T=2, D=2, task_sizes=[3, 3], sigma=0.5)
    # n_t = D+1 rows: exact interpolation, SSE 0 up to rounding
    s = oracle.tuple_sse(p.F, p.y, (0, 1), p.task_offsets)
    assert s <= 1e-20
    q = tiny_problem(50, S=5, n=6, T=2, D=2, task_sizes=[2, 4], sigma=0.5)
    assert oracle.tuple_sse(q.F, q.y, (0, 1), q.task_offsets) == math.inf


def test_scored_count_is_binomial_and_paper_counts():
    for S, D in [(9, 1), (9, 4), (12, 3), (10, 5)]:
        p = tiny_problem(51, S=S, n=D + 8, D=D)
        _, _, cnt = oracle.topk(p.F, p.y, D, 3)
        assert cnt == math.comb(S, D)
    rows = [l.split(None, 3) for l in open(os.path.join(GOLDEN, "paper_model_counts.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for S, D, count, _cite in rows:
        assert math.comb(int(S), int(D)) == int(count)


def test_invalid_arguments_raise():
    p = tiny_problem(52, S=5, n=10, D=2)
    with pytest.raises(ValueError):
        oracle.tuple_sse(p.F, p.y, (1, 1))
    with pytest.raises(ValueError):
        oracle.tuple_sse(p.F, p.y, (0, 9))
    with pytest.raises(ValueError):
        oracle.topk(p.F, p.y, 6, 3)
