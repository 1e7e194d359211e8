"""Pins of the SIS / feature-creation / dimension-loop oracle
(oracle/sisso_ref.py) against things it does not compute itself: a
hand-worked Pearson coefficient, numpy's corrcoef, the l0 oracle's
Householder-QR fits (one-dimensional models), invariances, planted targets
and closed forms of the operators.  Planted mistakes in copies of the oracle
must fail at least one pin."""
import math

import numpy as np
import pytest

import oracle
from oracle import sisso_ref as R
from synth import make_problem, tiny_problem


def _multitask(seed=5, S=12, T=3):
    return tiny_problem(seed, S=S, n=90, T=T, D=1, sigma=0.5, task_sizes=[20, 31, 39][:T])


def _ctot(p, y=None):
    y = p.y if y is None else y
    return sum(float(((y[a:b] - y[a:b].mean()) ** 2).sum()) for a, b in zip(p.task_offsets[:-1], p.task_offsets[1:]))


# ------------------------------------------------------------------ Pearson
def test_pearson_hand_worked():
    # x = (1, 2, 3), y = (2, 4, 7): centred x (-1, 0, 1), centred y
    # (-7/3, -1/3, 8/3); numerator 5, sums of squares 2 and 114/9
    assert abs(R.pearson([1, 2, 3], [2, 4, 7]) - 15 / math.sqrt(228)) <= 1e-15


def test_pearson_matches_numpy_corrcoef():
    rng = np.random.default_rng(1)
    for n in (3, 17, 500):
        x, y = rng.normal(size=n), rng.normal(size=n) + 0.3 * rng.normal(size=n)
        assert abs(R.pearson(x, y) - np.corrcoef(x, y)[0, 1]) <= 1e-13


# -------------------------------------------------------------------- SIS
def test_sis_score_is_one_minus_sse_share_of_the_one_feature_fit():
    # one task and several: the score equals 1 - SSE / sum_t c_t of the
    # one-feature least-squares fit with an intercept per task (QR oracle)
    for p in (tiny_problem(3, S=10, n=60, D=1, sigma=0.7), _multitask()):
        ctot = _ctot(p)
        for j in range(p.S):
            sse = oracle.tuple_sse(p.F, p.y, (j,), p.task_offsets)
            assert abs(R.sis_score(p.F[j], [p.y], p.task_offsets) - (1.0 - sse / ctot)) <= 1e-12


def test_sis_top_m_equals_one_dimensional_l0_ranking():
    p = _multitask(seed=9, S=25)
    sc = R.sis_scores(p.F, [p.y], p.task_offsets)
    oidx, _, _ = oracle.topk(p.F, p.y, 1, 10, p.task_offsets)
    assert R.top_m(sc, 10) == [int(t[0]) for t in oidx]


def test_sis_score_invariances():
    p = _multitask(seed=11)
    x, y = p.F[4], p.y
    base = R.sis_score(x, [y], p.task_offsets)
    assert abs(R.sis_score(-3.0 * x + 7.0, [y], p.task_offsets) - base) <= 1e-12
    assert abs(R.sis_score(x, [0.25 * y - 2.0], p.task_offsets) - base) <= 1e-12
    perm = np.random.default_rng(0).permutation(p.task_offsets[1])   # permute the first task's rows
    x2, y2 = x.copy(), y.copy()
    x2[:len(perm)], y2[:len(perm)] = x[perm], y[perm]
    assert abs(R.sis_score(x2, [y2], p.task_offsets) - base) <= 1e-12


def test_sis_several_residuals():
    p = tiny_problem(21, S=8, n=50, D=1, sigma=0.5)
    r2 = p.y + p.F[2]
    one = R.sis_scores(p.F, [p.y], None)
    two = R.sis_scores(p.F, [p.y, r2], None)
    assert np.all(two >= one - 1e-15)
    # a residual repeated changes nothing; a residual equal to a feature makes
    # that feature's score exactly explain it
    np.testing.assert_array_equal(R.sis_scores(p.F, [p.y, p.y], None), one)
    assert abs(R.sis_scores(p.F, [p.y, p.F[5]], None)[5] - 1.0) <= 1e-12


def test_constant_feature_has_no_score():
    p = _multitask(seed=13)
    x = p.F[0].copy()
    x[p.task_offsets[1]:p.task_offsets[2]] = 2.5       # constant on task 1
    assert math.isnan(R.sis_score(x, [p.y], p.task_offsets))
    sc = np.array([1.0, np.nan, 0.5, 1.0, np.inf * 0])
    assert R.top_m(sc, 5) == [0, 3, 2]


def test_top_m_ties_by_lower_index():
    assert R.top_m([0.5, 0.9, 0.5, 0.9, 0.1], 4) == [1, 3, 0, 2]


# --------------------------------------------------------- feature creation
def test_operators_closed_forms():
    a = np.array([0.5, 1.0, 2.0, 3.0])
    b = np.array([2.0, -1.0, 0.25, 3.0])
    np.testing.assert_allclose(R.apply_op("log", R.apply_op("exp", a)), a, rtol=1e-15)
    np.testing.assert_allclose(R.apply_op("neg_exp", a) * R.apply_op("exp", a), 1.0, rtol=1e-15)
    np.testing.assert_allclose(R.apply_op("sq", R.apply_op("sqrt", a)), a, rtol=1e-15)
    np.testing.assert_allclose(R.apply_op("cb", R.apply_op("cbrt", a)), a, rtol=1e-14)
    np.testing.assert_allclose(R.apply_op("six_pow", a), a ** 6, rtol=1e-15)
    np.testing.assert_allclose(R.apply_op("inv", a) * a, 1.0, rtol=1e-15)
    np.testing.assert_allclose(R.apply_op("abs_diff", a, b), R.apply_op("abs_diff", b, a), rtol=0)
    np.testing.assert_allclose(R.apply_op("div", a, b) * b, a, rtol=1e-15)
    np.testing.assert_allclose(R.apply_op("sin", a) ** 2 + R.apply_op("cos", a) ** 2, 1.0, rtol=1e-15)
    np.testing.assert_array_equal(R.apply_op("sub", a, b), -R.apply_op("sub", b, a))


def test_value_rules():
    X = np.array([[1.0, 2.0, 3.0, 4.0],
                  [0.0, 1.0, 2.0, 3.0],     # a zero: invalid divisor, log -inf
                  [-1.0, 1.0, 2.0, 3.0],    # negative: sqrt / log NaN
                  [2.0, 2.0, 2.0, 2.0],     # constant
                  [1e5, 1.0, 1.0, 1.0]])
    _, ok = R.create("div", X, [(0, 1), (1, 0), (0, 4)], 1e-5, 1e8)
    assert ok.tolist() == [False, True, True]
    _, ok = R.create("log", X, [(1, 0), (2, 0), (0, 0)], 1e-5, 1e8)
    assert ok.tolist() == [False, False, True]
    _, ok = R.create("mul", X, [(0, 3), (3, 3), (4, 4)], 1e-5, 1e8)   # 2x is fine; 4 constant; 1e10 too large
    assert ok.tolist() == [True, False, False]
    _, ok = R.create("sub", X, [(0, 1)], 1e-5, 1e8)                   # all ones: constant
    assert ok.tolist() == [False]
    _, ok = R.create("mul", X * 1e-4, [(0, 0)], 1e-5, 1e8)            # max |v| = 1.6e-7 < lower
    assert ok.tolist() == [False]


# ---------------------------------------------------------------- residuals
def test_model_residual_is_orthogonal_and_matches_sse():
    p = _multitask(seed=17)
    tup = (1, 4, 7)
    r, coef = R.model_residual(p.F, p.y, tup, p.task_offsets)
    assert coef.shape == (p.T, 4)
    for a, b in zip(p.task_offsets[:-1], p.task_offsets[1:]):
        assert abs(r[a:b].sum()) <= 1e-10
        for j in tup:
            assert abs(p.F[j, a:b] @ r[a:b]) <= 1e-10
    assert abs(float(r @ r) - oracle.tuple_sse(p.F, p.y, tup, p.task_offsets)) <= 1e-10 * float(r @ r)


# ----------------------------------------------------------- dimension loop
def test_dimension_loop_finds_planted_models():
    p = make_problem(n=300, S=60, D=2, k=5, seed=88, beta=(1.5, -0.8), sigma=0.01)
    res = R.sisso(p.F, p.y, p.task_offsets, D_max=2, m_sis=10, n_res=5, k=5)
    assert [r["D"] for r in res] == [1, 2]
    s1, s2 = res[0]["subspace"], res[1]["subspace"]
    assert len(s1) == 10 and len(s2) == 20 and len(set(s2)) == 20 and s2[:10] == s1
    # D = 1: the best one-feature model is the best SIS feature
    assert res[0]["models"][0] == (s1[0],)
    # D = 2 finds the planted pair, with SSE at the noise level
    assert res[1]["models"][0] == tuple(p.planted)
    assert res[1]["sse"][0] <= 2.0 * 300 * 0.01 ** 2
    # the second dimension screens against the residuals of the first
    r1 = [R.model_residual(p.F, p.y, t, None)[0] for t in res[0]["models"][:5]]
    sc = R.sis_scores(p.F, r1, None)
    sc[s1] = np.nan
    assert s2[10:] == R.top_m(sc, 10)


# ------------------------------------------------------------ planted mistakes
def _pins_pass():
    try:
        test_pearson_hand_worked()
        test_sis_score_is_one_minus_sse_share_of_the_one_feature_fit()
        test_sis_top_m_equals_one_dimensional_l0_ranking()
        test_sis_several_residuals()
        test_constant_feature_has_no_score()
        test_top_m_ties_by_lower_index()
        test_value_rules()
        test_model_residual_is_orthogonal_and_matches_sse()
    except (AssertionError, AttributeError, TypeError, ValueError):
        return False
    return True


def _pearson_uncentred_y_norm(x, y):
    x, y = np.asarray(x, float), np.asarray(y, float)
    xbar, ybar = x.mean(), y.mean()
    return float(((x - xbar) * (y - ybar)).sum() / math.sqrt(((x - xbar) ** 2).sum() * (y ** 2).sum()))


def _sis_min_over_residuals(x, residuals, offsets=None):
    return min(R.__dict__["_orig_sis_score"](x, [y], offsets) for y in residuals)


def _sis_unweighted(x, residuals, offsets=None):
    offs = R._offsets(len(x), offsets)
    vals = [R.pearson(x[a:b], residuals[0][a:b]) ** 2 for a, b in zip(offs[:-1], offs[1:])]
    return float(np.mean(vals))


def _top_m_high_index(scores, m):
    s = np.asarray(scores, float)
    live = [i for i in range(len(s)) if np.isfinite(s[i])]
    live.sort(key=lambda i: (-s[i], -i))
    return live[:m]


def _valid_no_lower(v, lower, upper):
    v = np.asarray(v, float)
    return bool(np.all(np.isfinite(v)) and np.max(np.abs(v)) <= upper and np.any(v != v[0]))


def _residual_no_intercept(F, y, tup, offsets=None):
    F, y = np.asarray(F, float), np.asarray(y, float)
    offs = R._offsets(len(y), offsets)
    r = np.empty_like(y)
    for a, b in zip(offs[:-1], offs[1:]):
        A = np.column_stack([F[j, a:b] for j in tup])
        beta, *_ = np.linalg.lstsq(A, y[a:b], rcond=None)
        r[a:b] = y[a:b] - A @ beta
    return r, None


@pytest.mark.parametrize("name,attr,fn", [
    ("pearson_uncentred_y_norm", "pearson", _pearson_uncentred_y_norm),
    ("sis_min_over_residuals", "sis_score", _sis_min_over_residuals),
    ("sis_unweighted_tasks", "sis_score", _sis_unweighted),
    ("top_m_high_index_ties", "top_m", _top_m_high_index),
    ("value_rules_no_lower_bound", "value_valid", _valid_no_lower),
    ("residual_no_intercept", "model_residual", _residual_no_intercept),
])
def test_planted_mistake_is_caught(monkeypatch, name, attr, fn):
    assert _pins_pass()
    monkeypatch.setitem(R.__dict__, "_orig_sis_score", R.sis_score)
    monkeypatch.setattr(R, attr, fn)
    assert not _pins_pass(), f"planted mistake {name} passes every pin"


def test_sis_score_non_finite_feature_has_no_score():
    """Eq. (1) is undefined for a feature with a non-finite value: no score,
    whatever the residuals."""
    rng = np.random.default_rng(3)
    y = rng.normal(size=40)
    for bad in (np.inf, -np.inf, np.nan):
        x = rng.normal(size=40)
        x[17] = bad
        assert math.isnan(R.sis_score(x, [y, y * 2.0 + 1.0]))
