"""FP64 reference of the steps around the l0 search: sure-independence
screening (SIS), feature creation, model residuals and the SISSO dimension
loop.  TEST INFRASTRUCTURE ONLY: the tests call it to check the GPU kernels;
the library never does, and the two share no code.

What it computes (paper, section "SISSO" and "Feature generation and SIS"):

* SIS score of a feature x against a target or residual y: the Pearson
  correlation r of eq. (1), written out as sums over the samples.  With
  several tasks, r_t is taken over each task's rows and the feature scores
  sum_t c_t r_t^2 / sum_t c_t, with c_t = sum_{i in t} (y_i - mean_t y)^2,
  i.e. the share of the total variation that a one-feature fit with an
  intercept per task explains (for one task, r^2, so the order is the order
  of |r|).  This is also 1 - SSE / sum_t c_t of the one-dimensional l0
  model, which the paper notes is the exact l0 solution.  With several
  residuals (the paper keeps the residuals of the best few models of the
  previous dimension) a feature scores its best (largest) value over them.
  A feature that is constant on some task (centred sum of squares <= 1e-10
  of its raw sum of squares there, the l0 search's rule) or has a
  non-finite value has no score (NaN) and is never selected; a task where the residual is identically zero
  contributes nothing.
* Top-m selection: the m largest finite scores, ties by lower index, listed
  by (score descending, index ascending).
* Feature creation: a new feature is an operator applied to one or two child
  features, sample by sample.  Value rules (section "Feature generation and
  SIS"): every value finite, the largest absolute value within
  [lower, upper], and the values not all identical.  The rules the paper
  applies to the children before evaluating (e.g. no zero in a divisor) only
  skip work: each such feature also fails a value rule (a zero divisor
  gives an infinite or NaN value), so they are not repeated here.
* Residual of a model (tuple, intercept and coefficients per task from the
  least-squares fit): y - (alpha_t + X_t beta_t) on each task's rows.
* Dimension loop (section "SISSO", the descriptor-identification flowchart):
  for D = 1 .. D_max, screen every candidate feature not yet in the subspace
  against the target (D = 1) or the residuals of the n_res best models of
  dimension D - 1, append the m_sis best to the subspace, and run the l0
  search of all D-tuples of the subspace.  The subspace matrix lists the
  features in the order they were selected; model tuples are reported as
  sorted global feature indices.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

RANK_EPS = 1e-10

# operator codes (same numbering as the library's feature-creation entry)
BINARY = {"add": 0, "sub": 1, "mul": 2, "div": 3, "abs_diff": 4}
UNARY = {"exp": 16, "neg_exp": 17, "log": 18, "abs": 19, "sqrt": 20, "cbrt": 21, "sq": 22, "cb": 23,
         "inv": 24, "sin": 25, "cos": 26, "six_pow": 27}
OPS = {**BINARY, **UNARY}


def _offsets(n, offsets):
    if offsets is None:
        return np.array([0, n], dtype=np.int64)
    return np.asarray(offsets, dtype=np.int64)


def pearson(x, y) -> float:
    """Eq. (1): sum (x_i - xbar)(y_i - ybar) / sqrt(sum (x_i - xbar)^2 sum (y_i - ybar)^2)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xbar = x.sum() / len(x)
    ybar = y.sum() / len(y)
    num = ((x - xbar) * (y - ybar)).sum()
    den = math.sqrt(((x - xbar) ** 2).sum() * ((y - ybar) ** 2).sum())
    return float(num / den)


def sis_score(x, residuals: Sequence, offsets=None) -> float:
    """SIS score of one feature (see the module text); NaN if it is constant
    on some task."""
    x = np.asarray(x, dtype=np.float64)
    offs = _offsets(len(x), offsets)
    if not np.all(np.isfinite(x)):
        return float("nan")  # eq. (1) is undefined for a non-finite value
    for a, b in zip(offs[:-1], offs[1:]):
        xt = x[a:b]
        c = xt - xt.sum() / len(xt)
        if (c * c).sum() <= RANK_EPS * (xt * xt).sum():
            return float("nan")
    best = -math.inf
    for y in residuals:
        y = np.asarray(y, dtype=np.float64)
        num, den = 0.0, 0.0
        for a, b in zip(offs[:-1], offs[1:]):
            yt = y[a:b]
            ct = float(((yt - yt.sum() / len(yt)) ** 2).sum())
            den += ct
            if ct > 0.0:
                num += ct * pearson(x[a:b], yt) ** 2
        best = max(best, num / den if den > 0.0 else 0.0)
    return float(best)


def sis_scores(X, residuals: Sequence, offsets=None) -> np.ndarray:
    """Scores of every feature; X is (M, n), one feature per row."""
    return np.array([sis_score(x, residuals, offsets) for x in np.asarray(X, dtype=np.float64)])


def top_m(scores, m: int) -> List[int]:
    """Indices of the m largest finite scores, by (score desc, index asc)."""
    s = np.asarray(scores, dtype=np.float64)
    live = [i for i in range(len(s)) if np.isfinite(s[i])]
    live.sort(key=lambda i: (-s[i], i))
    return live[:m]


def apply_op(op: str, a, b=None) -> np.ndarray:
    """Values of op(a, b) (binary) or op(a) (unary), sample by sample."""
    a = np.asarray(a, dtype=np.float64)
    with np.errstate(all="ignore"):
        if op == "add":
            return a + b
        if op == "sub":
            return a - b
        if op == "mul":
            return a * b
        if op == "div":
            return a / b
        if op == "abs_diff":
            return np.abs(a - b)
        if op == "exp":
            return np.exp(a)
        if op == "neg_exp":
            return np.exp(-a)
        if op == "log":
            return np.log(a)
        if op == "abs":
            return np.abs(a)
        if op == "sqrt":
            return np.sqrt(a)
        if op == "cbrt":
            return np.cbrt(a)
        if op == "sq":
            return a * a
        if op == "cb":
            return a * a * a
        if op == "inv":
            return 1.0 / a
        if op == "sin":
            return np.sin(a)
        if op == "cos":
            return np.cos(a)
        if op == "six_pow":
            return (a * a * a) * (a * a * a)
    raise ValueError(op)


def value_valid(v, lower: float, upper: float) -> bool:
    """Value rules: all finite, max |v| in [lower, upper], not all identical."""
    v = np.asarray(v, dtype=np.float64)
    if not np.all(np.isfinite(v)):
        return False
    mx = float(np.max(np.abs(v)))
    if mx < lower or mx > upper:
        return False
    return bool(np.any(v != v[0]))


def create(op: str, X, pairs, lower: float, upper: float):
    """Values (P, n) and validity (P,) of op over candidate child pairs.
    X is (M, n); pairs is (P, 2) (the second entry is ignored for unary ops)."""
    X = np.asarray(X, dtype=np.float64)
    vals, ok = [], []
    for i, j in np.asarray(pairs).reshape(-1, 2):
        v = apply_op(op, X[i], X[j] if op in BINARY else None)
        vals.append(v)
        ok.append(value_valid(v, lower, upper))
    return np.array(vals).reshape(len(ok), X.shape[1]), np.array(ok, dtype=bool)


def model_residual(F, y, tup: Sequence[int], offsets=None):
    """Residual of the least-squares fit with an intercept per task, and the
    coefficients (T, D+1): [alpha_t, beta_t...].  F is (S, n)."""
    F = np.asarray(F, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    offs = _offsets(len(y), offsets)
    r = np.empty_like(y)
    coefs = []
    for a, b in zip(offs[:-1], offs[1:]):
        A = np.column_stack([np.ones(b - a)] + [F[j, a:b] for j in tup])
        beta, *_ = np.linalg.lstsq(A, y[a:b], rcond=None)
        r[a:b] = y[a:b] - A @ beta
        coefs.append(beta)
    return r, np.array(coefs)


def sisso(X, y, offsets, D_max: int, m_sis: int, n_res: int, k: int) -> List[Dict]:
    """The dimension loop (see the module text).  X is (M, n).  Returns, per
    dimension D, the subspace (global indices in selection order) and the
    top-k models (sorted global index tuples and SSEs, by (SSE, lex position
    tuple in the subspace))."""
    import oracle

    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    offs = _offsets(len(y), offsets)
    sub: List[int] = []
    residuals = [y]
    out = []
    for D in range(1, D_max + 1):
        sc = sis_scores(X, residuals, offs)
        for i in sub:
            sc[i] = np.nan
        sub = sub + top_m(sc, m_sis)
        Fs = X[sub]
        kk = min(k, math.comb(len(sub), D))
        pidx, sse, _ = oracle.topk(Fs, y, D, kk, offs)
        models = [tuple(sorted(sub[int(p)] for p in row)) for row, s in zip(pidx, sse) if np.isfinite(s)]
        sses = [float(s) for s in sse if np.isfinite(s)]
        out.append(dict(D=D, subspace=list(sub), models=models, sse=sses,
                        positions=[tuple(int(p) for p in row) for row, s in zip(pidx, sse) if np.isfinite(s)]))
        residuals = [model_residual(X, y, t, offs)[0] for t in models[:n_res]]
    return out
