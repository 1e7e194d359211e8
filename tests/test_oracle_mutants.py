"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake (a dropped term, a wrong sign, an off-by-one
index, a wrong reduction) in a temporary copy of ``oracle/oracle_l0.c``,
builds it with gcc, and checks that at least one of the quick pins below
fails on it, while the unmodified source passes all of them.
"""
import ctypes
import itertools
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from synth import tiny_problem

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle_l0.c")

MUTANTS = {
    "reflector_sign": ("for (i = c; i < nt; ++i) z[i] -= f * x[i];",
                       "for (i = c; i < nt; ++i) z[i] += f * x[i];"),
    "rhs_factor_dropped": ("f = 2.0 * dot / vtv;\n            for (i = c; i < nt; ++i) b[i] -= f * x[i];",
                           "f = dot / vtv;\n            for (i = c; i < nt; ++i) b[i] -= f * x[i];"),
    "tail_off_by_one": ("for (i = ncol; i < nt; ++i) s += b[i] * b[i];",
                        "for (i = ncol + 1; i < nt; ++i) s += b[i] * b[i];"),
    "no_intercept": ("for (i = 0; i < nt; ++i) A[i] = 1.0;",
                     "for (i = 0; i < nt; ++i) A[i] = (double)(i == 0);"),
    "rank_eps_too_loose": ("(alpha * alpha) / cnorm2[c] <= ORACLE_RANK_EPS",
                           "(alpha * alpha) / cnorm2[c] <= 1e-2"),
    "tasks_not_summed": ("task_fit(F, y, n, off[t], off[t + 1], tup, D, work, &st, NULL);\n                    s += st;",
                         "task_fit(F, y, n, off[t], off[t + 1], tup, D, work, &st, NULL);\n                    s = st;"),
    "odometer_skips": ("while (m >= lead && tup[m] == S - D + m) --m;",
                       "while (m >= lead && tup[m] >= S - D + m - 1) --m;"),
    "tie_break_reversed": ("if (a->tup[j] < b->tup[j]) return -1;\n        if (a->tup[j] > b->tup[j]) return 1;",
                           "if (a->tup[j] < b->tup[j]) return 1;\n        if (a->tup[j] > b->tup[j]) return -1;"),
    "coef_transposed_R": ("s -= A[(int64_t)c * nt + j] * x[c];",
                          "s -= A[(int64_t)j * nt + c] * x[c];"),
    "task_rows_shifted": ("for (i = 0; i < nt; ++i) b[i] = y[r0 + i];",
                          "for (i = 0; i < nt; ++i) b[i] = y[i];"),
    "no_intercept_collinearity_rule": ("if (cnorm2[c] <= ORACLE_RANK_EPS * rnorm2[c] ||",
                                       "if (cnorm2[c] == 0.0 ||"),
}


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
                           "-shared", "-o", str(so), str(src), "-lm"])
    return oracle._configure(ctypes.CDLL(str(so)))


def _lstsq(F, y, tup, offs):
    tot, coefs = 0.0, []
    for t in range(len(offs) - 1):
        a, b = offs[t], offs[t + 1]
        X = np.column_stack([np.ones(b - a)] + [F[j, a:b] for j in tup])
        beta, *_ = np.linalg.lstsq(X, y[a:b], rcond=None)
        r = y[a:b] - X @ beta
        tot += float(r @ r)
        coefs.append(beta)
    return tot, np.array(coefs)


def _pins_pass() -> bool:
    """Quick pins; True iff all hold."""
    try:
        # (1) every tuple vs lstsq, multi-task with an offset first task
        p = tiny_problem(61, S=7, n=36, T=2, D=3, sigma=0.3, task_sizes=[14, 22])
        got = oracle.all_sse(p.F, p.y, 3, p.task_offsets)
        for s, tup in zip(got, itertools.combinations(range(7), 3)):
            ref, _ = _lstsq(p.F, p.y, tup, p.task_offsets)
            if not abs(s - ref) <= 1e-10 * ref:
                return False
        # (2) coefficients vs lstsq
        s, coef = oracle.tuple_sse(p.F, p.y, (1, 3, 6), p.task_offsets, with_coef=True)
        _, ref_c = _lstsq(p.F, p.y, (1, 3, 6), p.task_offsets)
        if not np.allclose(coef, ref_c, rtol=1e-9, atol=1e-11):
            return False
        # (3) top-k scored count, order, ties (duplicate column -> exact ties)
        q = tiny_problem(62, S=9, n=25, D=2, sigma=0.5)
        F = q.F.copy()
        F[7] = F[1]
        # tuples (a, 1) and (a, 7) are scored by identical arithmetic: exact ties
        idx, sse, cnt = oracle.topk(F, q.y, 2, 36)
        if cnt != math.comb(9, 2):
            return False
        keys = [(v, tuple(t)) for v, t in zip(sse, idx) if np.isfinite(v)]
        if keys != sorted(keys) or len(keys) != 35:
            return False
        for a in (0,):
            s1, s7 = oracle.tuple_sse(F, q.y, (a, 1)), oracle.tuple_sse(F, q.y, (a, 7))
            if s1 != s7:
                return False
        ref = sorted((_lstsq(F, q.y, t, [0, q.n])[0], t) for t in itertools.combinations(range(9), 2)
                     if t != (1, 7))
        if not np.allclose([v for v, _ in keys], [v for v, _ in ref], rtol=1e-10):
            return False
        pos = [t for _, t in keys]
        if set(pos) != {t for _, t in ref} or pos.index((0, 1)) > pos.index((0, 7)):
            return False
        # (5) multi-task top-k against summed lstsq fits
        idx5, sse5, _ = oracle.topk(p.F, p.y, 3, 6, p.task_offsets)
        ref5 = sorted((_lstsq(p.F, p.y, t, p.task_offsets)[0], t) for t in itertools.combinations(range(7), 3))
        if [t for _, t in ref5[:6]] != [tuple(t) for t in idx5]:
            return False
        # (6) a column constant on one task up to rounding makes its tuples
        #     rank-deficient (1 - uncentred R^2 on the intercept ~1e-26)
        u = tiny_problem(64, S=4, n=30, T=2, D=2, sigma=0.5, task_sizes=[15, 15])
        H = u.F.copy()
        H[2, 15:] = 3.0 * (1.0 + 1e-13 * np.random.default_rng(3).standard_normal(15))
        if oracle.tuple_sse(H, u.y, (0, 2), u.task_offsets) != math.inf:
            return False
        # (4) a moderately collinear (valid) tuple is kept
        r = tiny_problem(63, S=4, n=30, D=2, sigma=0.5)
        G = r.F.copy()
        G[1] = G[0] + 0.05 * G[1]
        if not np.isfinite(oracle.tuple_sse(G, r.y, (0, 1))):
            return False
        return True
    except ValueError:
        return False


@pytest.fixture
def swap_lib():
    saved = oracle._lib
    yield
    oracle._lib = saved


def test_unmodified_oracle_passes(tmp_path, swap_lib):
    oracle._lib = _build(tmp_path, "orig", open(SRC).read())
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path, swap_lib):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique/found"
    oracle._lib = _build(tmp_path, name, text.replace(old, new))
    assert not _pins_pass(), f"planted mistake {name} was not caught"
