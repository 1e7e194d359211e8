"""Tie-aware comparison of a GPU top-k against the CPU oracle.

Several top-k lists are correct when SSE values tie, so the comparison
follows one fixed reading: with s_k the oracle's k-th SSE and the tie band
B = {T : |SSE_oracle(T) - s_k| <= tau}, tau = max(1e-9 s_k, 1e-12 c_tot),
the GPU list must contain exactly the oracle's tuples outside B, only tuples
of the oracle list or of B, and k entries (or as many as there are
full-rank tuples).  Every returned SSE must match the oracle's SSE of the
same tuple to a relative 1e-10 (absolute 1e-12 c_tot for SSE below
1e-6 c_tot), and the list must be ordered by (SSE, lexicographic tuple).
"""
from __future__ import annotations

import math

import numpy as np

import oracle


def total_ss(p) -> float:
    c = 0.0
    for t in range(p.T):
        v = p.y[p.task_offsets[t]:p.task_offsets[t + 1]]
        d = v - v.mean()
        c += float(d @ d)
    return c


def compare_topk(p, D, k, gidx, gsse, oidx, osse, rel_tol=1e-10, tie_rel=1e-9, gcoef=None):
    ctot = total_ss(p)
    gl = [tuple(int(v) for v in t) for t, s in zip(gidx, gsse) if np.isfinite(s)]
    ol = [tuple(int(v) for v in t) for t, s in zip(oidx, osse) if np.isfinite(s)]
    assert len(gl) == len(ol), f"GPU returned {len(gl)} full-rank tuples, oracle {len(ol)}"
    # unused rows are marked
    for t, s in zip(gidx, gsse):
        if not np.isfinite(s):
            assert all(v == -1 for v in t)
    if not ol:
        return
    sk = float(osse[len(ol) - 1])
    tau = max(tie_rel * sk, 1e-12 * ctot)
    oset = set(ol)
    gset = set(gl)
    # SSE of each GPU tuple against the oracle's score of that tuple
    for t, s in zip(gl, gsse[:len(gl)]):
        ref = float(osse[ol.index(t)]) if t in oset else oracle.tuple_sse(p.F, p.y, t, p.task_offsets)
        tol = rel_tol * ref if ref >= 1e-6 * ctot else 1e-12 * ctot
        assert abs(s - ref) <= tol, f"SSE mismatch for {t}: gpu {s!r} oracle {ref!r}"
        if t not in oset:
            assert abs(ref - sk) <= tau, f"GPU tuple {t} (SSE {ref}) outside oracle top-k and tie band"
    for t, s in zip(ol, osse[:len(ol)]):
        if t not in gset:
            assert abs(float(s) - sk) <= tau, f"oracle tuple {t} (SSE {s}) missing from GPU top-k"
    # ordering by (SSE, lex)
    keys = list(zip([float(v) for v in gsse[:len(gl)]], gl))
    for a, b in zip(keys, keys[1:]):
        assert a[0] < b[0] or (a[0] == b[0] and a[1] < b[1]) or abs(a[0] - b[0]) <= tau, (a, b)
    # coefficients of the tuples that are common to both, against the oracle's fit
    if gcoef is not None:
        for r, t in enumerate(gl[:5]):
            _, oc = oracle.tuple_sse(p.F, p.y, t, p.task_offsets, with_coef=True)
            np.testing.assert_allclose(gcoef[r], oc, rtol=1e-7, atol=1e-9 * max(1.0, np.max(np.abs(oc))))
