"""Precision form of the Gram (BF16 slices on MFMA, exact FP32 chunk sums,
FP64 accumulation) against FP64 arithmetic and the CPU oracle.

Error bound used below (per sample k, features i and j, chunk maxima
M_i, M_j of the centred values over the 256-sample chunk holding k): with
2^(E-1) <= M < 2^E, x = 2^(E-7) (A + r), A = a_0 + a_1 2^-8 + a_2 2^-16,
|A| < 128 + 2^-17, |r| <= 2^-17.  The kept slice pairs (s + u <= 2) miss
a_1 a_2' 2^-24 + a_2 a_1' 2^-24 + a_2 a_2' 2^-32 (<= 2^-9 + 2^-18) and the
remainders add |A_i r_j| + |r_i A_j| + |r_i r_j| (<= 2^-9 + 2^-33), so the
product of one sample is off by at most 2^(E_i + E_j - 14) (2^-8 + 2^-17)
<= 1.01 * 2^-20 M_i M_j.  Hence
    |G_lp[i, j] - G[i, j]| <= 1.01 * 2^-20 sum_k M_i M_j / (|x_i| |x_j|)
plus FP64 rounding.  The search and the re-score are FP64, so the returned
SSEs match the oracle to the FP64 tolerance.

FP16 form (two slices of 11 bits): x = 2^(E-10) (A + r), A = a_0 + a_1 2^-11,
|A| <= 2^10 + 2^-1, |r| <= 2^-12.  The dropped pair a_1 a_1' 2^-22 (<= 2^-2)
and the remainders (<= 2^-1 + 2^-24) leave at most 0.76 * 2^(E_i + E_j - 20)
<= 3.04 * 2^-20 M_i M_j per sample.  The FP32 chunk sums round: P_0 and P_1
stay below 2^29, so each of the 8 accumulating MFMAs of a chunk, and the
rounding of each 32-term product sum, is off by at most 2^5; over a chunk
<= 2^9 in units of 2^(E_i + E_j - 20), i.e. <= 2^-9 M_i M_j per chunk.
"""
import math

import numpy as np
import pytest

import oracle
from synth import make_config, make_problem
from tests.parity import compare_topk, total_ss

pytestmark = pytest.mark.gpu
XC = 256


def _say(msg):
    print(msg, flush=True)


def _centred(p, t):
    a, b = p.task_offsets[t], p.task_offsets[t + 1]
    return p.F[:, a:b] - p.F[:, a:b].mean(axis=1, keepdims=True)


def _np_gram(X, raw):
    """Correlation matrix of the centred rows X; a row constant up to 1e-10
    (|x - mean|^2 <= 1e-10 |x|^2, x the raw row) is all zeros, diagonal too."""
    ss = np.sum(X * X, axis=1)
    live = ss > 1e-10 * np.sum(raw * raw, axis=1)
    nrm = np.sqrt(ss)
    inv = np.where(live, 1.0 / np.where(live, nrm, 1.0), 0.0)
    G = (X @ X.T) * np.outer(inv, inv)
    np.fill_diagonal(G, live.astype(np.float64))
    return G, nrm, live


def _bound(X, nrm, form="bf16"):
    n = X.shape[1]
    nch = (n + XC - 1) // XC
    Xp = np.zeros((X.shape[0], nch * XC))
    Xp[:, :n] = np.abs(X)
    M = Xp.reshape(X.shape[0], nch, XC).max(axis=2)           # chunk maxima
    cnt = np.full(nch, XC, dtype=np.float64)
    cnt[-1] = n - (nch - 1) * XC
    S_ = (M * cnt) @ M.T                                         # sum over samples of M_i M_j
    if form == "fp16":
        per_chunk = M @ M.T                                      # sum over chunks of M_i M_j
        return (3.04 * 2.0 ** -20 * S_ + 2.0 ** -9 * per_chunk) / np.outer(nrm, nrm) + 1e-13
    return 1.01 * 2.0 ** -20 * S_ / np.outer(nrm, nrm) + 1e-13


def _sampled(S, nsample):
    """The entries the report samples (same multiplicative hash)."""
    out = []
    for e in range(nsample):
        h = ((e + 1) * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
        out.append(((h >> 20) % S, (h >> 40) % S))
    return out


FORMS = ("bf16", "fp16")
SLICES = {"bf16": 3, "fp16": 2}
# the FP32 solve form (f2): FP64 Gram, per-tuple solves in FP32, FP64 re-score
SEARCH_FORMS = FORMS + ("fp32",)


def _lp_search(p, D, k, form="bf16", **kw):
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd import _binding as B
    prec = {"bf16": B.SISSO_PREC_BF16_COMP, "fp16": B.SISSO_PREC_FP16_COMP, "fp32": B.SISSO_PREC_FP32_SOLVE}[form]
    return L0Search(p.F, p.y, p.task_offsets, D_max=D, k_max=k, precision=prec, **kw)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,S,T,seed", [(3000, 150, 1, 311), (1500, 200, 3, 312), (90, 40, 1, 313)])
def test_precision_gram_within_bound_and_report(n, S, T, seed, form):
    _say(f"precision gram form={form} n={n} S={S} T={T} seed={seed}")
    tasks = dict(T=T, lo=n // (2 * T), hi=2 * n // T) if T > 1 else None
    p = make_problem(n=n, S=S, D=2, k=10, seed=seed, beta=(1.5, -0.8), sigma=0.05, tasks=tasks)
    s = _lp_search(p, 2, 10, form)
    s.gram()
    worst = 0.0
    for t in range(p.T):
        G, b, c = s.gram_read(t)
        X = _centred(p, t)
        raw = p.F[:, p.task_offsets[t]:p.task_offsets[t + 1]]
        Gr, nrm, live = _np_gram(X, raw)
        err = np.abs(G - Gr)
        bound = np.where(np.outer(live, live), _bound(X, np.where(live, nrm, 1.0), form), 0.0) + 1e-13
        assert np.all(err <= bound), f"task {t}: max excess {np.max(err - bound)}"
        assert np.array_equal(G, G.T)
        # F^T y and |y|^2 stay exact FP64
        yc = p.y[p.task_offsets[t]:p.task_offsets[t + 1]]
        yc = yc - yc.mean()
        bref = np.where(live, (X @ yc) / np.where(live, nrm, 1.0), 0.0)
        np.testing.assert_allclose(b, bref, rtol=1e-12, atol=1e-12 * math.sqrt(c))
        worst = max(worst, max(err[i, j] for i, j in _sampled(p.S, 512)))
    rep = s.precision_report(512)
    assert rep["slices"] == SLICES[form] and rep["gram_entries"] == 512 * p.T
    assert abs(rep["gram_max_abs_err"] - worst) <= 1e-12
    s.close()


@pytest.mark.parametrize("form", SEARCH_FORMS)
@pytest.mark.parametrize("n,S,D,T,seed", [(4000, 100, 2, 1, 321), (3000, 60, 3, 1, 322), (2400, 45, 3, 3, 323),
                                          (600, 30, 4, 1, 324), (1200, 40, 4, 3, 325)])
def test_precision_search_matches_oracle(n, S, D, T, seed, form):
    _say(f"precision search form={form} n={n} S={S} D={D} T={T} seed={seed}")
    beta = (1.5, -0.8, 0.6, -0.4)[:D]
    tasks = dict(T=T, lo=n // (2 * T), hi=2 * n // T) if T > 1 else None
    p = make_problem(n=n, S=S, D=D, k=20, seed=seed, beta=beta, sigma=0.05, tasks=tasks)
    s = _lp_search(p, D, 20, form)
    s.gram().search(D, 20)
    gi, gs, gc = s.topk()
    rep = s.precision_report(256)
    s.close()
    oi, osse, _ = oracle.topk(p.F, p.y, D, 20, p.task_offsets)
    # the exact re-score of KP = 2 (k + 16) candidates leaves the returned list
    # exact: the FP64 tie band applies
    compare_topk(p, D, 20, gi, gs, oi, osse, gcoef=gc)
    # the ranked (approximate-Gram) SSEs of the results: the FP16 Gram keeps 22
    # bits against 24 and rounds its chunk sums, so its error is a few times
    # larger; the FP32 solves lose ~2^-23 c to cancellation in c - |z|^2 and
    # more when a pivot is small, against SSEs of ~1e-3 c here
    _say(f"ranked SSE error {rep['sse_max_rel_err']:.3e}, Gram error {rep['gram_max_abs_err']:.3e}")
    assert rep["sse_max_rel_err"] < {"bf16": 1e-4, "fp16": 1e-3, "fp32": 1e-1}[form]
    if form == "fp32":
        # the FP32 form's Gram is the FP64 one
        assert rep["slices"] == 0 and rep["gram_max_abs_err"] < 1e-12


@pytest.fixture(scope="module")
def c3():
    _say("generating precision_s4096_d2 (n=50000, S=4096)")
    return make_config("precision_s4096_d2")


def test_precision_full_size_sampled(c3):
    """Full C3 shape: every returned SSE is the oracle's SSE of that tuple, and
    no sampled tuple beats the k-th result (the oracle cannot enumerate all
    8.4e6 tuples at n = 50000 within a test)."""
    p = c3
    _say(f"precision full size n={p.F.shape[1]} S={p.S} D={p.D} k={p.k}")
    s = _lp_search(p, p.D, p.k)
    s.gram().search(p.D, p.k)
    gi, gs, _ = s.topk(with_coef=False)
    rep = s.precision_report(4096)
    s.close()
    _say(f"report {rep}")
    assert np.all(np.isfinite(gs)) and np.all(np.diff(gs) >= 0)
    for t, v in zip(gi, gs):
        ref = oracle.tuple_sse(p.F, p.y, tuple(int(x) for x in t), p.task_offsets)
        assert abs(v - ref) <= 1e-10 * ref, (t, v, ref)
    planted = tuple(sorted(int(x) for x in p.planted))
    assert tuple(int(x) for x in gi[0]) == planted
    rng = np.random.default_rng(7)
    top = {tuple(int(x) for x in t) for t in gi}
    sk = float(gs[-1])
    for _ in range(300):
        t = tuple(sorted(int(x) for x in rng.choice(p.S, size=p.D, replace=False)))
        if t in top:
            continue
        assert oracle.tuple_sse(p.F, p.y, t, p.task_offsets) >= sk * (1 - 1e-9)
    assert rep["gram_max_abs_err"] < 1e-5
