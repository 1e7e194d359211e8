"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every case prints its name, seed and shape before it touches the GPU.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from synth import make_config, make_problem, tiny_problem
from tests.parity import compare_topk, total_ss

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(msg, flush=True)


def _run(p, D, k, D_max=None, k_max=None, rng=None):
    from paper_2502_20072_amd import L0Search
    s = L0Search(p.F, p.y, p.task_offsets, D_max=D_max or max(D, 1), k_max=k_max or k)
    s.gram()
    if rng is None:
        s.search(D, k)
    else:
        s.search_range(D, k, *rng)
    out = s.topk()
    s.close()
    return out


def _np_gram(p, t):
    a, b = p.task_offsets[t], p.task_offsets[t + 1]
    X = p.F[:, a:b] - p.F[:, a:b].mean(axis=1, keepdims=True)
    yc = p.y[a:b] - p.y[a:b].mean()
    nrm = np.sqrt(np.sum(X * X, axis=1))
    G = (X @ X.T) / np.outer(nrm, nrm)
    np.fill_diagonal(G, 1.0)
    return G, (X @ yc) / nrm, float(yc @ yc)


@pytest.mark.parametrize("S,n,T", [(1, 7, 1), (37, 50, 1), (128, 300, 1), (200, 100, 1),
                                   (130, 1000, 3), (257, 700, 2)])
def test_gram_matches_numpy(S, n, T):
    from paper_2502_20072_amd import L0Search
    _say(f"gram S={S} n={n} T={T}")
    p = tiny_problem(100 + S, S=S, n=n, T=T, D=1)
    s = L0Search(p.F, p.y, p.task_offsets, D_max=1, k_max=1)
    s.gram()
    for t in range(T):
        G, b, c = s.gram_read(t)
        Gr, br, cr = _np_gram(p, t)
        np.testing.assert_allclose(G, Gr, rtol=0, atol=1e-13)
        assert np.array_equal(G, G.T)
        np.testing.assert_allclose(b, br, rtol=1e-12, atol=1e-12 * math.sqrt(cr))
        assert abs(c - cr) <= 1e-12 * cr
    s.close()


def test_statistics_forms_agree_bitwise():
    """The column statistics hold a task's rows in registers (2 to 32 per
    lane, the smallest count that covers the largest task) or stream them
    (tasks over 2048 rows).  The additions keep the same order in every form,
    so b_t and c_t of the same rows are bitwise equal whichever form the
    other tasks select, and agree with the plain definition to rounding."""
    from paper_2502_20072_amd import L0Search
    rng = np.random.default_rng(77)
    S = 40
    parts = {m: (rng.standard_normal((S, m)) * 3.0 + 1.5, rng.standard_normal(m)) for m in (100, 2000, 2100)}

    def stats(sizes):
        F = np.ascontiguousarray(np.concatenate([parts[m][0] for m in sizes], axis=1))
        y = np.concatenate([parts[m][1] for m in sizes])
        off = np.cumsum([0] + list(sizes)).astype(np.int64)
        s = L0Search(F, y, off, D_max=1, k_max=1)
        s.gram()
        out = {m: s.gram_read(t)[1:] for t, m in enumerate(sizes)}
        s.close()
        return out

    forms = {"2 per lane": stats((100,)), "32 per lane": stats((100, 2000)), "streamed": stats((100, 2000, 2100)),
             "32 per lane, alone": stats((2000,))}
    _say("statistics forms: " + ", ".join(forms))
    for m in (100, 2000):
        got = [(name, f[m]) for name, f in forms.items() if m in f]
        b0, c0 = got[0][1]
        for name, (b, c) in got[1:]:
            assert np.array_equal(b, b0), (m, name)
            assert c == c0, (m, name)
        X, y = parts[m]
        Xc = X - X.mean(axis=1, keepdims=True)
        yc = y - y.mean()
        cr = float(yc @ yc)
        np.testing.assert_allclose(b0, (Xc @ yc) / np.sqrt(np.sum(Xc * Xc, axis=1)), rtol=0,
                                   atol=1e-12 * math.sqrt(cr))
        assert abs(c0 - cr) <= 1e-12 * cr


SWEEP = []
_rng = np.random.default_rng(2024)
for _i in range(40):
    _D = int(_rng.integers(1, 5))
    _T = int(_rng.integers(1, 5))
    _S = int(_rng.integers(_D, 41))
    _n = int(_rng.integers((_D + 2) * _T, 65 + 20 * _T))
    SWEEP.append((1000 + _i, _S, _n, _D, _T))


@pytest.mark.parametrize("seed,S,n,D,T", SWEEP)
def test_tiny_sweep_vs_oracle(seed, S, n, D, T):
    _say(f"sweep seed={seed} S={S} n={n} D={D} T={T}")
    sizes = None
    if T > 1:
        r = np.random.default_rng(seed)
        cuts = np.sort(r.choice(np.arange(1, n), size=T - 1, replace=False))
        sizes = np.diff(np.concatenate([[0], cuts, [n]]))
        if np.any(sizes < D + 2):
            sizes = None
    p = tiny_problem(seed, S=S, n=n, T=T, D=D, sigma=0.3, task_sizes=sizes)
    k = min(12, math.comb(S, D))
    gidx, gsse, gcoef = _run(p, D, k)
    oidx, osse, _ = oracle.topk(p.F, p.y, D, k, p.task_offsets)
    compare_topk(p, D, k, gidx, gsse, oidx, osse, gcoef=gcoef)


@pytest.mark.parametrize("D", [1, 2, 3, 4])
def test_planted_exact_found(D):
    _say(f"planted exact D={D}")
    p = make_problem(n=80, S=70, D=D, k=10, seed=7 + D, beta=(1.5, -0.8, 0.6, -0.4)[:D], sigma=0.0)
    gidx, gsse, _ = _run(p, D, 10)
    assert list(gidx[0]) == p.planted
    assert gsse[0] <= 1e-20 * total_ss(p)


def test_config_plain_s200_d2_golden():
    _say("golden plain_s200_d2")
    g = json.load(open(os.path.join(GOLDEN, "oracle_topk_plain_s200_d2.json")))
    p = make_config("plain_s200_d2")
    gidx, gsse, gcoef = _run(p, g["D"], g["k"])
    compare_topk(p, g["D"], g["k"], gidx, gsse, np.array(g["idx"]), np.array(g["sse"]), gcoef=gcoef)


def test_config_plain_s1000_d3_golden():
    path = os.path.join(GOLDEN, "oracle_topk_plain_s1000_d3.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle result for plain_s1000_d3 not generated")
    _say("golden plain_s1000_d3 (n=2000, S=1000, D=3, k=100)")
    g = json.load(open(path))
    p = make_config("plain_s1000_d3")
    gidx, gsse, gcoef = _run(p, 3, 100)
    compare_topk(p, 3, 100, gidx, gsse, np.array(g["idx"]), np.array(g["sse"]), gcoef=gcoef)
    assert [int(v) for v in gidx[0]] == p.planted


def test_range_split_equals_full():
    _say("range split S=60 n=90 D=3")
    p = tiny_problem(77, S=60, n=90, D=3, sigma=0.4)
    N = math.comb(60, 3)
    k = 40
    fidx, fsse, _ = _run(p, 3, k)
    parts = []
    cuts = [0, 1, 5000, 17111, N]
    for a, b in zip(cuts, cuts[1:]):
        kk = min(k, b - a)
        i, s, _ = _run(p, 3, kk, k_max=k, rng=(a, b))
        for t, v in zip(i, s):
            if np.isfinite(v):
                from paper_2502_20072_amd import rank_of
                r = rank_of(60, t)
                assert a <= r < b
                parts.append((float(v), tuple(int(x) for x in t)))
    parts.sort()
    assert [t for _, t in parts[:k]] == [tuple(int(x) for x in t) for t in fidx]
    np.testing.assert_array_equal([v for v, _ in parts[:k]], fsse)


def test_rank_deficient_never_returned():
    _say("rank-deficient columns S=30")
    p = tiny_problem(78, S=30, n=60, D=3, sigma=0.3)
    F = p.F.copy()
    F[5] = 0.5 * F[3] - 2.0 * F[4] + 1.0     # exact combination
    F[9] = F[3]                              # exact duplicate
    F[12] = 4.0                              # constant
    y = p.y + 3.0 * F[3] - 1.0 * F[4]
    from synth.problems import Problem
    q = Problem(F=F, y=y, task_offsets=p.task_offsets, planted=[], D=3, k=50, exprs=p.exprs, meta={})
    gidx, gsse, _ = _run(q, 3, 50)
    for t in gidx:
        t = tuple(int(v) for v in t)
        assert not {3, 4, 5} <= set(t) and not {3, 9} <= set(t) and 12 not in t
    oidx, osse, _ = oracle.topk(F, y, 3, 50)
    compare_topk(q, 3, 50, gidx, gsse, oidx, osse)


def test_task_constant_column_excluded():
    """A column constant on one task up to rounding (relative 1e-13) makes all
    its tuples rank-deficient, as in the oracle; a relative spread of 1e-3 is
    kept.  Same construction as the oracle's pin, at search size."""
    p = tiny_problem(71, S=30, n=400, T=2, D=3, task_sizes=[180, 220], sigma=0.3)
    F = p.F.copy()
    rng = np.random.default_rng(5)
    F[3, 180:] = 5.0 * (1.0 + 1e-13 * rng.standard_normal(220))
    F[4, 180:] = 5.0 * (1.0 + 1e-3 * rng.standard_normal(220))
    _say("task-constant column S=30 n=400 T=2 D=3")
    from paper_2502_20072_amd import L0Search
    s = L0Search(F, p.y, p.task_offsets, D_max=3, k_max=60)
    s.gram().search(3, 60)
    gi, gs, _ = s.topk()
    G, b, _ = s.gram_read(1)
    s.close()
    assert G[3, 3] == 0.0 and np.all(G[3] == 0.0) and b[3] == 0.0 and G[4, 4] == 1.0
    assert all(3 not in tuple(t) for t in gi)
    q = type(p)(**{**p.__dict__, "F": F})
    oi, osse, _ = oracle.topk(F, p.y, 3, 60, p.task_offsets)
    compare_topk(q, 3, 60, gi, gs, oi, osse)


def test_deterministic_repeat():
    _say("determinism S=120 n=150 D=3")
    p = tiny_problem(79, S=120, n=150, D=3, sigma=0.5)
    a = _run(p, 3, 64)
    b = _run(p, 3, 64)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_abi_errors_and_states():
    from paper_2502_20072_amd import L0Search, SissoError
    from paper_2502_20072_amd import _binding as B
    _say("abi errors")
    p = tiny_problem(80, S=10, n=20, D=2)
    s = L0Search(p.F, p.y, p.task_offsets, D_max=2, k_max=5)
    with pytest.raises(SissoError) as e:
        s.search(2, 5)
    assert e.value.code == B.SISSO_ESTATE
    s.gram()
    for D, k, code in [(3, 5, B.SISSO_ENOTSUP), (0, 5, B.SISSO_EINVAL), (2, 0, B.SISSO_EINVAL),
                       (2, 6, B.SISSO_EINVAL)]:
        with pytest.raises(SissoError) as e:
            s.search(D, k)
        assert e.value.code == code
    with pytest.raises(SissoError) as e:
        B.sisso_l0_topk(s.handle, 5, 2, 1)
    assert e.value.code == B.SISSO_ESTATE
    with pytest.raises(SissoError) as e:
        s.search_range(2, 5, 10, 10)
    assert e.value.code == B.SISSO_EINVAL
    s.search(2, 3)
    with pytest.raises(SissoError) as e:
        s.topk(4)
    assert e.value.code == B.SISSO_ESTATE
    idx, sse, _ = s.topk(3)
    assert np.all(np.isfinite(sse))
    s.close()
    # too few rows in a task for D
    q = tiny_problem(81, S=6, n=9, T=2, D=2, task_sizes=[3, 6])
    s = L0Search(q.F, q.y, q.task_offsets, D_max=2, k_max=3).gram()
    with pytest.raises(SissoError) as e:
        s.search(2, 3)
    assert e.value.code == B.SISSO_EINVAL
    s.close()


def test_nonfinite_input_reported():
    from paper_2502_20072_amd import L0Search, SissoError
    from paper_2502_20072_amd import _binding as B
    _say("non-finite input")
    p = tiny_problem(82, S=8, n=20, D=2)
    F = p.F.copy()
    F[3, 7] = np.nan
    s = L0Search(F, p.y, p.task_offsets, D_max=2, k_max=3).gram().search(2, 3)
    with pytest.raises(SissoError) as e:
        s.topk()
    assert e.value.code == B.SISSO_EINVAL
    s.close()


def test_fewer_valid_tuples_than_k():
    _say("fewer valid tuples than k")
    p = tiny_problem(83, S=4, n=30, D=2, sigma=0.3)
    F = p.F.copy()
    F[1] = F[0]
    F[3] = F[2]
    from synth.problems import Problem
    q = Problem(F=F, y=p.y, task_offsets=p.task_offsets, planted=[], D=2, k=6, exprs=p.exprs, meta={})
    gidx, gsse, _ = _run(q, 2, 6)
    assert np.sum(np.isfinite(gsse)) == 4
    oidx, osse, _ = oracle.topk(F, p.y, 2, 6)
    compare_topk(q, 2, 6, gidx, gsse, oidx, osse)


@pytest.mark.parametrize("S,n,seed", [(3, 12, 90), (5, 20, 91), (129, 70, 92), (131, 60, 93), (257, 50, 94)])
def test_d3_one_task_tile_edges(S, n, seed):
    """One task, D = 3 (pair-record table, two columns per lane, 32-row by
    128-column tiles): sizes at and past the tile and chunk edges (S - 2 rows,
    S odd, S just past 128 and 256), and columns that make pairs rank
    deficient on both sides of a chunk edge."""
    _say(f"d3 one task S={S} n={n} seed={seed}")
    p = tiny_problem(seed, S=S, n=n, D=3, sigma=0.2)
    F = p.F.copy()
    if S > 130:
        F[128] = F[127]                      # duplicate across the first chunk edge
        F[130] = 2.0                         # constant column in the second chunk
        F[S - 1] = 0.5 * F[1] - F[2] + 3.0   # exact combination, last column
    from synth.problems import Problem
    q = Problem(F=F, y=p.y, task_offsets=p.task_offsets, planted=[], D=3, k=40, exprs=p.exprs, meta={})
    k = min(40, math.comb(S, 3))
    gidx, gsse, _ = _run(q, 3, k)
    oidx, osse, _ = oracle.topk(F, p.y, 3, k)
    compare_topk(q, 3, k, gidx, gsse, oidx, osse)
    if S > 130:
        for t in gidx:
            t = set(int(v) for v in t)
            assert not {127, 128} <= t and 130 not in t and not {1, 2, S - 1} <= t


@pytest.mark.parametrize("S,n,T,seed", [(5, 40, 2, 95), (70, 300, 3, 96), (129, 260, 2, 97), (257, 400, 4, 98)])
def test_d3_multitask_filter_task(S, n, T, seed):
    """Several tasks, D = 3: the sweep filters on the task of largest
    |y_t - mean|^2 alone (its SSE bounds the summed SSE from below) and scores
    flagged tuples over every task.  The target is scaled up on a task that is
    not the first, so the filter task is an inner one; a column constant on
    another task and a pair of columns equal on one task only make tuples
    rank deficient in a task the filter does not look at."""
    _say(f"d3 multi-task S={S} n={n} T={T} seed={seed}")
    w = 1.0 + np.random.default_rng(seed).random(T)
    sizes = np.floor(n * w / w.sum()).astype(np.int64)
    sizes[-1] += n - sizes.sum()
    p = tiny_problem(seed, S=S, n=n, T=T, D=3, sigma=0.3, task_sizes=sizes)
    F, y, off = p.F.copy(), p.y.copy(), p.task_offsets
    big = T - 1
    y[off[big]:off[big + 1]] *= 10.0
    if S >= 70:
        F[4, off[0]:off[1]] = 3.0                    # constant on task 0 only
        F[9, off[1]:off[2]] = F[8, off[1]:off[2]]    # equal to column 8 on task 1 only
    from synth.problems import Problem
    q = Problem(F=F, y=y, task_offsets=off, planted=[], D=3, k=30, exprs=p.exprs, meta={})
    k = min(30, math.comb(S, 3))
    gidx, gsse, gcoef = _run(q, 3, k)
    oidx, osse, _ = oracle.topk(F, y, 3, k, off)
    compare_topk(q, 3, k, gidx, gsse, oidx, osse, gcoef=gcoef)
    if S >= 70:
        for t in gidx:
            t = set(int(v) for v in t)
            assert 4 not in t and not {8, 9} <= t


def test_multitask_full_size_sampled():
    """The 16-task workload at full size (S = 1500, 5.6e8 tuples): every
    returned SSE is the oracle's SSE of that tuple, the planted tuple is first,
    and no tuple that shares two features with the best one (4,491 tuples, the
    likeliest competitors) nor a random sample beats the k-th result."""
    p = make_config("multitask_t16_s1500_d3")
    _say(f"multi-task full size S={p.S} T={len(p.task_offsets) - 1} n={p.F.shape[1]}")
    gidx, gsse, _ = _run(p, 3, p.k)
    assert np.all(np.isfinite(gsse)) and np.all(np.diff(gsse) >= 0)
    for t, v in zip(gidx, gsse):
        ref = oracle.tuple_sse(p.F, p.y, tuple(int(x) for x in t), p.task_offsets)
        assert abs(v - ref) <= 1e-10 * ref, (t, v, ref)
    assert tuple(int(x) for x in gidx[0]) == tuple(sorted(p.planted))
    top = {tuple(int(x) for x in t) for t in gidx}
    sk = float(gsse[-1])
    best = [int(x) for x in gidx[0]]
    cands = set()
    for drop in range(3):
        keep = [best[m] for m in range(3) if m != drop]
        for f in range(p.S):
            if f not in keep:
                cands.add(tuple(sorted(keep + [f])))
    rng = np.random.default_rng(11)
    for _ in range(300):
        cands.add(tuple(sorted(int(x) for x in rng.choice(p.S, size=3, replace=False))))
    for t in cands:
        if t in top:
            continue
        assert oracle.tuple_sse(p.F, p.y, t, p.task_offsets) >= sk * (1 - 1e-9), t


def test_d3_multitask_range_split():
    """Several tasks, D = 3, searched in lexicographic rank ranges: each part
    holds only its range's tuples and the merged parts equal the oracle's
    top-k (the range test sits in the queued-step scoring)."""
    _say("d3 multi-task range split S=70 n=360 T=3")
    p = tiny_problem(99, S=70, n=360, T=3, D=3, sigma=0.4, task_sizes=[100, 140, 120])
    N = math.comb(70, 3)
    k = 30
    oidx, osse, _ = oracle.topk(p.F, p.y, 3, k, p.task_offsets)
    parts = []
    cuts = [0, 7, 9000, 30001, N]
    from paper_2502_20072_amd import rank_of
    for a, b in zip(cuts, cuts[1:]):
        kk = min(k, b - a)
        i, s, _ = _run(p, 3, kk, k_max=k, rng=(a, b))
        for t, v in zip(i, s):
            if np.isfinite(v):
                assert a <= rank_of(70, t) < b
                parts.append((float(v), tuple(int(x) for x in t)))
    parts.sort()
    gi = np.array([t for _, t in parts[:k]])
    gs = np.array([v for v, _ in parts[:k]])
    compare_topk(p, 3, k, gi, gs, oidx, osse)


def test_d3_many_tasks():
    """20 tasks (padded to 32): the several-task D = 3 search with 32 lanes
    per tuple in the exact scoring and the one-task-per-workgroup Gram
    finish, against the oracle."""
    _say("d3 20 tasks S=40 n=400")
    sizes = [20] * 20
    p = tiny_problem(101, S=40, n=400, T=20, D=3, sigma=0.3, task_sizes=sizes)
    k = 25
    gidx, gsse, gcoef = _run(p, 3, k)
    oidx, osse, _ = oracle.topk(p.F, p.y, 3, k, p.task_offsets)
    compare_topk(p, 3, k, gidx, gsse, oidx, osse, gcoef=gcoef)


@pytest.mark.parametrize("S,n,seed", [(4, 10, 60), (5, 12, 61), (6, 14, 62), (33, 30, 63), (35, 20, 64),
                                      (66, 24, 65), (129, 22, 66), (131, 20, 67)])
def test_d4_record_table_edges_vs_oracle(S, n, seed):
    """D = 4, one task: the pair-group record-table sweep at sizes around its
    group (4 pairs), row-block (32) and column-chunk (128) edges."""
    _say(f"d4 table edges S={S} n={n}")
    p = tiny_problem(seed, S=S, n=n, D=4, sigma=0.4)
    k = min(40, math.comb(S, 4))
    gidx, gsse, gcoef = _run(p, 4, k)
    oidx, osse, _ = oracle.topk(p.F, p.y, 4, k, p.task_offsets)
    compare_topk(p, 4, k, gidx, gsse, oidx, osse, gcoef=gcoef)


def test_d4_range_split_equals_full():
    _say("d4 range split S=40 n=60")
    p = tiny_problem(78, S=40, n=60, D=4, sigma=0.4)
    N = math.comb(40, 4)
    k = 30
    fidx, fsse, _ = _run(p, 4, k)
    parts = []
    cuts = [0, 1, 20000, 54321, N]
    for a, b in zip(cuts, cuts[1:]):
        i, s, _ = _run(p, 4, min(k, b - a), k_max=k, rng=(a, b))
        for t, v in zip(i, s):
            if np.isfinite(v):
                from paper_2502_20072_amd import rank_of
                assert a <= rank_of(40, t) < b
                parts.append((float(v), tuple(int(x) for x in t)))
    parts.sort()
    assert [t for _, t in parts[:k]] == [tuple(int(x) for x in t) for t in fidx]
    np.testing.assert_array_equal([v for v, _ in parts[:k]], fsse)


def test_d4_constant_and_collinear_columns_never_returned():
    _say("d4 constant / collinear columns")
    p = tiny_problem(79, S=24, n=40, D=4, sigma=0.3)
    F = p.F.copy()
    F[5] = 2.0                        # constant column
    F[9] = 3.0 * F[2] - 1.0           # exactly collinear with column 2 (with the intercept)
    p.F = F
    gidx, gsse, _ = _run(p, 4, 25)
    for t in gidx:
        t = [int(v) for v in t]
        assert 5 not in t and not (2 in t and 9 in t)
    oidx, osse, _ = oracle.topk(p.F, p.y, 4, 25, p.task_offsets)
    compare_topk(p, 4, 25, gidx, gsse, oidx, osse)


@pytest.mark.parametrize("grid", [16, 1024])
def test_full_lists_merge_vs_oracle(grid):
    """A target of pure noise (no tuple stands out) searched over the tuples
    whose first index is below 100 (a rank range, 6.1M tuples, S = 400,
    D = 3, k = 100): the lists fill, so the merge receives more candidates
    (about 3,600) than its selection buffer holds (1,920).  With
    1024 workgroups (4096 lists) the selection first cuts at the KP-th
    smallest of the lists' first entries; with 16 workgroups (64 lists,
    fewer than KP) it sorts every candidate.  Both return the oracle's
    top-k of the range."""
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd import _binding as B
    from synth.problems import Problem
    p = tiny_problem(91, S=400, n=40, T=1, D=3, sigma=0.3)
    y = np.random.default_rng(92).standard_normal(p.n)
    p = Problem(F=p.F, y=y, task_offsets=p.task_offsets, planted=[], D=3, k=100, exprs=p.exprs, meta={})
    r1 = math.comb(p.S, 3) - math.comb(p.S - 100, 3)
    _say(f"full lists S={p.S} n={p.n} ranks [0, {r1}) grid={grid}")
    s = L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=100)
    s.gram()
    s.set_search_grid(grid)
    s.search_range(3, 100, 0, r1)
    gidx, gsse, gcoef = s.topk()
    st = B.sisso_l0_search_stats(s.handle)
    s.close()
    _say(f"candidates offered {st['candidates']}")
    oidx, osse, _ = oracle.topk(p.F, p.y, 3, 100, p.task_offsets, i1_range=(0, 100))
    compare_topk(p, 3, 100, gidx, gsse, oidx, osse, gcoef=gcoef)
