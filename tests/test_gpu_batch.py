"""Batched form: many independent problems in one HIP graph launch.

Batched results must equal the unbatched ones bitwise, on every replay of the
graph (with other GPU work in between), and match the CPU oracle."""
import numpy as np
import pytest

import oracle
from synth import make_problem
from tests.parity import compare_topk

pytestmark = pytest.mark.gpu


def _problems(count=6, seed0=4100):
    rng = np.random.default_rng(7)
    out = []
    for i in range(count):
        S = int(rng.integers(20, 90))
        n = int(rng.integers(40, 300))
        out.append(make_problem(n=n, S=S, D=3, k=10, seed=seed0 + i, beta=(1.5, -0.8, 0.6), sigma=0.3,
                                name=f"batch_{i}"))
    return out


def test_batch_equals_unbatched_and_replays():
    import torch
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd import _binding as B
    probs = _problems()
    print("batch of", len(probs), "problems S =", [p.S for p in probs], flush=True)
    hs = [L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=10) for p in probs]
    ref = []
    for s in hs:
        s.gram().search(3, 10)
        ref.append(s.topk())
    b = B.sisso_l0_batch_create([s.handle for s in hs], 3, 10)
    try:
        for rep in range(3):
            # unrelated eager work between replays
            x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
            (x * x).sum().item()
            B.sisso_l0_batch_launch(b)
            for s, (ri, rs, rc) in zip(hs, ref):
                s.last_D, s.last_k = 3, 10
                gi, gs, gc = s.topk()
                assert np.array_equal(gi, ri) and np.array_equal(gs, rs), f"replay {rep} differs"
                assert np.array_equal(np.nan_to_num(gc), np.nan_to_num(rc))
    finally:
        B.sisso_l0_batch_destroy(b)
    for p, (gi, gs, gc) in zip(probs[:3], ref[:3]):
        oi, osse, _ = oracle.topk(p.F, p.y, 3, 10)
        compare_topk(p, 3, 10, gi, gs, oi, osse, gcoef=gc)
    for s in hs:
        s.close()


def test_one_shot_batch_and_errors():
    from paper_2502_20072_amd import L0Search, SissoError
    from paper_2502_20072_amd import _binding as B
    probs = _problems(count=3, seed0=4200)
    hs = [L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=10) for p in probs]
    B.sisso_l0_search_batch([s.handle for s in hs], 3, 10)
    for p, s in zip(probs, hs):
        s.last_D, s.last_k = 3, 10
        gi, gs, _ = s.topk()
        oi, osse, _ = oracle.topk(p.F, p.y, 3, 10)
        compare_topk(p, 3, 10, gi, gs, oi, osse)
    with pytest.raises(SissoError):
        B.sisso_l0_batch_create([hs[0].handle, hs[0].handle], 3, 10)
    with pytest.raises(SissoError):
        B.sisso_l0_batch_create([s.handle for s in hs], 4, 10)   # D > D_max
    for s in hs:
        s.close()
