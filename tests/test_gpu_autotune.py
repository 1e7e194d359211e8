"""Launch tuning: every search grid size gives bit-identical results, and
the autotuner picks one of its candidates, caches it by shape in a JSON file
and reuses it without running anything."""
import json

import numpy as np
import pytest

import oracle
from synth import make_problem
from tests.parity import compare_topk

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_grid_size_does_not_change_results():
    from paper_2502_20072_amd import L0Search
    p = make_problem(n=500, S=120, D=3, k=30, seed=611, beta=(1.5, -0.8, 0.6), sigma=0.05)
    _say("grid invariance S=120 n=500 D=3 k=30")
    s = L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=30)
    s.gram()
    ref = None
    for w in (1, 7, 256, 1024, 2048):
        s.set_search_grid(w)
        s.search(3, 30)
        out = s.topk()
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), f"grid {w} differs"
            assert np.array_equal(np.nan_to_num(out[2]), np.nan_to_num(ref[2]))
    oi, osse, _ = oracle.topk(p.F, p.y, 3, 30)
    compare_topk(p, 3, 30, ref[0], ref[1], oi, osse)
    from paper_2502_20072_amd import SissoError
    with pytest.raises(SissoError):
        s.set_search_grid(0)
    s.close()
    # several column chunks and tile rows; grids that are and are not a
    # multiple of the eight XCDs the tiles are dealt over
    p = make_problem(n=300, S=300, D=3, k=50, seed=613, beta=(1.5, -0.8, 0.6), sigma=0.05)
    _say("grid invariance S=300 n=300 D=3 k=50")
    s = L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=50)
    s.gram()
    ref = None
    for w in (5, 1000, 1024, 1536):
        s.set_search_grid(w)
        s.search(3, 50)
        out = s.topk()
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), f"grid {w} differs"
    with pytest.raises(SissoError):
        s.set_search_grid(4096)
    s.close()


def test_autotune_picks_caches_and_reuses(tmp_path):
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd import _binding as B
    p = make_problem(n=400, S=150, D=3, k=20, seed=612, beta=(1.5, -0.8, 0.6), sigma=0.05)
    _say("autotune S=150 n=400 D=3 k=20")
    cache = str(tmp_path / "tune.json")
    s = L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=20)
    s.gram()
    g = s.autotune(3, 20, cache)
    assert g in (256, 512, 768, 1024, 1280, 1536, 2048)
    assert B.sisso_l0_search_grid(s.handle) == g
    gi, gs, _ = s.topk()          # the tuning run leaves a complete search behind
    oi, osse, _ = oracle.topk(p.F, p.y, 3, 20)
    compare_topk(p, 3, 20, gi, gs, oi, osse)
    data = json.load(open(cache))
    (key, val), = data.items()
    assert "|D=3|S=256|T=1|P=0" in key and val["search_wgs"] == g and val["ms"] > 0
    # a planted different value in the cache is what a second handle picks up
    data[key]["search_wgs"] = 768
    json.dump(data, open(cache, "w"))
    s2 = L0Search(p.F, p.y, p.task_offsets, D_max=3, k_max=20)
    s2.gram()
    assert s2.autotune(3, 20, cache) == 768
    s2.search(3, 20)
    gi2, gs2, _ = s2.topk()
    assert np.array_equal(gi2, gi) and np.array_equal(gs2, gs)
    s.close()
    s2.close()
