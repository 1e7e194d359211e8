"""The seeded input generator: determinism and the validity rules it applies."""
import numpy as np
import pytest

from synth import CONFIGS, make_config, make_problem, tiny_problem, make_batch_problems
from synth.problems import CORR_DUP


def test_deterministic_by_seed():
    a = make_config("plain_s200_d2")
    b = make_config("plain_s200_d2")
    assert np.array_equal(a.F, b.F) and np.array_equal(a.y, b.y)
    assert a.planted == b.planted
    c = make_config("plain_s200_d2", seed=102)
    assert not np.array_equal(a.F, c.F)


@pytest.mark.parametrize("name", ["plain_s200_d2", "plain_s1000_d3", "learned_s600_d4"])
def test_columns_valid(name):
    p = make_config(name)
    cfg = CONFIGS[name]
    assert p.F.shape == (cfg["S"], cfg["n"])
    assert p.F.flags.c_contiguous and p.F.dtype == np.float64
    assert np.all(np.isfinite(p.F)) and np.all(np.isfinite(p.y))
    assert np.allclose(p.F.mean(axis=1), 0.0, atol=1e-12)
    assert np.allclose(p.F.std(axis=1), 1.0, atol=1e-12)
    # no two kept columns are near-duplicates
    C = (p.F @ p.F.T) / p.n
    np.fill_diagonal(C, 0.0)
    assert np.max(np.abs(C)) <= CORR_DUP + 1e-9
    assert len(p.planted) == p.D and sorted(p.planted) == p.planted


def test_multitask_layout():
    p = make_problem(n=None, S=60, D=3, k=10, seed=7, beta=(1.5, -0.8, 0.6), sigma=0.05,
                     tasks=dict(T=16, lo=50, hi=500))
    offs = p.task_offsets
    assert offs[0] == 0 and offs[-1] == p.n and len(offs) == 17
    sizes = np.diff(offs)
    assert np.all(sizes >= 50) and np.all(sizes <= 500)
    assert len(p.meta["coefs"]) == 16


def test_batch_problem_ranges():
    ps = make_batch_problems(count=3, S_range=(20, 40), n_range=(30, 60))
    for p in ps:
        assert 20 <= p.S <= 40 and 30 <= p.n <= 60


def test_tiny_problem():
    p = tiny_problem(3, S=6, n=17, T=3)
    assert p.F.shape == (6, 17) and p.T == 3 and p.task_offsets[-1] == 17


def test_factor_generator_small():
    """The latent-factor generator of the large-subspace shape: deterministic,
    standardised, correlated but never duplicated columns, planted target."""
    from synth.problems import make_factor_problem
    kw = dict(n=300, S=700, D=2, k=10, seed=3, beta=(1.5, -0.8), sigma=0.0)
    a, b = make_factor_problem(**kw), make_factor_problem(**kw)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.y, b.y) and a.planted == b.planted
    assert a.F.shape == (700, 300) and a.F.flags.c_contiguous
    assert np.allclose(a.F.mean(axis=1), 0.0, atol=1e-12)
    assert np.allclose(a.F.std(axis=1), 1.0, atol=1e-12)
    C = (a.F @ a.F.T) / a.n
    np.fill_diagonal(C, 0.0)
    assert 0.05 < np.median(np.abs(C)) and np.max(np.abs(C)) <= CORR_DUP
    np.testing.assert_allclose(a.y, 1.5 * a.F[a.planted[0]] - 0.8 * a.F[a.planted[1]], atol=1e-12)
    assert make_config("paper_kaggle_s50000_d2", S=700, n=300).F.shape == (700, 300)


def test_decoy_generator():
    """Decoy subspaces: deterministic, standardised, the planted features
    correlate with the target at about 1/sqrt(D), the decoys at r_decoy,
    and the planted tuple fits the target almost exactly."""
    from synth import make_decoy_problem
    a, b = make_decoy_problem(800, 120, 5), make_decoy_problem(800, 120, 5)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.y, b.y) and a.planted == b.planted
    assert np.allclose(a.F.mean(axis=1), 0.0, atol=1e-12) and np.allclose(a.F.std(axis=1), 1.0, atol=1e-12)
    yc = (a.y - a.y.mean()) / a.y.std()
    r = a.F @ yc / a.n
    assert np.all(np.abs(r[a.planted] - 0.5) < 0.1)
    assert len(a.meta["decoys"]) == 20 and abs(np.mean(r[a.meta["decoys"]]) - 0.7) < 0.05
    A = np.column_stack([np.ones(a.n), a.F[a.planted].T])
    res = a.y - A @ np.linalg.lstsq(A, a.y, rcond=None)[0]
    assert res @ res < 1e-2 * ((a.y - a.y.mean()) @ (a.y - a.y.mean()))
