"""Seeded synthetic l0 problems with the shape of SISSO's descriptor stage.

What is drawn (paper, section "SISSO" and "Feature generation and SIS"):
primary features are vectors over the samples; candidate features are
expression trees of operators applied to primaries, with the *rung* being the
tree height; invalid features (non-finite values, constants, near-duplicates)
are removed by value-based rules.  The l0 step then searches D-tuples of the
surviving features.  The paper's two data sets (thermal conductivity, NOMAD
2018 band gaps; section "Test Cases") are not available, so every input here
is synthetic: random primaries, random rung<=2 trees, and a target that is
planted as an exact linear combination of a few candidate features plus noise.

Readings of unspecified details (all recorded in the problem's ``meta``):

* primaries ~ lognormal(0, 0.5), i.e. sigma = 0.5 is the standard deviation of
  the underlying normal;
* a tree has rung 1 or 2 with equal probability; its operator is uniform over
  the ten of {+, -, *, /, |a-b|, exp, log, sqrt, ^2, ^3}; rung-1 children are
  primaries; a rung-2 tree has at least one rung-1 child;
* candidates are kept in draw order (the primaries first) until exactly S
  survive: non-finite, zero-variance and |Pearson r| > 0.9999 to any kept
  column are dropped;
* kept columns are standardised over all rows (mean 0, population std 1);
* noise "N(0, s)" uses s as the standard deviation.

Layout: ``F`` has shape (S, n) and is C-contiguous, i.e. it is the n x S matrix
stored column-major (each feature's samples contiguous).  Multi-task problems
store the rows of task t contiguously at [task_offsets[t], task_offsets[t+1]).

This module holds no least-squares arithmetic; it only draws inputs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

BINARY_OPS = ("add", "sub", "mul", "div", "absdiff")
UNARY_OPS = ("exp", "log", "sqrt", "sq", "cb")
ALL_OPS = BINARY_OPS + UNARY_OPS
CORR_DUP = 0.9999


@dataclasses.dataclass
class Problem:
    F: np.ndarray            # (S, n) float64, C-contiguous == n x S column-major
    y: np.ndarray            # (n,) float64
    task_offsets: np.ndarray  # (T+1,) int64
    planted: List[int]        # planted feature indices (sorted)
    D: int
    k: int
    exprs: List[str]
    meta: Dict

    @property
    def S(self) -> int:
        return int(self.F.shape[0])

    @property
    def n(self) -> int:
        return int(self.F.shape[1])

    @property
    def T(self) -> int:
        return int(len(self.task_offsets) - 1)


def _apply(op: str, a: np.ndarray, b: Optional[np.ndarray]) -> np.ndarray:
    with np.errstate(all="ignore"):
        if op == "add":
            return a + b
        if op == "sub":
            return a - b
        if op == "mul":
            return a * b
        if op == "div":
            return a / b
        if op == "absdiff":
            return np.abs(a - b)
        if op == "exp":
            return np.exp(a)
        if op == "log":
            return np.log(a)
        if op == "sqrt":
            return np.sqrt(a)
        if op == "sq":
            return a * a
        if op == "cb":
            return a * a * a
    raise ValueError(op)


def _fmt(op: str, a: str, b: Optional[str]) -> str:
    sym = {"add": "+", "sub": "-", "mul": "*", "div": "/"}
    if op in sym:
        return f"({a} {sym[op]} {b})"
    if op == "absdiff":
        return f"|{a} - {b}|"
    if op in ("sq", "cb"):
        return f"({a})^{2 if op == 'sq' else 3}"
    return f"{op}({a})"


class _TreeSampler:
    """Draws random rung-1 / rung-2 operator trees over the primaries."""

    def __init__(self, rng: np.random.Generator, prim: np.ndarray):
        self.rng = rng
        self.prim = prim
        self.names = [f"x{i}" for i in range(prim.shape[0])]

    def rung1(self):
        rng = self.rng
        op = ALL_OPS[int(rng.integers(len(ALL_OPS)))]
        if op in BINARY_OPS:
            i, j = rng.choice(self.prim.shape[0], size=2, replace=False)
            return _apply(op, self.prim[i], self.prim[j]), _fmt(op, self.names[i], self.names[j])
        i = int(rng.integers(self.prim.shape[0]))
        return _apply(op, self.prim[i], None), _fmt(op, self.names[i], None)

    def rung2(self):
        rng = self.rng
        op = ALL_OPS[int(rng.integers(len(ALL_OPS)))]
        a, ea = self.rung1()
        if op in UNARY_OPS:
            return _apply(op, a, None), _fmt(op, ea, None)
        if rng.random() < 0.5:
            b, eb = self.rung1()
        else:
            j = int(rng.integers(self.prim.shape[0]))
            b, eb = self.prim[j], self.names[j]
        if rng.random() < 0.5:
            a, b, ea, eb = b, a, eb, ea
        return _apply(op, a, b), _fmt(op, ea, eb)

    def draw(self):
        if self.rng.random() < 0.5:
            return self.rung1()
        return self.rung2()


def _unit_centered(x: np.ndarray) -> Optional[np.ndarray]:
    with np.errstate(all="ignore"):
        xc = x - x.mean()
        nrm = math.sqrt(float(xc @ xc))
    if not np.isfinite(nrm) or nrm == 0.0:
        return None
    return xc / nrm


def make_features(rng: np.random.Generator, n: int, S: int, n_primary: int = 10,
                  batch: int = 256, max_draws: Optional[int] = None):
    """Draw candidate features until exactly S survive the validity rules.

    Returns (F, exprs) with F of shape (S, n), standardised per column.
    """
    prim = rng.lognormal(mean=0.0, sigma=0.5, size=(n_primary, n))
    sampler = _TreeSampler(rng, prim)
    kept_raw: List[np.ndarray] = []
    kept_unit = np.empty((S, n), dtype=np.float64)
    exprs: List[str] = []
    m = 0
    draws = 0
    max_draws = max_draws if max_draws is not None else 200 * S + 1000
    queue = [(prim[i], f"x{i}") for i in range(n_primary)]
    while m < S:
        cands = []
        while len(cands) < batch and draws < max_draws:
            if queue:
                v, e = queue.pop(0)
            else:
                v, e = sampler.draw()
            draws += 1
            if not np.all(np.isfinite(v)):
                continue
            u = _unit_centered(v)
            if u is None or not np.all(np.isfinite(u)):
                continue
            cands.append((v, e, u))
        if not cands:
            raise RuntimeError(f"feature generator exhausted after {draws} draws with {m} kept")
        U = np.stack([c[2] for c in cands])
        # |corr| of each candidate against all kept columns (Pearson r of
        # centered unit vectors is their dot product).
        if m > 0:
            cmax = np.max(np.abs(kept_unit[:m] @ U.T), axis=0)
        else:
            cmax = np.zeros(len(cands))
        accepted: List[int] = []
        for j, (v, e, u) in enumerate(cands):
            if m >= S:
                break
            if cmax[j] > CORR_DUP:
                continue
            if accepted:
                cin = np.max(np.abs(U[accepted] @ u))
                if cin > CORR_DUP:
                    continue
            accepted.append(j)
            kept_raw.append(v)
            kept_unit[m] = u
            exprs.append(e)
            m += 1
    F = np.stack(kept_raw)
    mu = F.mean(axis=1, keepdims=True)
    sd = F.std(axis=1, keepdims=True)
    F = np.ascontiguousarray((F - mu) / sd)
    return F, exprs, draws


# Config table: the five workloads (names are their role; sizes from the spec
# of the benchmark); planted coefficients/noise follow the module docstring.
CONFIGS: Dict[str, Dict] = {
    "plain_s200_d2": dict(n=100, S=200, D=2, k=10, seed=101,
                          beta=(1.5, -0.8), sigma=0.01, tasks=None),
    "plain_s1000_d3": dict(n=2000, S=1000, D=3, k=100, seed=202,
                           beta=(1.5, -0.8, 0.6), sigma=0.05, tasks=None),
    "precision_s4096_d2": dict(n=50000, S=4096, D=2, k=100, seed=303,
                               beta=(1.5, -0.8), sigma=0.05, tasks=None),
    "multitask_t16_s1500_d3": dict(n=None, S=1500, D=3, k=100, seed=404,
                                   beta=(1.5, -0.8, 0.6), sigma=0.05,
                                   tasks=dict(T=16, lo=50, hi=5000)),
    "learned_s600_d4": dict(n=2000, S=600, D=4, k=100, seed=505,
                            beta=(1.5, -0.8, 0.6, -0.4), sigma=0.05, tasks=None),
    # the shapes of the paper's two test cases (section "Test Cases"), with
    # synthetic values: the thermal-conductivity case (two tasks of 78 rows,
    # a 5000-feature subspace, D = 3) and the Kaggle band-gap subset (2400
    # samples, a 50,000-feature subspace, D = 2; latent-factor columns, see
    # make_factor_problem)
    "paper_thermal_t2_s5000_d3": dict(n=None, S=5000, D=3, k=100, seed=909,
                                      beta=(1.5, -0.8, 0.6), sigma=0.05,
                                      tasks=dict(T=2, lo=78, hi=79)),
    "paper_kaggle_s50000_d2": dict(n=2400, S=50000, D=2, k=100, seed=910,
                                   beta=(1.5, -0.8), sigma=0.05, tasks=None,
                                   generator="factor"),
}


def _task_sizes(rng: np.random.Generator, T: int, lo: int, hi: int) -> np.ndarray:
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=T))).astype(np.int64)


def make_problem(n: int, S: int, D: int, k: int, seed: int, beta: Sequence[float],
                 sigma: float, tasks: Optional[Dict] = None, name: str = "custom") -> Problem:
    rng = np.random.Generator(np.random.PCG64(seed))
    if tasks is not None:
        sizes = _task_sizes(rng, tasks["T"], tasks["lo"], tasks["hi"])
        n = int(sizes.sum())
        offs = np.zeros(len(sizes) + 1, dtype=np.int64)
        offs[1:] = np.cumsum(sizes)
    else:
        offs = np.array([0, n], dtype=np.int64)
    F, exprs, draws = make_features(rng, n, S)
    planted = sorted(int(i) for i in rng.choice(S, size=len(beta), replace=False))
    T = len(offs) - 1
    y = np.empty(n, dtype=np.float64)
    coefs = []
    base = np.asarray(beta, dtype=np.float64)
    for t in range(T):
        a, b = int(offs[t]), int(offs[t + 1])
        if tasks is not None:
            bt = base * (1.0 + 0.25 * rng.standard_normal(len(base)))
            at = float(rng.uniform(-1.0, 1.0))
        else:
            bt, at = base, 0.0
        y[a:b] = at + bt @ F[planted, a:b] + sigma * rng.standard_normal(b - a)
        coefs.append((at, bt.tolist()))
    meta = dict(name=name, seed=seed, n=n, S=S, D=D, k=k, sigma=sigma,
                planted=planted, coefs=coefs, draws=draws, T=T)
    return Problem(F=F, y=y, task_offsets=offs, planted=planted, D=D, k=k,
                   exprs=exprs, meta=meta)


def make_config(name: str, seed: Optional[int] = None, **override) -> Problem:
    cfg = dict(CONFIGS[name])
    if seed is not None:
        cfg["seed"] = seed
    cfg.update(override)
    if cfg.pop("generator", "trees") == "factor":
        return make_factor_problem(name=name, **cfg)
    return make_problem(name=name, **cfg)


def make_factor_problem(n: int, S: int, D: int, k: int, seed: int, beta: Sequence[float],
                        sigma: float, tasks: Optional[Dict] = None, n_factors: int = 20,
                        name: str = "custom") -> Problem:
    """A large subspace of mutually correlated features, as a screening step
    leaves it: column j = z a_j + e_j with z (n x n_factors) latent factors
    ~ N(0, 1), loadings a_j ~ N(0, 1) and own noise e_j ~ N(0, 1), then
    standardised.  The tree generator's duplicate filter compares every
    candidate with every kept column (S^2 n operations), which is minutes at
    S = 50,000; here no two columns are near-duplicates by construction (each
    has its own unit-variance noise).  The target is planted on D columns
    drawn without replacement, plus N(0, sigma^2) noise; one task."""
    assert tasks is None
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n, n_factors))
    F = np.empty((S, n), dtype=np.float64)
    step = 4096
    for j0 in range(0, S, step):
        j1 = min(S, j0 + step)
        a = rng.standard_normal((n_factors, j1 - j0))
        F[j0:j1] = (z @ a + rng.standard_normal((n, j1 - j0))).T
    F -= F.mean(axis=1, keepdims=True)
    F /= F.std(axis=1, keepdims=True)
    planted = sorted(int(i) for i in rng.choice(S, size=len(beta), replace=False))
    y = np.asarray(beta, dtype=np.float64) @ F[planted] + sigma * rng.standard_normal(n)
    offs = np.array([0, n], dtype=np.int64)
    meta = dict(name=name, seed=seed, n=n, S=S, D=D, k=k, sigma=sigma, planted=planted,
                coefs=[(0.0, list(beta))], draws=S, T=1, generator="factor", n_factors=n_factors)
    return Problem(F=np.ascontiguousarray(F), y=y, task_offsets=offs, planted=planted, D=D, k=k,
                   exprs=[f"f{j}" for j in range(S)], meta=meta)


def make_decoy_problem(n: int, S: int, seed: int, D: int = 4, k: int = 100, r_decoy: float = 0.7,
                       frac_decoy: float = 1 / 6, sigma: float = 0.05) -> Problem:
    """A subspace in which many features are noisy proxies of the target.

    The target is the sum of D mutually independent N(0, 1) features plus
    N(0, sigma^2) noise, so each of them correlates with it at about
    1 / sqrt(D); a fraction frac_decoy of the other features are decoys, the
    standardised target plus independent noise scaled so that each
    correlates with it at r_decoy (and, through the target, with each
    other); the rest are independent N(0, 1).  A screening step that ranks
    features one by one keeps such decoys, and pairs of decoys fit the
    target better than pairs of the D features, although the D features
    together fit it almost exactly.  Columns standardised; one task."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((S, n))
    planted = sorted(int(i) for i in rng.choice(S, size=D, replace=False))
    y = X[planted].sum(axis=0) + sigma * rng.standard_normal(n)
    ys = (y - y.mean()) / y.std()
    rest = np.array([j for j in range(S) if j not in planted])
    decoys = rng.choice(rest, size=int(S * frac_decoy), replace=False)
    eta = math.sqrt(1.0 / (r_decoy * r_decoy) - 1.0)
    for j in decoys:
        X[j] = ys + eta * rng.standard_normal(n)
    X = (X - X.mean(axis=1, keepdims=True)) / X.std(axis=1, keepdims=True)
    meta = dict(name="decoy", seed=seed, n=n, S=S, D=D, k=k, sigma=sigma, planted=planted, r_decoy=r_decoy,
                frac_decoy=frac_decoy, decoys=sorted(int(j) for j in decoys), T=1)
    return Problem(F=np.ascontiguousarray(X), y=y, task_offsets=np.array([0, n], dtype=np.int64),
                   planted=planted, D=D, k=k, exprs=[f"d{j}" for j in range(S)], meta=meta)


def make_batch_problem(i: int, seed0: int = 4100, D: int = 3, k: int = 100,
                       S_range=(200, 2000), n_range=(100, 5000), sigma: float = 0.05) -> Problem:
    """Problem i of the batch of independent single-task searches (seed seed0 + i)."""
    rng = np.random.Generator(np.random.PCG64(seed0 + i))
    S = int(rng.integers(S_range[0], S_range[1] + 1))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    return make_problem(n=n, S=S, D=D, k=k, seed=seed0 + i, beta=(1.5, -0.8, 0.6),
                        sigma=sigma, name=f"batch_{i}")


def make_batch_problems(count: int = 64, seed0: int = 4100, D: int = 3, k: int = 100,
                        S_range=(200, 2000), n_range=(100, 5000), sigma: float = 0.05):
    """Independent single-task searches of different S and n (one seed each)."""
    return [make_batch_problem(i, seed0, D, k, S_range, n_range, sigma) for i in range(count)]


def tiny_problem(seed: int, S: int, n: int, T: int = 1, D: int = 2, k: int = 5,
                 planted: Optional[Sequence[int]] = None, sigma: float = 0.1,
                 task_sizes: Optional[Sequence[int]] = None) -> Problem:
    """Small Gaussian problem for sweeps (no operator trees, just columns)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if task_sizes is None:
        base = n // T
        task_sizes = [base + (1 if t < n - base * T else 0) for t in range(T)]
    offs = np.zeros(T + 1, dtype=np.int64)
    offs[1:] = np.cumsum(task_sizes)
    n = int(offs[-1])
    F = np.ascontiguousarray(rng.standard_normal((S, n)))
    if planted is None:
        planted = sorted(int(i) for i in rng.choice(S, size=min(D, S), replace=False))
    beta = rng.uniform(0.5, 1.5, size=len(planted)) * rng.choice([-1.0, 1.0], size=len(planted))
    y = F[list(planted)].T @ beta + sigma * rng.standard_normal(n)
    for t in range(T):
        y[offs[t]:offs[t + 1]] += rng.uniform(-1, 1)
    meta = dict(name="tiny", seed=seed, n=n, S=S, D=D, k=k, T=T, planted=list(planted))
    return Problem(F=F, y=y, task_offsets=offs, planted=list(planted), D=D, k=k,
                   exprs=[f"g{i}" for i in range(S)], meta=meta)


def integer_problem(seed: int, S: int, n: int, lo: int = -4, hi: int = 4, T: int = 1) -> Problem:
    """Small-integer data (exactly representable) for exact rational pins."""
    rng = np.random.Generator(np.random.PCG64(seed))
    F = rng.integers(lo, hi + 1, size=(S, n)).astype(np.float64)
    y = rng.integers(3 * lo, 3 * hi + 1, size=n).astype(np.float64)
    base = n // T
    sizes = [base + (1 if t < n - base * T else 0) for t in range(T)]
    offs = np.zeros(T + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    meta = dict(name="integer", seed=seed, n=n, S=S, T=T)
    return Problem(F=np.ascontiguousarray(F), y=y, task_offsets=offs, planted=[], D=2, k=5,
                   exprs=[f"z{i}" for i in range(S)], meta=meta)


def input_digest(p: Problem) -> str:
    """SHA-256 of a problem's generated inputs (F, y, task offsets), so a
    stored result can be tied to the exact bytes it was computed from."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(p.F).tobytes())
    h.update(np.ascontiguousarray(p.y).tobytes())
    h.update(np.ascontiguousarray(p.task_offsets).tobytes())
    return h.hexdigest()
