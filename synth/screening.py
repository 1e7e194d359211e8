"""Seeded inputs of one screening pass over a rung of created features.

The paper's last rung is never stored: each screening pass re-creates its
features from their children, operator by operator, and scores them against
the target or the residuals of the previous dimension's best models
(section "Feature generation and SIS").  A workload here is

* children: the features of an l0 workload (rung <= 2 trees, standardised),
  shape (Mc, n), one child per row;
* candidates: every unordered child pair (i < j, lexicographic) under each
  binary operator of ``ops``; candidate c = o * P + p is operator o on pair p;
* residuals: nres vectors over the samples.  Row 0 is the target; rows
  1..nres-1 are stand-ins for the residuals of the previous dimension's best
  models: the target plus seeded N(0, 0.3^2) noise.  The cost of a pass does
  not depend on their values;
* the value rules' bounds and the subspace size m.

This module only draws inputs; it holds none of the screening arithmetic.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Tuple

import numpy as np

from .problems import make_config, make_problem

SCREEN_OPS = ("add", "sub", "mul", "div", "abs_diff")

SCREEN_CONFIGS: Dict[str, Dict] = {
    # the 1000 features of the plain D = 3 workload (n = 2000, one task),
    # ten residuals, a 1000-feature subspace
    "sis_s1000_n2000": dict(children=("config", "plain_s1000_d3"), nres=10, m=1000, seed=606),
    # the thermal-conductivity case's shape: two tasks of 78 samples
    "sis_t2_s1000_n156": dict(children=("problem", dict(n=None, S=1000, D=3, k=100, seed=707,
                                                        beta=(1.5, -0.8, 0.6), sigma=0.05,
                                                        tasks=dict(T=2, lo=78, hi=79))),
                              nres=10, m=1000, seed=708),
}


@dataclasses.dataclass
class ScreenWorkload:
    X: np.ndarray             # (Mc, n) children, C-contiguous
    y: np.ndarray             # (n,) target
    R: np.ndarray             # (nres, n) residuals (row 0 = y)
    task_offsets: np.ndarray  # (T+1,) int64
    pairs: np.ndarray         # (P, 2) int32, every i < j in lexicographic order
    ops: Tuple[str, ...]
    m: int
    lower: float
    upper: float
    meta: Dict

    @property
    def n(self) -> int:
        return int(self.X.shape[1])

    @property
    def P(self) -> int:
        return int(self.pairs.shape[0])

    @property
    def candidates(self) -> int:
        return self.P * len(self.ops)


def all_pairs(Mc: int) -> np.ndarray:
    """Every (i, j) with 0 <= i < j < Mc, lexicographic, as int32 (P, 2)."""
    i, j = np.triu_indices(Mc, k=1)
    return np.ascontiguousarray(np.stack([i, j], axis=1).astype(np.int32))


def make_screen_workload(name: str) -> ScreenWorkload:
    cfg = SCREEN_CONFIGS[name]
    kind, spec = cfg["children"]
    p = make_config(spec) if kind == "config" else make_problem(name=f"{name}.children", **spec)
    rng = np.random.Generator(np.random.PCG64(cfg["seed"]))
    nres = cfg["nres"]
    R = np.empty((nres, p.n), dtype=np.float64)
    R[0] = p.y
    for q in range(1, nres):
        R[q] = p.y + 0.3 * rng.standard_normal(p.n)
    meta = dict(name=name, children=p.meta["name"], children_seed=p.meta["seed"], residual_seed=cfg["seed"],
                nres=nres, m=cfg["m"], Mc=p.S, n=p.n, T=p.T)
    return ScreenWorkload(X=p.F, y=p.y, R=R, task_offsets=p.task_offsets, pairs=all_pairs(p.S), ops=SCREEN_OPS,
                          m=cfg["m"], lower=1e-5, upper=1e8, meta=meta)


def screen_digest(w: ScreenWorkload) -> str:
    """SHA-256 of a workload's drawn inputs (children, residuals, offsets)."""
    import hashlib
    h = hashlib.sha256()
    for a in (w.X, w.R, w.task_offsets):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
