"""Write the stored oracle result of a screening workload.

Calls only the CPU oracle (``oracle/sisso_ref.py``: feature creation with the
value rules, the SIS score of eq. (1), top-m) and the seeded input generator
(``synth/``).  Usage:  python tests/golden/make_golden_sis.py NAME [NAME ...]

Every candidate of the workload (operator o on child pair p, candidate index
o * P + p) is created, checked by the value rules and scored against the
workload's residuals; candidates that fail a rule have no score.  The output
``oracle_sis_<NAME>.json`` holds the m best (index, score) by (score
descending, index ascending), the number of candidates that passed the rules
and a SHA-256 of the drawn inputs.  The work is split over a process pool.
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sisso_ref as R  # noqa: E402
from synth import make_screen_workload, screen_digest  # noqa: E402

CHUNK = 4096
_W = None


def _init(name):
    global _W
    _W = make_screen_workload(name)


def _score_chunk(args):
    o, p0, p1 = args
    w = _W
    vals, ok = R.create(w.ops[o], w.X, w.pairs[p0:p1], w.lower, w.upper)
    res = list(w.R)
    sc = np.full(p1 - p0, np.nan)
    for q in range(p1 - p0):
        if ok[q]:
            sc[q] = R.sis_score(vals[q], res, w.task_offsets)
    return o, p0, sc


def write(name: str, workers: int) -> str:
    w = make_screen_workload(name)
    jobs = [(o, p0, min(p0 + CHUNK, w.P)) for o in range(len(w.ops)) for p0 in range(0, w.P, CHUNK)]
    scores = np.full(w.candidates, np.nan)
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers, initializer=_init, initargs=(name,)) as pool:
        for done, (o, p0, sc) in enumerate(pool.imap_unordered(_score_chunk, jobs), 1):
            scores[o * w.P + p0:o * w.P + p0 + len(sc)] = sc
            if done % 100 == 0:
                print(f"{name}: {done}/{len(jobs)} chunks, {time.time() - t0:.0f}s", flush=True)
    top = R.top_m(scores, w.m)
    out = dict(workload=name, meta=w.meta, ops=list(w.ops), P=w.P, candidates=w.candidates, m=w.m,
               lower=w.lower, upper=w.upper, n_valid=int(np.isfinite(scores).sum()),
               input_sha256=screen_digest(w), idx=[int(i) for i in top], score=[float(scores[i]) for i in top],
               oracle_seconds=round(time.time() - t0, 1))
    path = os.path.join(HERE, f"oracle_sis_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}: {w.candidates} candidates, {out['n_valid']} valid, {out['oracle_seconds']}s -> {path}",
          flush=True)
    return path


if __name__ == "__main__":
    nw = min(8, os.cpu_count() or 1)
    for arg in sys.argv[1:]:
        write(arg, nw)
