"""Write the stored oracle results used by the GPU parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generator
(``synth/``).  Usage:  python tests/golden/make_golden.py NAME [NAME ...]

NAME is a workload of ``synth.CONFIGS`` or ``batch64_d3.<i>`` (problem i of
the 64-problem batch); ``NAME:lo:hi`` restricts the first tuple index to
[lo, hi), i.e. the lexicographic rank range [0, C(S,D) - C(S-hi,D)) when
lo = 0.

Each output file ``oracle_topk_<NAME>.json`` holds the oracle's top-k
(indices, SSE) of the named workload, the number of tuples it scored and a
SHA-256 of the generated inputs, so a test can tell whether the generator
reproduced the same bytes on its machine.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import input_digest, make_batch_problem, make_config  # noqa: E402


def problem(name: str):
    if name.startswith("batch64_d3."):
        return make_batch_problem(int(name.split(".")[1]))
    return make_config(name)


def write(name: str, i1_range=None, tag: str = "") -> str:
    t_gen = time.time()
    p = problem(name)
    t0 = time.time()
    print(f"{name}{tag}: inputs drawn in {t0 - t_gen:.1f}s, oracle running", flush=True)
    idx, sse, cnt = oracle.topk(p.F, p.y, p.D, p.k, p.task_offsets, i1_range=i1_range)
    dt = time.time() - t0
    out = dict(workload=name, seed=p.meta["seed"], D=p.D, k=p.k, S=p.S, n=p.n, T=p.T,
               i1_range=list(i1_range) if i1_range else None, n_scored=cnt,
               input_sha256=input_digest(p), planted=p.planted,
               idx=idx.tolist(), sse=[float(v) for v in sse], oracle_seconds=round(dt, 1))
    path = os.path.join(HERE, f"oracle_topk_{name}{tag}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(f"{name}{tag}: {cnt} tuples in {dt:.1f}s -> {path}", flush=True)
    return path


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        if ":" in arg:       # NAME:lo:hi  restricts the first index to [lo, hi)
            name, lo, hi = arg.split(":")
            write(name, (int(lo), int(hi)), tag=f"_i1_{lo}_{hi}")
        else:
            write(arg)
