"""Benchmark of the l0 hot path on one MI355X.

One step = the whole hot path over one resident problem: per-task
statistics and the Gram precompute (sisso_gram), the exhaustive search of
all C(S, D) tuples with top-k selection and exact re-scoring
(sisso_l0_search), and the top-k readout (sisso_l0_topk, which
synchronises).  Inputs are generated once (seeded, synthetic) and live in
HBM before the timed region starts.

Prints one JSON line: tuples/s over whole steps, the roofline figure of the
search kernel (timed live with HIP events recorded on the library's stream)
and the CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "l0 tuples/sec at D=3 (plain FP64 vs chosen form) at oracle-matching top-k"
FP64_PEAK = 78.6e12      # MI355X FP64 vector, FLOP/s
HBM_PEAK = 8.0e12        # bytes/s


# Algorithmic FP64 operations of one tuple-task solve (FMA = 2): the
# incremental root-free Cholesky row of the last index against the prefix,
# the pivot, the projected right-hand side and the division-free filter, as
# counted for the method (D = 1: 4, D = 2: 10, D = 3: 17, D = 4: 26).
ALG_FLOP = {1: 4, 2: 10, 3: 17, 4: 26}


def search_flop_per_tuple(D: int, T: int) -> float:
    """Algorithmic FP64 operations per tuple: ALG_FLOP[D] per task."""
    return float(ALG_FLOP[D] * T)


def issued_flop_per_tuple(D: int, T: int) -> float:
    """FP64 operations the search kernel actually issues per tuple.

    Per task, with the prefix's Cholesky row and the k-dependent part of the
    sub-prefix solve hoisted out of the sweep: u = g - v.w (D-2 FMA),
    d = d' - alpha u^2 (1 MUL + 1 FMA), zeta = zeta' - zs u (1 FMA), and the
    division-free test zeta^2 >= pi d (2 MUL).  FMA counts 2.
    Single task: 2(D-2) + 3 + 2 + 2.
    """
    per_task = 2 * (D - 2) + 3 + 2 + 2
    if T == 1 or D == 3:
        # D = 3 with several tasks sweeps with the one-task test on the task of
        # largest |y_t - mean|^2 (its SSE bounds the sum from below); only the
        # few tuples it passes are scored over every task
        return float(per_task)
    # many tasks: the test becomes p - zeta^2 r with r a Newton-refined
    # reciprocal (1 RCP + 2 FMA + 1 MUL + 1 FMA) and a sum over tasks (1 ADD)
    return float(T * (2 * (D - 2) + 3 + 2 + 1 + 1 + 2 * 2 + 2 + 1))


def performed_flop(D: int, T: int, ntup: int) -> tuple:
    """(FLOP, pruned) of the work one search performs.

    One task, or several tasks at D != 3: every tuple is solved in every task,
    ALG_FLOP[D] * T per tuple.  Several tasks at D = 3: the sweep solves every
    tuple in one task only (its SSE is a lower bound of the sum over tasks, so
    the tuples it rejects are pruned exactly) and only the survivors are solved
    in every task; the work performed is the one-task sweep, ALG_FLOP[3] per
    tuple, and the few survivors' solves are not counted.
    """
    if T > 1 and D == 3:
        return float(ALG_FLOP[3]) * ntup, True
    return search_flop_per_tuple(D, T) * ntup, False


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from its committed
    counter summary (profiles/<kernel>_<workload>_traffic.md), or None when
    there is none or the kernel source changed since the counters were taken
    (the summary records the sha256 of the source file)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            key, val = line[2:].split(":", 1)
            fields[key.strip()] = val.strip().strip("`")
    src = os.path.join(ROOT, fields.get("source", ""))
    if not os.path.isfile(src) or "source sha256" not in fields or "bytes per launch" not in fields:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields["source sha256"]:
        return None
    return float(fields["bytes per launch"])


# MFMA products per Gram K-step: FP64 one, the BF16 form's three slices six
# (s + u <= 2), the FP16 form's two slices three
GRAM_PRODUCTS = {"fp64": 1, "bf16": 6, "fp16": 3, "fp32": 1}
MFMA_PEAK = {"fp64": 78.6e12, "bf16": 2.5e15, "fp16": 2.5e15, "fp32": 78.6e12}


def gram_roofline(p, name: str, prec: int, gram_ms: float) -> dict:
    """Roofline of the Gram phase: algorithmic FLOP n (S (S + 1) + 2 S) (the
    correlation matrix and F^T y, every task's rows once) times the MFMA
    products the form issues, over the phase time (the Gram launch and its
    finishing pass), against the MFMA peak of the type it runs in."""
    from paper_2502_20072_amd import _binding as B
    form = {B.SISSO_PREC_FP64: "fp64", B.SISSO_PREC_BF16_COMP: "bf16", B.SISSO_PREC_FP16_COMP: "fp16",
            B.SISSO_PREC_FP32_SOLVE: "fp32"}[prec]
    alg = float(p.n) * (p.S * (p.S + 1) + 2 * p.S)
    kern = "gram_lp_kernel" if form in ("bf16", "fp16") else "gram_kernel"
    achieved = alg * GRAM_PRODUCTS[form] / (gram_ms * 1e-3)
    return dict(bound="mfma", kernel=kern, achieved=achieved / 1e12, peak=MFMA_PEAK[form] / 1e12, unit="TFLOP/s",
                frac=achieved / MFMA_PEAK[form], traffic=measured_traffic(kern, name), algorithmic_flop=alg,
                mfma_products=GRAM_PRODUCTS[form], gram_ms=gram_ms,
                note="phase time: the Gram launch and its finishing pass (the partial sums summed, "
                     "scaled and tiled)")


def cpu_baseline(p, D: int, k: int, target_s: float = 15.0):
    """The oracle on a bounded sample: all tuples whose first index is < a.

    a is chosen from a short probe so the run takes about target_s seconds.
    """
    import oracle

    t0 = time.perf_counter()
    _, _, cnt = oracle.topk(p.F, p.y, D, k, p.task_offsets, i1_range=(p.S // 2, p.S // 2 + 1))
    probe_s = time.perf_counter() - t0
    rate0 = cnt / max(probe_s, 1e-9)
    # tuples with first index < a: C(S, D) - C(S - a, D)
    total = math.comb(p.S, D)
    a = 1
    while a < p.S and (total - math.comb(p.S - a, D)) / rate0 < target_s:
        a += 1
    t0 = time.perf_counter()
    _, _, cnt = oracle.topk(p.F, p.y, D, k, p.task_offsets, i1_range=(0, a))
    dt = time.perf_counter() - t0
    return dict(value=cnt / dt, unit="tuples/s", cores=oracle.threads(), kind="oracle",
                sample=f"{cnt} tuples with first index in [0, {a}) of the {p.meta['name']} "
                       f"workload, {dt:.1f} s, per-tuple Householder QR")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_s1000_d3")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--precision", choices=("fp64", "bf16", "fp16", "fp32"), default="fp64",
                    help="precision form: bf16/fp16 slice the Gram (FP64 search), fp32 runs the "
                         "per-tuple solves in FP32 (FP64 Gram); the re-score is FP64 in every form")
    ap.add_argument("--tune-cache", default=os.environ.get("SISSO_AUTOTUNE_CACHE"),
                    help="JSON cache of the search-grid autotuner (default: tune every run)")
    ap.add_argument("--form", choices=("exhaustive", "learned", "screen"), default="exhaustive",
                    help="learned: train the proposal network (untimed), then time proposal + exact "
                         "evaluation against exhaustive search on the same GPU; screen: one screening "
                         "pass over a created rung (--workload sis_s1000_n2000 or sis_t2_s1000_n156)")
    ap.add_argument("--budget", type=float, default=0.01, help="learned form: fraction of C(S, D) evaluated")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the timed region, copy a buffer of this many MiB three times with torch "
                         "(a plain copy kernel of known size, to calibrate HBM byte counters)")
    ap.add_argument("--chosen-form", default="multitask_t16_s1500_d3",
                    help="workload of the chosen (several-task) form reported beside the plain line; '' for none")
    ap.add_argument("--search-grid", type=int, default=0,
                    help="fix the search grid (workgroups) instead of autotuning it, e.g. for counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the search shards by "
                                   "lexicographic rank range across GPUs, but no "
                                   "multi-GPU path is built", "n_gpus": args.gpus}))
        return 2

    import torch

    from synth import make_config
    import __graft_entry__ as ge

    ge._ensure_built()
    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    from paper_2502_20072_amd import _binding as B

    if args.workload == "batch64_d3":
        return bench_batch(args)
    if args.form == "screen":
        return bench_screen(args)
    p = make_config(args.workload)
    if args.form == "learned":
        return bench_learned(args, p)
    prec = {"fp64": B.SISSO_PREC_FP64, "bf16": B.SISSO_PREC_BF16_COMP, "fp16": B.SISSO_PREC_FP16_COMP,
            "fp32": B.SISSO_PREC_FP32_SOLVE}[args.precision]
    res = bench_exhaustive(args, p, args.workload, prec, args.steps, args.warmup, args.search_grid)
    res = {"metric": METRIC, **res}
    if args.chosen_form and args.workload != args.chosen_form:
        # the chosen form (several tasks of uneven size, D = 3) beside the
        # plain FP64 line; its own top-k is checked on a stored oracle range
        q = make_config(args.chosen_form)
        cf = bench_exhaustive(args, q, args.chosen_form, B.SISSO_PREC_FP64, max(1, args.steps // 2),
                              max(1, args.warmup), 0)
        res["chosen_form"] = cf
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(p, p.D, p.k, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    return 0


def golden_check(p, name: str, idx, sse, i1_range=None):
    """Compare a top-k with the stored oracle result of the same workload.

    Returns (matches, note).  matches is None when there is no stored result
    or the regenerated inputs differ from the ones it was computed on
    (sha256 of F, y and the task offsets).  Otherwise True iff the index
    lists are identical and every SSE is within a relative 1e-10."""
    import numpy as np
    from synth import input_digest

    tag = f"_i1_{i1_range[0]}_{i1_range[1]}" if i1_range else ""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_topk_{name}{tag}.json")
    if not os.path.exists(path):
        return None, f"no stored oracle result {os.path.basename(path)}"
    g = json.load(open(path))
    if g.get("input_sha256") != input_digest(p):
        return None, "regenerated inputs differ from the stored result's (sha256)"
    gi = [tuple(int(v) for v in t) for t in idx]
    oi = [tuple(int(v) for v in t) for t in g["idx"]]
    gs, osse = np.asarray(sse, dtype=np.float64), np.array(g["sse"])
    # position by position the SSEs agree (both lists are sorted by SSE);
    # the tuple sets agree except for tuples tied with the k-th SSE within
    # tau = 1e-9 s_k, which either list may hold
    rel = float(np.max(np.abs(gs - osse) / osse))
    sk = float(osse[-1])
    tau = 1e-9 * sk
    gset, oset = set(gi), set(oi)
    g_sse = dict(zip(gi, gs))
    o_sse = dict(zip(oi, osse))
    stray = [t for t in gset - oset if abs(g_sse[t] - sk) > tau] + [t for t in oset - gset if abs(o_sse[t] - sk) > tau]
    ok = bool(not stray and rel <= 1e-10 and len(gi) == len(oi))
    order = "same order" if gi == oi else "same set up to near-ties" if gset == oset else "sets differ"
    return ok, (f"{os.path.basename(path)}: {order}, {len(stray)} tuples outside the k-th tie band differ, "
                f"max rel SSE diff by position {rel:.2e}")


def bench_exhaustive(args, p, name: str, prec: int, steps: int, warmup: int, search_grid: int) -> dict:
    """Time whole steps (gram + search + topk) of one workload; returns the
    fields of a bench line (without the metric)."""
    import numpy as np
    import torch

    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd import _binding as B

    D, k = p.D, p.k
    ntup = math.comb(p.S, D)
    print(f"bench: workload={name} n={p.n} S={p.S} T={p.T} D={D} k={k} tuples={ntup}",
          file=sys.stderr, flush=True)
    s = L0Search(p.F, p.y, p.task_offsets, D_max=D, k_max=k, device="cuda:0", precision=prec)
    # launch tuning on the problem itself (changes no arithmetic), before timing
    s.gram()
    if search_grid > 0:
        s.set_search_grid(search_grid)
        grid = search_grid
    else:
        grid = s.autotune(D, k, args.tune_cache)

    def step():
        s.gram()
        s.search(D, k)
        return s.topk(k)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    out = None
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / steps * 1e3
    # correctness of the last timed step's output against the stored oracle
    # result: over every tuple where one exists, else over the tuples whose
    # first index is below a (that rank range searched again and compared)
    if p.T == 1 and os.path.exists(os.path.join(ROOT, "tests", "golden", f"oracle_topk_{name}.json")):
        matches, note = golden_check(p, name, out[0], out[1])
    else:
        a = 2
        for cand in (100, 2, 1):
            if os.path.exists(os.path.join(ROOT, "tests", "golden", f"oracle_topk_{name}_i1_0_{cand}.json")):
                a = cand
                break
        r1 = ntup - math.comb(p.S - a, D)
        s.search_range(D, k, 0, r1)
        ri, rs, _ = s.topk(k)
        matches, note = golden_check(p, name, ri, rs, (0, a))
        note += f" (rank range [0, {r1}) = first index in [0, {a}))"

    # per-phase times with HIP events on the library's stream (separate pass,
    # same launches), averaged over the same number of steps
    B.sisso_l0_profile(s.handle, True)
    acc = {ph: 0.0 for ph in B.PHASES}
    for _ in range(steps):
        s.gram()
        s.search(D, k)
        ms = B.sisso_l0_phase_ms(s.handle)
        for ph in acc:
            acc[ph] += ms[ph] / steps
    B.sisso_l0_profile(s.handle, False)
    search_s = acc["search"] * 1e-3
    f32 = prec == B.SISSO_PREC_FP32_SOLVE
    # the FP32 form runs the general kernel for every D and (with a plain
    # sweep, no filter task) solves every tuple in every task
    flop, pruned = (ALG_FLOP[D] * p.T * ntup, False) if f32 else performed_flop(D, p.T, ntup)
    achieved = flop / search_s
    kname = "search_kernel" if f32 else {3: "search3_kernel",
                                         4: "search4_kernel" if p.T == 1 else "search_kernel"}.get(D, "search_kernel")
    roofline = dict(bound="alu", kernel=kname, achieved=achieved / 1e12, peak=FP64_PEAK / 1e12,
                    unit="TFLOP/s", frac=achieved / FP64_PEAK, traffic=measured_traffic(kname, name),
                    flop_per_tuple=flop / ntup, issued_flop_per_tuple=issued_flop_per_tuple(D, p.T),
                    search_ms=acc["search"], search_tuples_per_s=ntup / search_s)
    if f32:
        roofline["note"] = ("FP32 solves without packed FP32 instructions (the build disables them): "
                            "the vector FP32 rate equals the FP64 one, 256 CU x 64 lanes x 2 x 2.4 GHz")
    if pruned:
        roofline["pruned"] = ("several tasks at D=3: the sweep solves every tuple in the task of largest "
                              "|y_t - mean|^2 only (an exact lower bound of the sum); the survivors' "
                              "all-task solves are not counted")
    search_roofline = None
    if acc["gram"] > acc["search"]:
        # the Gram dominates the step: its roofline is the line's, the
        # search's is kept beside it
        search_roofline, roofline = roofline, gram_roofline(p, name, prec, acc["gram"])
    res = {
        "value": ntup * steps / dt,
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (solves; f64 Gram and re-score)" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": name, "n": p.n, "S": p.S, "T": p.T, "D": D, "k": k,
                   "tuples": ntup, "form": {B.SISSO_PREC_FP64: "plain FP64",
                                            B.SISSO_PREC_BF16_COMP: "precision form (Gram from three BF16 slices, "
                                                                    "FP64 search and re-score)",
                                            B.SISSO_PREC_FP16_COMP: "precision form (Gram from two FP16 slices, "
                                                                    "FP64 search and re-score)",
                                            B.SISSO_PREC_FP32_SOLVE: "FP32 per-tuple solves (FP64 Gram, "
                                                                     "FP64 re-score)"}[prec],
                   "search_grid": grid},
        "topk_matches_oracle": matches,
        "oracle_check": note,
        "phase_ms": acc,
        "roofline": roofline,
    }
    if search_roofline is not None:
        res["search_roofline"] = search_roofline
    if p.T > 1:
        res["tuple_task_solves_per_s"] = ntup * p.T * steps / dt
    if prec != B.SISSO_PREC_FP64:
        res["precision_report"] = s.precision_report(4096)
    s.close()
    return res


def bench_batch(args) -> int:
    """64 independent single-task searches (S ~ U[200, 2000], n ~ U[100, 5000],
    D = 3, k = 100; seeds 4100 + i) captured once as one HIP graph and
    launched as a whole (gram + search of every problem, up to 16 concurrent
    branches).  value = sum of C(S_i, 3) per second of graph launches."""
    import torch

    from synth import make_batch_problems
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd import _binding as B

    probs = make_batch_problems(64)
    D, k = 3, 100
    stream = torch.cuda.Stream()
    hs = [L0Search(p.F, p.y, p.task_offsets, D_max=D, k_max=k, stream=stream) for p in probs]
    b = B.sisso_l0_batch_create([s.handle for s in hs], D, k)
    for _ in range(args.warmup):
        B.sisso_l0_batch_launch(b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(1, args.steps // 4)
    e0.record(stream)
    for _ in range(steps):
        B.sisso_l0_batch_launch(b)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ntup = sum(math.comb(p.S, D) for p in probs)
    for s_ in hs:
        s_.last_D, s_.last_k = D, k
    planted_first = sum(tuple(int(v) for v in s_.topk(with_coef=False)[0][0]) == tuple(sorted(p.planted))
                        for s_, p in zip(hs, probs))
    B.sisso_l0_batch_destroy(b)
    for s_ in hs:
        s_.close()
    res = {"metric": METRIC, "value": ntup / (ms * 1e-3), "unit": "tuples/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batch64_d3", "problems": len(probs), "tuples": ntup, "D": D, "k": k,
                      "form": "batched: one HIP graph, gram + search per problem"},
           "planted_tuple_first": f"{planted_first}/{len(probs)}"}
    print(json.dumps(res), flush=True)
    return 0


def bench_learned(args, p) -> int:
    """Learned proposal vs exhaustive search at the workload's D (one GPU).

    Training (not timed): 150 seeded problems with S=200 (every pair, labelled
    by its best extension: exhaustive D=3 grouped by pair) and 50 with S=60
    (every triple, exhaustive D=4), n=500, generated like the workload.
    Timed: the exhaustive search of all C(S, D) tuples, and the proposal
    (features of every (D-1)-prefix, BF16 network inference, top selection,
    exact search of the kept prefixes' extensions), each after the Gram.
    recall@k: |proposal top-k n exhaustive top-k| / k.
    """
    import numpy as np
    import torch

    from synth import make_problem
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd.learned import (ProposalNet, training_set, propose_and_search, propose_two_stage,
                                              r2_scorer, recall)

    D, k = p.D, p.k
    beta = (1.5, -0.8, 0.6)
    t0 = time.perf_counter()
    tr2 = [make_problem(n=500, S=200, D=3, k=10, seed=5000 + i, beta=beta, sigma=0.05) for i in range(150)]
    tr3 = [make_problem(n=500, S=60, D=4, k=10, seed=5150 + i, beta=beta + (-0.4,), sigma=0.05) for i in range(50)]
    X2, Y2 = training_set(tr2, 2)
    X3, Y3 = training_set(tr3, 3)
    X, Y = torch.cat([X2, X3]), torch.cat([Y2, Y3])
    net = ProposalNet(seed=0)
    hist = net.fit(X, Y, epochs=6, batch=8192, lr=2e-3)
    train_s = time.perf_counter() - t0
    print(f"bench: trained on {X.shape[0]} prefixes in {train_s:.1f} s, loss {hist[0]:.4f} -> {hist[-1]:.4f}",
          file=sys.stderr, flush=True)

    s = L0Search(p.F, p.y, p.task_offsets, D_max=D, k_max=k, device="cuda:0")
    s.gram()
    s.autotune(D, k, args.tune_cache)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    t_exh = timed(lambda: s.search(D, k), max(1, args.steps // 4))
    ei, es, _ = s.topk()
    info = {}

    def prop():
        info.update(propose_and_search(s, D, k, net.predict, budget_frac=args.budget))
    t_prop = timed(prop, max(1, args.steps // 4))
    li, ls, _ = s.topk()
    rec = recall(li, ei)
    propose_and_search(s, D, k, r2_scorer, budget_frac=args.budget)
    rec_r2 = recall(s.topk()[0], ei)
    # sub-enumeration: (D-2)-prefixes first, then the extensions of the best
    info2 = {}

    def prop2():
        info2.update(propose_two_stage(s, D, k, net.predict, budget_frac=args.budget))
    t_two = timed(prop2, max(1, args.steps // 4))
    rec_two = recall(s.topk()[0], ei)
    propose_two_stage(s, D, k, r2_scorer, budget_frac=args.budget)
    rec_two_r2 = recall(s.topk()[0], ei)
    s.close()
    decoy = decoy_comparison(args.budget) if D == 4 else None
    ntup = math.comb(p.S, D)
    res = {
        "metric": f"l0 tuples/sec at D={D} (learned proposal, exact FP64 evaluation; recall@{k} vs exhaustive)",
        "value": ntup / (t_prop * 1e-3), "unit": "tuples/s (covered)", "n_gpus": 1, "steps": max(1, args.steps // 4),
        "warmup": 1, "ms_per_step": t_prop, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (network: fp32 train, bf16 infer)", "data": "synthetic",
        "config": {"workload": args.workload, "n": p.n, "S": p.S, "D": D, "k": k, "budget": args.budget,
                   "form": "learned proposal", **info},
        f"recall_at_{k}": rec, f"recall_at_{k}_r2_only": rec_r2,
        "exhaustive_ms": t_exh, "proposal_ms": t_prop, "speedup_vs_exhaustive": t_exh / t_prop,
        "two_stage": {"ms": t_two, "speedup_vs_exhaustive": t_exh / t_two, f"recall_at_{k}": rec_two,
                      f"recall_at_{k}_r2_only": rec_two_r2, **info2},
        "train": {"prefixes": int(X.shape[0]), "seconds": train_s, "loss_first_epoch": hist[0],
                  "loss_last_epoch": hist[-1]},
    }
    if decoy is not None:
        res["decoy_subspaces"] = decoy
    print(json.dumps(res), flush=True)
    return 0


def screen_flop_per_sample(nres: int) -> int:
    """Algorithmic FP64 operations per sample of one created feature in a
    screening pass (FMA = 2): the operator 1, the task sum 1, the centring 1,
    the centred and the raw sums of squares 2 + 2, one product sum per
    residual 2 nres."""
    return 7 + 2 * nres


def screen_cpu_baseline(w, target_s: float):
    """The oracle (one process) creating and scoring the first candidates of
    the workload's first operator, as many as fit in about target_s."""
    import numpy as np
    from oracle import sisso_ref as R

    res = list(w.R)
    done, t0 = 0, time.perf_counter()
    while done < w.P and time.perf_counter() - t0 < target_s:
        q = min(done + 256, w.P)
        vals, ok = R.create(w.ops[0], w.X, w.pairs[done:q], w.lower, w.upper)
        for v, good in zip(vals, ok):
            if good:
                R.sis_score(v, res, w.task_offsets)
        done = q
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="candidates/s", cores=1, kind="oracle",
                sample=f"the first {done} '{w.ops[0]}' candidates of {w.meta['name']}, created, checked and "
                       f"scored against {len(res)} residuals in {dt:.1f} s (numpy, one process)")


def screen_golden_check(w, idx, score):
    """Compare a top-m with the stored oracle result of the workload: the
    same candidates except those tied with the m-th score within 1e-12,
    scores to 1e-12 position by position."""
    import numpy as np
    from synth import screen_digest

    path = os.path.join(ROOT, "tests", "golden", f"oracle_sis_{w.meta['name']}.json")
    if not os.path.exists(path):
        return None, f"no stored oracle result {os.path.basename(path)}"
    g = json.load(open(path))
    if g.get("input_sha256") != screen_digest(w):
        return None, "regenerated inputs differ from the stored result's (sha256)"
    gi, gs = [int(v) for v in idx], np.asarray(score, dtype=np.float64)
    oi, osc = g["idx"], np.array(g["score"])
    if len(gi) != len(oi):
        return False, f"{len(gi)} selected against the oracle's {len(oi)}"
    diff = float(np.max(np.abs(gs - osc))) if len(gi) else 0.0
    sm = float(osc[-1]) if len(oi) else 0.0
    gsc, osd = dict(zip(gi, gs)), dict(zip(oi, osc))
    stray = [c for c in set(gi) - set(oi) if abs(gsc[c] - sm) > 1e-12] + \
            [c for c in set(oi) - set(gi) if abs(osd[c] - sm) > 1e-12]
    ok = bool(not stray and diff <= 1e-12)
    order = "same order" if gi == oi else "same set up to near-ties" if set(gi) == set(oi) else "sets differ"
    return ok, f"{os.path.basename(path)}: {order}, {len(stray)} outside the m-th tie band, max score diff {diff:.1e}"


def bench_screen(args) -> int:
    """One screening pass over a created rung (one GPU).

    Step (the paper's form, features never stored): for each binary operator,
    sisso_sis_score_op creates every child-pair candidate sample by sample,
    applies the value rules and scores it against the residuals; then
    sisso_topm selects the m best of all candidates (and synchronises).
    Beside it, the stored form: the valid candidates are first written out
    (sisso_fc_eval, untimed), then sisso_sis_score reads them from HBM and
    sisso_topm selects.  Both forms must select the same candidates; the
    fused form's selection is checked against the stored oracle result.
    Last, one run of the dimension loop (sisso_fit, D = 1..3) over the
    stored candidates is timed after one untimed run.
    """
    import numpy as np
    import torch

    from synth import make_screen_workload
    from paper_2502_20072_amd import _binding as B

    w = make_screen_workload(args.workload)
    dev = "cuda:0"
    X = torch.from_numpy(w.X).to(dev)
    Rr = torch.from_numpy(w.R).to(dev)
    pairs = torch.from_numpy(w.pairs).to(dev)
    h = B.SisScreen(Rr, w.task_offsets)
    P, nops, m = w.P, len(w.ops), w.m
    M = P * nops
    scores = torch.empty(M, dtype=torch.float64, device=dev)
    out_idx = torch.empty(m, dtype=torch.int64, device=dev)
    out_sc = torch.empty(m, dtype=torch.float64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nops + 2)]
    steps, warm = args.steps, args.warmup
    kern_ms = np.zeros(nops)

    def fused(record):
        for o, op in enumerate(w.ops):
            if record:
                ev[2 * o].record()
            h.score_op(op, X, pairs, w.lower, w.upper, scores[o * P:(o + 1) * P])
            if record:
                ev[2 * o + 1].record()
        return B.sisso_topm(scores, m, out_idx, out_sc)

    for _ in range(warm):
        fused(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cnt = fused(True)
        kern_ms += [ev[2 * o].elapsed_time(ev[2 * o + 1]) for o in range(nops)]
    torch.cuda.synchronize()
    fused_ms = (time.perf_counter() - t0) * 1e3 / steps
    kern_ms /= steps
    f_idx, f_sc = out_idx[:cnt].cpu().numpy(), out_sc[:cnt].cpu().numpy()
    n_valid = int(torch.isfinite(scores).sum())
    ok, note = screen_golden_check(w, f_idx, f_sc)

    # the stored form over the same candidates: the valid ones written out
    valid = torch.empty(P, dtype=torch.uint8, device=dev)
    cand = []
    for o, op in enumerate(w.ops):
        B.sisso_fc_eval(op, X, pairs, w.lower, w.upper, None, valid)
        cand.append(torch.nonzero(valid, as_tuple=False).flatten() + o * P)
    cand = torch.cat(cand)
    Mv = int(cand.numel())
    Xs = torch.empty((Mv, w.n), dtype=torch.float64, device=dev)
    vtmp = torch.empty(Mv, dtype=torch.uint8, device=dev)
    at = 0
    for o, op in enumerate(w.ops):
        sel = cand[(cand >= o * P) & (cand < (o + 1) * P)] - o * P
        pv = pairs[sel].contiguous()
        B.sisso_fc_eval(op, X, pv, w.lower, w.upper, Xs[at:at + pv.shape[0]], vtmp[at:at + pv.shape[0]])
        at += pv.shape[0]
    sscores = torch.empty(Mv, dtype=torch.float64, device=dev)
    s_idx = torch.empty(m, dtype=torch.int64, device=dev)
    s_sc = torch.empty(m, dtype=torch.float64, device=dev)

    def stored(record):
        if record:
            ev[-2].record()
        h.score(Xs, sscores)
        if record:
            ev[-1].record()
        return B.sisso_topm(sscores, m, s_idx, s_sc)

    for _ in range(warm):
        stored(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    skern = 0.0
    for _ in range(steps):
        scnt = stored(True)
        skern += ev[-2].elapsed_time(ev[-1])
    torch.cuda.synchronize()
    stored_ms = (time.perf_counter() - t0) * 1e3 / steps
    skern /= steps
    s_sel = cand[s_idx[:scnt]].cpu().numpy()
    same = bool(np.array_equal(s_sel, f_idx) and np.array_equal(s_sc[:scnt].cpu().numpy(), f_sc))
    h.close()

    # the dimension loop over the stored candidates: screening of all of them
    # per dimension, top-m, l0 search of the subspace, residuals
    y = torch.from_numpy(w.y).to(dev)
    fit_args = dict(D_max=3, m_sis=100, n_res=10, k=10)
    B.sisso_fit(Xs, y, w.task_offsets, **fit_args)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit = B.sisso_fit(Xs, y, w.task_offsets, **fit_args)
    fit_ms = (time.perf_counter() - t0) * 1e3
    best = [int(cand[int(c)]) for c in fit["models"][2][0] if c >= 0]
    del Xs

    nres = int(w.R.shape[0])
    flop = screen_flop_per_sample(nres) * w.n
    fused_kern = float(kern_ms.sum())
    achieved = M * flop / (fused_kern * 1e-3)
    sbytes = Mv * (w.n * 8 + 8)
    res = {
        "metric": "SIS candidates screened/sec (created on the fly, scored against residuals, top-m)",
        "value": M / (fused_ms * 1e-3), "unit": "candidates/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": fused_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.meta["name"], "n": w.n, "T": w.meta["T"], "children": w.meta["Mc"],
                   "ops": list(w.ops), "candidates": M, "nres": nres, "m": m},
        "valid_candidates": n_valid, "topm_matches_oracle": ok, "oracle_check": note,
        "kernel_ms": {op: float(t) for op, t in zip(w.ops, kern_ms)},
        "roofline": {"bound": "alu", "kernel": "screen_kernel (created features, 5 launches)",
                     "achieved": achieved / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK,
                     "traffic": measured_traffic("screen_kernel_created", w.meta["name"]),
                     "flop_per_sample": screen_flop_per_sample(nres), "kernel_ms": fused_kern},
        "stored": {"ms_per_step": stored_ms, "candidates_per_s": Mv / (stored_ms * 1e-3), "features": Mv,
                   "same_selection_as_fused": same,
                   "roofline": {"bound": "hbm", "kernel": "screen_kernel (stored features)",
                                "achieved": sbytes / (skern * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                "frac": sbytes / (skern * 1e-3) / HBM_PEAK,
                                "traffic": measured_traffic("screen_kernel_stored", w.meta["name"]),
                                "bytes_per_feature": w.n * 8 + 8, "kernel_ms": skern}},
        "dimension_loop": {"ms": fit_ms, **fit_args, "candidates": Mv,
                           "best_D3_model": best, "best_D3_sse": float(fit["sse"][2][0])},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = screen_cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    return 0


def decoy_comparison(budget: float) -> dict:
    """The network against the R^2 feature alone where they differ: eight
    decoy subspaces (make_decoy_problem, n = 2000, S = 600, D = 4, k = 100,
    seeds 7500-7507; the network trained on 60 + 20 smaller decoy problems),
    two-stage proposal at the same budget, recall@100 against exhaustive."""
    import numpy as np
    import torch

    from synth import make_decoy_problem
    from paper_2502_20072_amd import L0Search
    from paper_2502_20072_amd.learned import ProposalNet, training_set, propose_two_stage, r2_scorer, recall

    X2, Y2 = training_set([make_decoy_problem(500, 200, 7000 + i) for i in range(60)], 2)
    X3, Y3 = training_set([make_decoy_problem(500, 60, 7100 + i) for i in range(20)], 3)
    net = ProposalNet(seed=0)
    net.fit(torch.cat([X2, X3]), torch.cat([Y2, Y3]), epochs=6, batch=8192, lr=2e-3)
    rec = {"net": [], "r2": []}
    for seed in range(7500, 7508):
        p = make_decoy_problem(2000, 600, seed)
        s = L0Search(p.F, p.y, p.task_offsets, D_max=4, k_max=100, device="cuda:0")
        s.gram().search(4, 100)
        ei, _, _ = s.topk()
        for name, sc in (("net", net.predict), ("r2", r2_scorer)):
            propose_two_stage(s, 4, 100, sc, budget_frac=budget)
            rec[name].append(recall(s.topk()[0], ei))
        s.close()
    return {"instances": 8, "budget": budget, "two_stage": True,
            "recall_at_100_net": {"mean": float(np.mean(rec["net"])), "min": float(np.min(rec["net"]))},
            "recall_at_100_r2_only": {"mean": float(np.mean(rec["r2"])), "min": float(np.min(rec["r2"]))},
            "per_instance": rec}


if __name__ == "__main__":
    sys.exit(main())
