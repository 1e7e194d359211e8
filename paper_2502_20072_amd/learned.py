"""Learned proposal for l0 searches at larger D.

A small network (include/sisso_mlp.h) scores every (D-1)-prefix of the
features from dimension-agnostic statistics of the prefix (its own fit,
the correlations of its features with y and with each other:
sisso_l0_prefix_features).  The prefixes with the best scores are extended
by every feature and those tuples are evaluated exactly
(sisso_l0_search_list), so a D-search touches a chosen fraction of the
C(S, D) tuples.  The two-stage form scores the (D-2)-prefixes first and
only the extensions of the best of them (sub-enumeration), so the network
runs on C(S, D-2) + a few thousand prefixes instead of C(S, D-1).  Exhaustive search stays the reference: recall@k is measured
against it.

Training data come from exhaustive evaluation at a smaller dimension: for
every m-subset P of a training problem, sisso_l0_prefix_best gives the best
SSE over all its extensions P + {j} (an exhaustive (m+1)-search grouped by
prefix); the network learns to predict -log10(best SSE / total SS) from the
prefix's features.  Training runs on the GPU with the library's FP32
forward/backward kernels and Adam; proposals use the BF16 MFMA inference
kernel.  This module only marshals tensors between those entry points.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _binding as B


def _stream(t) -> int:
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def all_prefixes(S: int, m: int, device="cuda:0"):
    """Every m-subset of {0..S-1} as int32 rows, in colexicographic order."""
    import torch
    n = math.comb(S, m)
    ranks = torch.arange(n, dtype=torch.int64, device=device)
    pre = torch.empty((n, m), dtype=torch.int32, device=device)
    B.sisso_colex_unrank(m, ranks, pre, _stream(ranks))
    return pre


def training_set(problems: Sequence, m: int, device="cuda:0"):
    """Features and targets of every m-subset of every problem (GPU).

    The target of a prefix is -log10(best extension SSE / total sum of
    squares), computed on the device by sisso_l0_prefix_target."""
    import torch
    from . import L0Search
    xs, ys = [], []
    for p in problems:
        s = L0Search(p.F, p.y, p.task_offsets, D_max=min(m + 1, 4), k_max=1, device=device)
        s.gram()
        pre = all_prefixes(p.S, m, device)
        feat = torch.empty((pre.shape[0], B.PROP_NF), dtype=torch.float32, device=device)
        best = torch.empty(pre.shape[0], dtype=torch.float64, device=device)
        target = torch.empty(pre.shape[0], dtype=torch.float32, device=device)
        B.sisso_l0_prefix_features(s.handle, m, pre, feat)
        B.sisso_l0_prefix_target(s.handle, m, pre, best, target)
        xs.append(feat)
        ys.append(target)
        torch.cuda.synchronize()
        s.close()
    return torch.cat(xs), torch.cat(ys)


class ProposalNet:
    """Parameters of the network (one FP32 device array) and its training."""

    def __init__(self, seed: int = 0, device="cuda:0"):
        import torch
        rng = np.random.default_rng(seed)
        nin, h = B.MLP_IN, B.MLP_HIDDEN
        parts = [rng.uniform(-1, 1, (nin, h)) * math.sqrt(6.0 / nin), np.zeros(h),
                 rng.uniform(-1, 1, (h, h)) * math.sqrt(6.0 / h), np.zeros(h),
                 rng.uniform(-1, 1, h) * math.sqrt(3.0 / h), np.zeros(1)]
        flat = np.concatenate([q.ravel() for q in parts]).astype(np.float32)
        assert flat.size == B.MLP_NPARAM
        self.device = device
        self.params = torch.from_numpy(flat).to(device)

    def fit(self, X, Y, epochs: int = 20, batch: int = 4096, lr: float = 2e-3, seed: int = 0) -> List[float]:
        """Adam on the mean squared error; returns the mean loss per epoch.

        Each epoch visits every example once in a seeded random order, in
        batches of ``batch`` (clamped to the number of examples); the last
        batch of an epoch holds the remainder."""
        import torch
        n = int(X.shape[0])
        if n < 1:
            raise ValueError("fit needs at least one training example")
        batch = max(1, min(int(batch), n))
        grad = torch.zeros_like(self.params)
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        ws = torch.empty(B.sisso_mlp_workspace_bytes(batch), dtype=torch.uint8, device=self.device)
        out = torch.empty(batch, dtype=torch.float32, device=self.device)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        st = _stream(self.params)
        gen = torch.Generator(device="cpu").manual_seed(seed)
        step, hist = 0, []
        for _ in range(epochs):
            perm = torch.randperm(n, generator=gen).to(self.device)
            tot, cnt = 0.0, 0
            for i, b0 in enumerate(range(0, n, batch)):
                idx = perm[b0:b0 + batch]
                xb, yb = X[idx].contiguous(), Y[idx].contiguous()
                nb = int(idx.shape[0])
                B.sisso_mlp_forward(self.params, xb, out[:nb], ws, st)
                B.sisso_mlp_backward(self.params, xb, yb, grad, loss, ws, st)
                step += 1
                B.sisso_mlp_adam(self.params, grad, m, v, step, lr, st)
                if i % 16 == 0:   # sample the loss without a sync per batch
                    tot += float(loss.item())
                    cnt += 1
            hist.append(tot / max(1, cnt))
        return hist

    def predict(self, X):
        """BF16 MFMA inference."""
        import torch
        out = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        B.sisso_mlp_infer_bf16(self.params, X.contiguous(), out, _stream(X))
        return out

    def forward_f32(self, X):
        import torch
        n = X.shape[0]
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        ws = torch.empty(B.sisso_mlp_workspace_bytes(n), dtype=torch.uint8, device=self.device)
        B.sisso_mlp_forward(self.params, X.contiguous(), out, ws, _stream(X))
        return out


def propose_and_search(search, D: int, k: int, scorer, budget_frac: float = 0.01,
                       chunk: int = 1 << 24) -> Dict:
    """Score every (D-1)-prefix, keep the best ones for a budget of
    budget_frac * C(S, D) tuples, and search their extensions exactly.
    scorer(features) -> scores (device float32).  The handle then holds the
    result (read with search.topk()).  Returns the sizes involved."""
    import torch
    S, m = search.S, D - 1
    npre = math.comb(S, m)
    dev = search.F.device
    scores = torch.empty(npre, dtype=torch.float32, device=dev)
    feat = torch.empty((min(chunk, npre), B.PROP_NF), dtype=torch.float32, device=dev)
    for r0 in range(0, npre, chunk):
        n = min(chunk, npre - r0)
        B.sisso_l0_prefix_features_range(search.handle, m, r0, n, feat[:n])
        scores[r0:r0 + n] = scorer(feat[:n])
    K = max(1, min(npre, math.ceil(budget_frac * math.comb(S, D) / (S - m))))
    cap = min(npre, 2 * K + 4096)
    ranks = torch.empty(cap, dtype=torch.int64, device=dev)
    ws = torch.empty(B.sisso_select_workspace_bytes(), dtype=torch.uint8, device=dev)
    cnt = B.sisso_select_top(scores, K, ranks, ws, _stream(scores))
    pre = torch.empty((cnt, m), dtype=torch.int32, device=dev)
    B.sisso_colex_unrank(m, ranks[:cnt], pre, _stream(ranks))
    B.sisso_l0_search_list(search.handle, D, k, pre)
    search.last_D, search.last_k = D, k
    return dict(prefixes_scored=npre, prefixes_kept=cnt, prefix_budget=K,
                tuples_evaluated=cnt * (S - m), tuples_total=math.comb(S, D))


def propose_two_stage(search, D: int, k: int, scorer, budget_frac: float = 0.01, keep_factor: float = 32.0,
                      min_keep: int = 256, chunk: int = 1 << 24) -> Dict:
    """Sub-enumeration: score every (D-2)-prefix (every pair at D = 4),
    keep the best, score every one-index extension of the kept ones
    (sisso_l0_prefix_extend), keep the best (D-1)-prefixes for a budget of
    budget_frac * C(S, D) tuples and search their extensions exactly.  The
    scorer sees C(S, D-2) + kept (S - D + 2) prefixes instead of
    C(S, D-1).  The first stage keeps enough prefixes for keep_factor times
    the second stage's count, and at least min_keep: the first stage's
    extensions are cheap to score, and too few kept prefixes is what loses
    recall at small budgets.  D >= 3."""
    import torch
    S, m1, m2 = search.S, D - 2, D - 1
    if m1 < 1:
        raise ValueError("the two-stage proposal needs D >= 3")
    dev = search.F.device
    n1 = math.comb(S, m1)
    scores1 = torch.empty(n1, dtype=torch.float32, device=dev)
    st = _stream(scores1)
    feat = torch.empty((min(chunk, n1), B.PROP_NF), dtype=torch.float32, device=dev)
    for r0 in range(0, n1, chunk):
        n = min(chunk, n1 - r0)
        B.sisso_l0_prefix_features_range(search.handle, m1, r0, n, feat[:n])
        scores1[r0:r0 + n] = scorer(feat[:n])
    K2 = max(1, min(math.comb(S, m2), math.ceil(budget_frac * math.comb(S, D) / (S - m2))))
    K1 = max(1, min(n1, max(int(min_keep), math.ceil(keep_factor * K2 / (S - m1)))))
    ws = torch.empty(B.sisso_select_workspace_bytes(), dtype=torch.uint8, device=dev)
    ranks1 = torch.empty(min(n1, 2 * K1 + 4096), dtype=torch.int64, device=dev)
    cnt1 = B.sisso_select_top(scores1, K1, ranks1, ws, st)
    pre1 = torch.empty((cnt1, m1), dtype=torch.int32, device=dev)
    B.sisso_colex_unrank(m1, ranks1[:cnt1], pre1, st)
    ext = torch.empty((cnt1 * (S - m1), m2), dtype=torch.int32, device=dev)
    B.sisso_l0_prefix_extend(search.handle, m1, pre1, ext)
    feat2 = torch.empty((ext.shape[0], B.PROP_NF), dtype=torch.float32, device=dev)
    B.sisso_l0_prefix_features(search.handle, m2, ext, feat2)
    scores2 = scorer(feat2)
    rows = torch.empty(min(ext.shape[0], 2 * K2 + 4096), dtype=torch.int64, device=dev)
    cnt2 = B.sisso_select_top(scores2, K2, rows, ws, st)
    pre2 = ext[rows[:cnt2]].contiguous()
    B.sisso_l0_search_list(search.handle, D, k, pre2)
    search.last_D, search.last_k = D, k
    return dict(stage1_scored=n1, stage1_kept=cnt1, stage2_scored=int(ext.shape[0]), prefixes_kept=cnt2,
                tuples_evaluated=cnt2 * (S - m2), tuples_total=math.comb(S, D))


def r2_scorer(feat):
    """The method without the network: rank prefixes by their own R^2."""
    return feat[:, 0].contiguous()


def recall(idx_a, idx_b) -> float:
    """|A n B| / |B| over rows of sorted index tuples."""
    a = {tuple(int(v) for v in t) for t in idx_a if t[0] >= 0}
    b = {tuple(int(v) for v in t) for t in idx_b if t[0] >= 0}
    return len(a & b) / max(1, len(b))
