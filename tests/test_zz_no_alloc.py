"""The selection entry point that allocates nothing (sisso_select_top_noalloc)
against the workspace form (sisso_select_top) through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[no-alloc] {msg}", flush=True)


def _select_both(B, torch, sc, K):
    st = torch.cuda.current_stream().cuda_stream
    d = torch.from_numpy(sc).to("cuda:0")
    cap = 2 * K + 4096
    out_ws = torch.full((cap,), -1, dtype=torch.int64, device="cuda:0")
    out_na = torch.full((cap,), -1, dtype=torch.int64, device="cuda:0")
    ws = torch.empty(B.sisso_select_workspace_bytes(), dtype=torch.uint8, device="cuda:0")
    n_ws = B.sisso_select_top(d, K, out_ws, ws, st)
    n_na = B.sisso_select_top_noalloc(d, K, out_na, st)
    return (n_ws, sorted(out_ws[:n_ws].cpu().numpy().tolist()),
            n_na, sorted(out_na[:n_na].cpu().numpy().tolist()))


def test_noalloc_select_matches_workspace_form_twice():
    import torch
    from paper_2502_20072_amd import _binding as B
    assert B.sisso_select_noalloc_scratch_bytes() >= B.sisso_select_workspace_bytes()
    rng = np.random.default_rng(2024)
    # two calls in a row on the same GPU, the second with a smaller input: the
    # fixed scratch keeps the first call's histograms and state, which the
    # second must not see
    for n, K in ((300000, 5000), (7000, 37)):
        sc = rng.normal(size=n).astype(np.float32)
        sc[::997] = np.nan
        _say(f"n={n} K={K}")
        n_ws, s_ws, n_na, s_na = _select_both(B, torch, sc, K)
        assert n_na == n_ws and s_na == s_ws
        # and the selected set is right: it holds the K largest finite scores
        order = np.argsort(-np.nan_to_num(sc, nan=-np.inf), kind="stable")
        assert n_na >= K and set(order[:K].tolist()) <= set(s_na)
        assert all(np.isfinite(sc[i]) for i in s_na)


def test_noalloc_select_rejects_bad_sizes_without_launching():
    import torch
    from paper_2502_20072_amd import _binding as B
    d = torch.zeros(10, dtype=torch.float32, device="cuda:0")
    out = torch.empty(16, dtype=torch.int64, device="cuda:0")
    with pytest.raises(B.SissoError, match="out of range"):
        B.sisso_select_top_noalloc(d, 11, out, torch.cuda.current_stream().cuda_stream)
