"""MI355X (gfx950) library for the l0 step of SISSO.

``L0Search`` holds one problem (features F, target y, task partition) in
device memory and drives the C ABI of ``libsisso_l0.so``: Gram precompute,
exhaustive search of all D-tuples, top-k readout.  torch provides the device
memory and the stream; all arithmetic runs in the library's HIP kernels.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import _binding as B
from ._binding import SissoError  # noqa: F401


class L0Search:
    """One l0 problem on the GPU.

    F: (S, n) float64 tensor on a ROCm device (row j = the samples of
       feature j, i.e. the n x S matrix stored column-major), or a numpy
       array that is copied to ``device``.
    y: (n,) float64.
    task_offsets: T+1 row offsets (default: one task).
    """

    def __init__(self, F, y, task_offsets: Optional[Sequence[int]] = None, D_max: int = 4,
                 k_max: int = 100, device: str = "cuda:0", stream=None, precision: int = B.SISSO_PREC_FP64):
        import torch

        if isinstance(F, np.ndarray):
            F = torch.from_numpy(np.ascontiguousarray(F, dtype=np.float64)).to(device)
        if isinstance(y, np.ndarray):
            y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).to(F.device)
        if F.dtype != torch.float64 or y.dtype != torch.float64:
            raise TypeError("F and y must be float64")
        if not (F.is_cuda and y.is_cuda):
            raise TypeError("F and y must be device tensors")
        self.F = F.contiguous()
        self.y = y.contiguous()
        S, n = self.F.shape
        if self.y.shape != (n,):
            raise ValueError("y must have one value per sample")
        if task_offsets is None:
            task_offsets = [0, n]
        self.offsets = np.ascontiguousarray(task_offsets, dtype=np.int64)
        self.S, self.n, self.T = int(S), int(n), len(self.offsets) - 1
        self.D_max, self.k_max = int(D_max), int(k_max)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.F.device)
        self.precision = int(precision)
        probe = B.make_desc(0, 0, self.offsets, self.n, self.S, self.D_max, self.k_max,
                            precision=self.precision)
        nbytes = B.sisso_l0_workspace_bytes(probe)
        if nbytes == 0:
            raise SissoError(B.SISSO_EINVAL, "problem shape out of range")
        # over-allocate so the workspace can be aligned to 256 bytes
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.F.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        self.workspace_bytes = nbytes
        self._desc = B.make_desc(self.F.data_ptr(), self.y.data_ptr(), self.offsets, self.n, self.S,
                                 self.D_max, self.k_max, aligned, nbytes, self.stream.cuda_stream,
                                 precision=self.precision)
        cur = torch.cuda.current_stream(self.F.device)
        if self.stream.cuda_stream != cur.cuda_stream:
            # the inputs (uploads, contiguous copies) and the workspace were
            # made on the current stream: the handle's stream waits for that
            # work, and the allocator is told that the handle's stream uses
            # these blocks (so it does not hand them out again while the
            # handle's work may still touch them)
            self.stream.wait_stream(cur)
            for t in (self.F, self.y, self._ws):
                t.record_stream(self.stream)
        self.handle = B.sisso_l0_create(self._desc)
        self.last_D = None
        self.last_k = None

    # --- C ABI calls (enqueue on self.stream) ---
    def gram(self) -> "L0Search":
        B.sisso_gram(self.handle)
        return self

    def search(self, D: int, k: int) -> "L0Search":
        B.sisso_l0_search(self.handle, D, k)
        self.last_D, self.last_k = D, k
        return self

    def search_range(self, D: int, k: int, r0: int, r1: int) -> "L0Search":
        B.sisso_l0_search_range(self.handle, D, k, r0, r1)
        self.last_D, self.last_k = D, k
        return self

    def topk(self, k: Optional[int] = None, with_coef: bool = True):
        """(idx (k, D) int32, sse (k,), coef (k, T, D+1) or None); synchronises."""
        k = self.last_k if k is None else k
        return B.sisso_l0_topk(self.handle, k, self.last_D, self.T, with_coef)

    def gram_read(self, t: int = 0):
        """(G (S, S), b (S,), c) of task t; synchronises."""
        return B.sisso_gram_read(self.handle, t, self.S)

    def scored(self) -> int:
        return B.sisso_l0_scored(self.handle)

    def autotune(self, D: int, k: int, cache_path: Optional[str] = None) -> int:
        """Pick the fastest search grid for (D, k) (cached by shape); leaves the
        handle with the result of a search of (D, k).  Returns the grid size."""
        g = B.sisso_l0_autotune(self.handle, D, k, cache_path)
        self.last_D, self.last_k = D, k
        return g

    def set_search_grid(self, workgroups: int) -> None:
        B.sisso_l0_set_search_grid(self.handle, workgroups)

    def precision_report(self, nsample: int = 4096) -> dict:
        """Gram error on sampled entries vs FP64 from F, and the ranked-vs-exact
        SSE error of the last search's results; synchronises."""
        return B.sisso_l0_precision_report(self.handle, nsample)

    def close(self) -> None:
        if getattr(self, "handle", None):
            B.sisso_l0_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rank_of(S: int, tup: Sequence[int]) -> int:
    return B.sisso_l0_rank_of(S, tup)


def unrank(S: int, D: int, r: int):
    return B.sisso_l0_unrank(S, D, r)
