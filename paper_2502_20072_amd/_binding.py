"""ctypes binding of libsisso_l0.so -- argument marshalling only.

Each function mirrors the C entry point of the same name in
``include/sisso_l0.h``.  Device memory (inputs and the workspace) comes from
torch; every step of the computation runs in the library's HIP kernels.  If
the shared library is missing the import of a function fails loudly: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsisso_l0.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sisso_l0.h")

SISSO_OK, SISSO_EINVAL, SISSO_ESTATE, SISSO_ENOMEM, SISSO_EDEVICE, SISSO_ENOTSUP = 0, -1, -2, -3, -4, -5
SISSO_PREC_FP64, SISSO_PREC_BF16_COMP, SISSO_PREC_FP16_COMP, SISSO_PREC_FP32_SOLVE = 0, 1, 2, 3


def _header_int(name: str) -> int:
    with open(HEADER) as f:
        m = re.search(r"#define\s+%s\s+(\d+)" % name, f.read())
    return int(m.group(1))


SISSO_MAX_D = _header_int("SISSO_MAX_D")
SISSO_MAX_T = _header_int("SISSO_MAX_T")
SISSO_MAX_K = _header_int("SISSO_MAX_K")


class SissoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class sisso_l0_desc(ctypes.Structure):
    _fields_ = [
        ("F", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("task_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("n_total", ctypes.c_int64),
        ("S", ctypes.c_int64),
        ("T", ctypes.c_int32),
        ("D_max", ctypes.c_int32),
        ("k_max", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


_lib = None


def load():
    """Load the in-tree shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the GPU path has no fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    h = ctypes.c_void_p
    lib.sisso_l0_workspace_bytes.argtypes = [P(sisso_l0_desc)]
    lib.sisso_l0_workspace_bytes.restype = ctypes.c_size_t
    lib.sisso_l0_create.argtypes = [P(sisso_l0_desc), P(h)]
    lib.sisso_l0_create.restype = ctypes.c_int32
    lib.sisso_gram.argtypes = [h]
    lib.sisso_gram.restype = ctypes.c_int32
    lib.sisso_l0_search.argtypes = [h, ctypes.c_int32, ctypes.c_int32]
    lib.sisso_l0_search.restype = ctypes.c_int32
    lib.sisso_l0_search_range.argtypes = [h, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64]
    lib.sisso_l0_search_range.restype = ctypes.c_int32
    lib.sisso_l0_topk.argtypes = [h, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double)]
    lib.sisso_l0_topk.restype = ctypes.c_int32
    lib.sisso_gram_read.argtypes = [h, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double),
                                    P(ctypes.c_double)]
    lib.sisso_gram_read.restype = ctypes.c_int32
    lib.sisso_l0_scored.argtypes = [h]
    lib.sisso_l0_scored.restype = ctypes.c_uint64
    lib.sisso_l0_destroy.argtypes = [h]
    lib.sisso_l0_destroy.restype = None
    lib.sisso_l0_last_error.argtypes = [h]
    lib.sisso_l0_last_error.restype = ctypes.c_char_p
    lib.sisso_l0_rank_of.argtypes = [ctypes.c_int64, ctypes.c_int32, P(ctypes.c_int32)]
    lib.sisso_l0_rank_of.restype = ctypes.c_uint64
    lib.sisso_l0_unrank.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, P(ctypes.c_int32)]
    lib.sisso_l0_unrank.restype = ctypes.c_int32
    _lib = lib
    return lib


def _check(rc: int, handle=None):
    if rc != SISSO_OK:
        msg = load().sisso_l0_last_error(handle)
        raise SissoError(rc, (msg or b"").decode())


# ------------------------------------------------------------ thin wrappers
def make_desc(F_ptr: int, y_ptr: int, offsets: np.ndarray, n_total: int, S: int, D_max: int,
              k_max: int, workspace_ptr: int = 0, workspace_bytes: int = 0, stream: int = 0,
              precision: int = SISSO_PREC_FP64) -> sisso_l0_desc:
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    d = sisso_l0_desc()
    d.F = F_ptr
    d.y = y_ptr
    d._offsets_keepalive = offsets
    d.task_offsets = offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.n_total = n_total
    d.S = S
    d.T = len(offsets) - 1
    d.D_max = D_max
    d.k_max = k_max
    d.precision = precision
    d.workspace = workspace_ptr
    d.workspace_bytes = workspace_bytes
    d.stream = stream
    return d


def sisso_l0_workspace_bytes(desc: sisso_l0_desc) -> int:
    return int(load().sisso_l0_workspace_bytes(ctypes.byref(desc)))


def sisso_l0_create(desc: sisso_l0_desc) -> int:
    out = ctypes.c_void_p()
    _check(load().sisso_l0_create(ctypes.byref(desc), ctypes.byref(out)), None)
    return out.value


def sisso_gram(h: int) -> None:
    _check(load().sisso_gram(h), h)


def sisso_l0_search(h: int, D: int, k: int) -> None:
    _check(load().sisso_l0_search(h, D, k), h)


def sisso_l0_search_range(h: int, D: int, k: int, r0: int, r1: int) -> None:
    _check(load().sisso_l0_search_range(h, D, k, r0, r1), h)


def sisso_l0_topk(h: int, k: int, D: int, T: int, with_coef: bool = True):
    idx = np.full((k, D), -1, dtype=np.int32)
    sse = np.full(k, np.inf)
    coef = np.full((k, T, D + 1), np.nan) if with_coef else None
    P = ctypes.POINTER
    _check(load().sisso_l0_topk(h, k, idx.ctypes.data_as(P(ctypes.c_int32)),
                                sse.ctypes.data_as(P(ctypes.c_double)),
                                coef.ctypes.data_as(P(ctypes.c_double)) if with_coef else None), h)
    return idx, sse, coef


def sisso_gram_read(h: int, t: int, S: int):
    G = np.empty((S, S))
    b = np.empty(S)
    c = np.empty(1)
    P = ctypes.POINTER(ctypes.c_double)
    _check(load().sisso_gram_read(h, t, G.ctypes.data_as(P), b.ctypes.data_as(P), c.ctypes.data_as(P)), h)
    return G, b, float(c[0])


def sisso_l0_scored(h: int) -> int:
    return int(load().sisso_l0_scored(h))


def sisso_l0_destroy(h: Optional[int]) -> None:
    load().sisso_l0_destroy(h)


def sisso_l0_last_error(h: Optional[int]) -> str:
    return (load().sisso_l0_last_error(h) or b"").decode()


def sisso_l0_rank_of(S: int, tup: Sequence[int]) -> int:
    t = np.ascontiguousarray(tup, dtype=np.int32)
    return int(load().sisso_l0_rank_of(S, len(t), t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))


def sisso_l0_unrank(S: int, D: int, r: int):
    t = np.zeros(D, dtype=np.int32)
    _check(load().sisso_l0_unrank(S, D, r, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return tuple(int(v) for v in t)


PHASES = ("stats", "gram", "prepass", "search", "merge", "rescore", "final")


def sisso_l0_profile(h: int, enable: bool) -> None:
    lib = load()
    lib.sisso_l0_profile.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.sisso_l0_profile.restype = ctypes.c_int32
    _check(lib.sisso_l0_profile(h, 1 if enable else 0), h)


def sisso_l0_phase_ms(h: int) -> dict:
    lib = load()
    lib.sisso_l0_phase_ms.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.sisso_l0_phase_ms.restype = ctypes.c_int32
    ms = np.zeros(len(PHASES))
    _check(lib.sisso_l0_phase_ms(h, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), h)
    return dict(zip(PHASES, ms.tolist()))


def sisso_l0_search_stats(h: int) -> dict:
    lib = load()
    lib.sisso_l0_search_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    lib.sisso_l0_search_stats.restype = ctypes.c_int32
    out = np.zeros(4, dtype=np.uint64)
    _check(lib.sisso_l0_search_stats(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), h)
    return dict(candidates=int(out[0]), items=int(out[1]),
                theta0=float(out[2:3].view(np.float64)[0]), theta_final=float(out[3:4].view(np.float64)[0]))


def sisso_l0_precision_report(h: int, nsample: int = 4096) -> dict:
    lib = load()
    lib.sisso_l0_precision_report.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.sisso_l0_precision_report.restype = ctypes.c_int32
    out = np.zeros(4)
    _check(lib.sisso_l0_precision_report(h, nsample, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), h)
    return dict(gram_max_abs_err=float(out[0]), gram_entries=int(out[1]), sse_max_rel_err=float(out[2]),
                slices=int(out[3]))


def sisso_gram_error(h: int) -> float:
    lib = load()
    lib.sisso_gram_error.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.sisso_gram_error.restype = ctypes.c_int32
    out = ctypes.c_double(0.0)
    _check(lib.sisso_gram_error(h, ctypes.byref(out)), h)
    return float(out.value)


def sisso_l0_set_search_grid(h: int, workgroups: int) -> None:
    lib = load()
    lib.sisso_l0_set_search_grid.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.sisso_l0_set_search_grid.restype = ctypes.c_int32
    _check(lib.sisso_l0_set_search_grid(h, workgroups), h)


def sisso_l0_search_grid(h: int) -> int:
    lib = load()
    lib.sisso_l0_search_grid.argtypes = [ctypes.c_void_p]
    lib.sisso_l0_search_grid.restype = ctypes.c_int32
    return int(lib.sisso_l0_search_grid(h))


def sisso_l0_autotune(h: int, D: int, k: int, cache_path: Optional[str] = None) -> int:
    lib = load()
    lib.sisso_l0_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.sisso_l0_autotune.restype = ctypes.c_int32
    out = ctypes.c_int32(0)
    path = cache_path.encode() if cache_path else None
    _check(lib.sisso_l0_autotune(h, D, k, path, ctypes.byref(out)), h)
    return int(out.value)


def _batch_sigs(lib):
    P = ctypes.POINTER
    lib.sisso_l0_batch_create.argtypes = [P(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          P(ctypes.c_void_p)]
    lib.sisso_l0_batch_create.restype = ctypes.c_int32
    lib.sisso_l0_batch_launch.argtypes = [ctypes.c_void_p]
    lib.sisso_l0_batch_launch.restype = ctypes.c_int32
    lib.sisso_l0_batch_destroy.argtypes = [ctypes.c_void_p]
    lib.sisso_l0_batch_destroy.restype = None
    lib.sisso_l0_batch_last_error.restype = ctypes.c_char_p
    lib.sisso_l0_search_batch.argtypes = [P(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.sisso_l0_search_batch.restype = ctypes.c_int32


def _batch_check(rc: int):
    if rc != SISSO_OK:
        raise SissoError(rc, (load().sisso_l0_batch_last_error() or b"").decode())


def sisso_l0_batch_create(handles, D: int, k: int) -> int:
    lib = load()
    _batch_sigs(lib)
    arr = (ctypes.c_void_p * len(handles))(*handles)
    out = ctypes.c_void_p()
    _batch_check(lib.sisso_l0_batch_create(arr, len(handles), D, k, ctypes.byref(out)))
    return out.value


def sisso_l0_batch_launch(b: int) -> None:
    lib = load()
    _batch_sigs(lib)
    _batch_check(lib.sisso_l0_batch_launch(b))


def sisso_l0_batch_destroy(b) -> None:
    lib = load()
    _batch_sigs(lib)
    lib.sisso_l0_batch_destroy(b)


def sisso_l0_search_batch(handles, D: int, k: int) -> None:
    lib = load()
    _batch_sigs(lib)
    arr = (ctypes.c_void_p * len(handles))(*handles)
    _batch_check(lib.sisso_l0_search_batch(arr, len(handles), D, k))


# ------------------------------------------------ prefix lists and the MLP
MLP_IN = 8
MLP_HIDDEN = 128
MLP_NPARAM = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1
PROP_NF = 8

_sigs_done = False


def _prop_sigs(lib):
    global _sigs_done
    if _sigs_done:
        return
    P, V, I32, I64, U64, SZ = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    for name, args in [("sisso_l0_prefix_best", [V, I32, V, I64, V]),
                       ("sisso_l0_prefix_target", [V, I32, V, I64, V, V]),
                       ("sisso_l0_prefix_features", [V, I32, V, I64, V]),
                       ("sisso_l0_prefix_features_range", [V, I32, U64, I64, V]),
                       ("sisso_l0_prefix_extend", [V, I32, V, I64, V]),
                       ("sisso_l0_search_list", [V, I32, I32, V, I64]),
                       ("sisso_mlp_forward", [V, V, I64, V, V, SZ, V]),
                       ("sisso_mlp_backward", [V, V, V, I64, V, V, V, SZ, V]),
                       ("sisso_mlp_adam", [V, V, V, V, I32, ctypes.c_float, V]),
                       ("sisso_mlp_infer_bf16", [V, V, I64, V, V]),
                       ("sisso_select_top", [V, I64, I64, V, I64, P(I64), V, SZ, V]),
                       ("sisso_select_top_noalloc", [V, I64, I64, V, I64, P(I64), V]),
                       ("sisso_colex_unrank", [I32, V, I64, V, V])]:
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I32
    lib.sisso_mlp_workspace_bytes.argtypes = [I64]
    lib.sisso_mlp_workspace_bytes.restype = SZ
    lib.sisso_select_workspace_bytes.argtypes = []
    lib.sisso_select_workspace_bytes.restype = SZ
    lib.sisso_select_noalloc_scratch_bytes.argtypes = []
    lib.sisso_select_noalloc_scratch_bytes.restype = SZ
    lib.sisso_select_last_error.argtypes = []
    lib.sisso_select_last_error.restype = ctypes.c_char_p
    _sigs_done = True


def _plib():
    lib = load()
    _prop_sigs(lib)
    return lib


def _ptr(t) -> int:
    return int(t.data_ptr())


def _raw_check(rc: int, what: str):
    if rc != SISSO_OK:
        raise SissoError(rc, f"{what} failed ({rc})")


def sisso_l0_prefix_best(h: int, m: int, prefixes, best) -> None:
    _check(_plib().sisso_l0_prefix_best(h, m, _ptr(prefixes), prefixes.shape[0], _ptr(best)), h)


def sisso_l0_prefix_target(h: int, m: int, prefixes, best, target) -> None:
    _check(_plib().sisso_l0_prefix_target(h, m, _ptr(prefixes), prefixes.shape[0], _ptr(best), _ptr(target)), h)


def sisso_l0_prefix_features(h: int, m: int, prefixes, feat) -> None:
    _check(_plib().sisso_l0_prefix_features(h, m, _ptr(prefixes), prefixes.shape[0], _ptr(feat)), h)


def sisso_l0_prefix_extend(h: int, m: int, prefixes, out) -> None:
    _check(_plib().sisso_l0_prefix_extend(h, m, _ptr(prefixes), prefixes.shape[0], _ptr(out)), h)


def sisso_l0_prefix_features_range(h: int, m: int, r0: int, n: int, feat) -> None:
    _check(_plib().sisso_l0_prefix_features_range(h, m, r0, n, _ptr(feat)), h)


def sisso_l0_search_list(h: int, D: int, k: int, prefixes) -> None:
    _check(_plib().sisso_l0_search_list(h, D, k, _ptr(prefixes), prefixes.shape[0]), h)


def sisso_mlp_workspace_bytes(n: int) -> int:
    return int(_plib().sisso_mlp_workspace_bytes(n))


def sisso_mlp_forward(params, x, out, ws, stream: int) -> None:
    _raw_check(_plib().sisso_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(out), _ptr(ws), ws.numel(), stream),
               "sisso_mlp_forward")


def sisso_mlp_backward(params, x, target, grad, loss, ws, stream: int) -> None:
    _raw_check(_plib().sisso_mlp_backward(_ptr(params), _ptr(x), _ptr(target), x.shape[0], _ptr(grad), _ptr(loss),
                                          _ptr(ws), ws.numel(), stream), "sisso_mlp_backward")


def sisso_mlp_adam(params, grad, m, v, step: int, lr: float, stream: int) -> None:
    _raw_check(_plib().sisso_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, stream), "sisso_mlp_adam")


def sisso_mlp_infer_bf16(params, x, out, stream: int) -> None:
    _raw_check(_plib().sisso_mlp_infer_bf16(_ptr(params), _ptr(x), x.shape[0], _ptr(out), stream),
               "sisso_mlp_infer_bf16")


def sisso_select_workspace_bytes() -> int:
    return int(_plib().sisso_select_workspace_bytes())


def sisso_select_top(scores, K: int, out, ws, stream: int) -> int:
    cnt = ctypes.c_int64(0)
    _raw_check(_plib().sisso_select_top(_ptr(scores), scores.shape[0], K, _ptr(out), out.shape[0], ctypes.byref(cnt),
                                        _ptr(ws), ws.numel(), stream), "sisso_select_top")
    return int(cnt.value)


def sisso_select_top_noalloc(scores, K: int, out, stream: int) -> int:
    """sisso_select_top on the library's fixed device scratch (no workspace)."""
    lib = _plib()
    cnt = ctypes.c_int64(0)
    rc = lib.sisso_select_top_noalloc(_ptr(scores), scores.shape[0], K, _ptr(out), out.shape[0],
                                      ctypes.byref(cnt), stream)
    if rc != SISSO_OK:
        raise SissoError(rc, "sisso_select_top_noalloc: " + lib.sisso_select_last_error().decode())
    return int(cnt.value)


def sisso_select_noalloc_scratch_bytes() -> int:
    return int(_plib().sisso_select_noalloc_scratch_bytes())


def sisso_colex_unrank(m: int, ranks, prefixes, stream: int) -> None:
    _raw_check(_plib().sisso_colex_unrank(m, _ptr(ranks), ranks.shape[0], _ptr(prefixes), stream),
               "sisso_colex_unrank")


# ---------------------------------------------------------------------------
# include/sisso_sis.h: screening, feature creation, residuals, top-m, the
# dimension loop.  Tensors are torch device tensors; marshalling only.
SISSO_OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "abs_diff": 4, "exp": 16, "neg_exp": 17, "log": 18,
             "abs": 19, "sqrt": 20, "cbrt": 21, "sq": 22, "cb": 23, "inv": 24, "sin": 25, "cos": 26,
             "six_pow": 27}


class sisso_sis_desc(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_void_p),
        ("task_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("n_total", ctypes.c_int64),
        ("T", ctypes.c_int32),
        ("nres", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


class sisso_fit_desc(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("task_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("n_total", ctypes.c_int64),
        ("M", ctypes.c_int64),
        ("T", ctypes.c_int32),
        ("D_max", ctypes.c_int32),
        ("m_sis", ctypes.c_int32),
        ("n_res", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
    ]


_sis_sigs_done = False


def _slib():
    global _sis_sigs_done
    lib = load()
    if _sis_sigs_done:
        return lib
    P, V, I32, I64, SZ, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    sigs = {
        "sisso_sis_workspace_bytes": ([P(sisso_sis_desc)], SZ),
        "sisso_sis_create": ([P(sisso_sis_desc), P(V)], I32),
        "sisso_sis_destroy": ([V], None),
        "sisso_sis_last_error": ([V], ctypes.c_char_p),
        "sisso_sis_score": ([V, V, I64, V], I32),
        "sisso_sis_score_op": ([V, I32, V, I64, V, I64, D, D, V, V], I32),
        "sisso_fc_eval": ([I32, V, I64, I64, V, I64, D, D, V, V, V], I32),
        "sisso_topm_workspace_bytes": ([I64, I32], SZ),
        "sisso_topm": ([V, I64, I32, V, V, P(I32), V, SZ, V], I32),
        "sisso_residuals": ([V, V, I64, I64, V, I32, V, V, I32, I32, V, V], I32),
        "sisso_fit_workspace_bytes": ([P(sisso_fit_desc)], SZ),
        "sisso_fit": ([P(sisso_fit_desc), V, V, V, V], I32),
        "sisso_fit_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _sis_sigs_done = True
    return lib


def _stream_of(t) -> int:
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def _ws(nbytes: int, device):
    """A 256-byte aligned workspace: (tensor kept alive, aligned address)."""
    import torch
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    return buf, (buf.data_ptr() + 255) & ~255


class SisScreen:
    """A screening handle (sisso_sis_create) for residuals R (n, nres) as a
    device float64 tensor stored residual-major: R[r] is residual r."""

    def __init__(self, R, task_offsets=None):
        R = R if R.dim() == 2 else R.reshape(1, -1)
        self.R = R.contiguous()
        nres, n = self.R.shape
        self.offsets = np.ascontiguousarray([0, n] if task_offsets is None else task_offsets, dtype=np.int64)
        self.n, self.T, self.nres = int(n), len(self.offsets) - 1, int(nres)
        lib = _slib()
        d = sisso_sis_desc(self.R.data_ptr(), self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           self.n, self.T, self.nres, None, 0, _stream_of(self.R))
        nbytes = lib.sisso_sis_workspace_bytes(ctypes.byref(d))
        if nbytes == 0:
            raise SissoError(SISSO_EINVAL, "screening shape out of range")
        self._buf, d.workspace = _ws(nbytes, self.R.device)
        d.workspace_bytes = nbytes
        h = ctypes.c_void_p()
        rc = lib.sisso_sis_create(ctypes.byref(d), ctypes.byref(h))
        if rc != SISSO_OK:
            raise SissoError(rc, lib.sisso_sis_last_error(None).decode())
        self.handle = h.value

    def _check(self, rc):
        if rc != SISSO_OK:
            raise SissoError(rc, _slib().sisso_sis_last_error(self.handle).decode())

    def score(self, X, scores):
        """X: (M, n) device float64 (feature-major); scores: (M,) float64."""
        self._check(_slib().sisso_sis_score(self.handle, X.data_ptr(), X.shape[0], scores.data_ptr()))

    def score_op(self, op: str, X, pairs, lower: float, upper: float, scores, valid=None):
        self._check(_slib().sisso_sis_score_op(self.handle, SISSO_OPS[op], X.data_ptr(), X.shape[0],
                                               pairs.data_ptr(), pairs.shape[0], lower, upper, scores.data_ptr(),
                                               valid.data_ptr() if valid is not None else None))

    def close(self):
        if getattr(self, "handle", None):
            _slib().sisso_sis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sisso_fc_eval(op: str, X, pairs, lower: float, upper: float, out, valid) -> None:
    rc = _slib().sisso_fc_eval(SISSO_OPS[op], X.data_ptr(), X.shape[1], X.shape[0], pairs.data_ptr(), pairs.shape[0],
                               lower, upper, out.data_ptr() if out is not None else None, valid.data_ptr(),
                               _stream_of(X))
    _raw_check(rc, "sisso_fc_eval")


def sisso_topm(scores, m: int, out_idx, out_score=None) -> int:
    lib = _slib()
    nbytes = lib.sisso_topm_workspace_bytes(scores.shape[0], m)
    if nbytes == 0:
        raise SissoError(SISSO_EINVAL, "top-m sizes out of range")
    buf, addr = _ws(nbytes, scores.device)
    cnt = ctypes.c_int32(0)
    rc = lib.sisso_topm(scores.data_ptr(), scores.shape[0], m, out_idx.data_ptr(),
                        out_score.data_ptr() if out_score is not None else None, ctypes.byref(cnt), addr, nbytes,
                        _stream_of(scores))
    _raw_check(rc, "sisso_topm")
    del buf
    return int(cnt.value)


def sisso_residuals(F, y, task_offsets_dev, idx, coef, R) -> None:
    """F (S, n), y (n,), task_offsets_dev (T+1,) int64 on the device, idx (r, D)
    int32, coef (r, T, D+1) float64, R (r, n) float64 out."""
    r, D = idx.shape
    rc = _slib().sisso_residuals(F.data_ptr(), y.data_ptr(), F.shape[1], F.shape[0], task_offsets_dev.data_ptr(),
                                 task_offsets_dev.shape[0] - 1, idx.data_ptr(), coef.data_ptr(), r, D, R.data_ptr(),
                                 _stream_of(F))
    _raw_check(rc, "sisso_residuals")


def sisso_fit(X, y, task_offsets, D_max: int, m_sis: int, n_res: int, k: int) -> dict:
    """The dimension loop (sisso_fit).  X (M, n) and y (n,) device float64."""
    lib = _slib()
    M, n = X.shape
    offs = np.ascontiguousarray([0, n] if task_offsets is None else task_offsets, dtype=np.int64)
    T = len(offs) - 1
    d = sisso_fit_desc(X.data_ptr(), y.data_ptr(), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n, M, T,
                       D_max, m_sis, n_res, k, None, 0, _stream_of(X))
    nbytes = lib.sisso_fit_workspace_bytes(ctypes.byref(d))
    if nbytes == 0:
        raise SissoError(SISSO_EINVAL, "dimension-loop sizes out of range")
    buf, d.workspace = _ws(nbytes, X.device)
    d.workspace_bytes = nbytes
    sub = np.zeros(D_max * m_sis, dtype=np.int32)
    models = np.zeros((D_max, k, D_max), dtype=np.int32)
    sse = np.zeros((D_max, k))
    coef = np.zeros((D_max, k, T, D_max + 1))
    rc = lib.sisso_fit(ctypes.byref(d), sub.ctypes.data, models.ctypes.data, sse.ctypes.data, coef.ctypes.data)
    del buf
    if rc != SISSO_OK:
        raise SissoError(rc, lib.sisso_fit_last_error().decode())
    return dict(subspace=sub, models=models, sse=sse, coef=coef)
