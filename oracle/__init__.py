"""CPU FP64 oracle for the SISSO l0 step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The GPU library does not import it and shares none of its code.

The arithmetic lives in ``oracle_l0.c`` (plain C99, per-tuple Householder QR,
as the paper's l0 section describes); this module only marshals numpy arrays
into it.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_l0.c")
_LIB = os.path.join(_HERE, "liboracle_l0.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    P = ctypes.POINTER
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    lib.oracle_tuple_sse.argtypes = [P(d), P(d), P(i64), ctypes.c_int, i64, i64, ctypes.c_int,
                                     P(i32), P(d), P(d)]
    lib.oracle_tuple_sse.restype = ctypes.c_int
    lib.oracle_l0_topk.argtypes = [P(d), P(d), P(i64), ctypes.c_int, i64, i64, ctypes.c_int,
                                   ctypes.c_int, i64, i64, P(i32), P(d), ctypes.c_int]
    lib.oracle_l0_topk.restype = i64
    lib.oracle_all_sse.argtypes = [P(d), P(d), P(i64), ctypes.c_int, i64, i64, ctypes.c_int,
                                   P(d), i64]
    lib.oracle_all_sse.restype = i64
    lib.oracle_max_d.restype = ctypes.c_int
    return lib


def _prep(F, y, offsets):
    F = np.ascontiguousarray(F, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    S, n = F.shape
    if offsets is None:
        offsets = np.array([0, n], dtype=np.int64)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    return F, y, offsets, S, n, len(offsets) - 1


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def tuple_sse(F, y, tup: Sequence[int], offsets=None, with_coef: bool = False):
    """SSE (summed over tasks) of one tuple; optionally coefficients (T, D+1)."""
    lib = _load()
    F, y, offsets, S, n, T = _prep(F, y, offsets)
    t = np.ascontiguousarray(tup, dtype=np.int32)
    D = len(t)
    out = np.zeros(1)
    coef = np.full((T, D + 1), np.nan) if with_coef else None
    rc = lib.oracle_tuple_sse(_ptr(F, ctypes.c_double), _ptr(y, ctypes.c_double),
                              _ptr(offsets, ctypes.c_int64), T, n, S, D, _ptr(t, ctypes.c_int32),
                              _ptr(out, ctypes.c_double),
                              _ptr(coef, ctypes.c_double) if with_coef else None)
    if rc != 0:
        raise ValueError("oracle_tuple_sse: invalid arguments")
    return (float(out[0]), coef) if with_coef else float(out[0])


def topk(F, y, D: int, k: int, offsets=None, i1_range: Optional[Tuple[int, int]] = None,
         threads: int = 0):
    """Top-k tuples by (SSE, lex).  Returns (idx (k, D) int32, sse (k,), n_scored)."""
    lib = _load()
    F, y, offsets, S, n, T = _prep(F, y, offsets)
    lo, hi = (0, S) if i1_range is None else i1_range
    idx = np.full((k, D), -1, dtype=np.int32)
    sse = np.full(k, np.inf)
    cnt = lib.oracle_l0_topk(_ptr(F, ctypes.c_double), _ptr(y, ctypes.c_double),
                             _ptr(offsets, ctypes.c_int64), T, n, S, D, k, lo, hi,
                             _ptr(idx, ctypes.c_int32), _ptr(sse, ctypes.c_double), threads)
    if cnt < 0:
        raise ValueError("oracle_l0_topk: invalid arguments")
    return idx, sse, int(cnt)


def all_sse(F, y, D: int, offsets=None) -> np.ndarray:
    """SSE of every D-tuple, in lexicographic order (small problems only)."""
    lib = _load()
    F, y, offsets, S, n, T = _prep(F, y, offsets)
    total = math.comb(S, D)
    out = np.empty(total)
    cnt = lib.oracle_all_sse(_ptr(F, ctypes.c_double), _ptr(y, ctypes.c_double),
                             _ptr(offsets, ctypes.c_int64), T, n, S, D,
                             _ptr(out, ctypes.c_double), total)
    if cnt != total:
        raise ValueError("oracle_all_sse: invalid arguments")
    return out


def max_d() -> int:
    return int(_load().oracle_max_d())


def threads() -> int:
    """OpenMP threads the oracle uses by default."""
    lib = _load()
    lib.oracle_threads.restype = ctypes.c_int
    return int(lib.oracle_threads())
