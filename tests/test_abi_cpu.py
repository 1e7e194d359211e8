"""C ABI checks that need no GPU: the library loads, exports every function
the header declares, sizes workspaces as a pure function of the shape,
rejects bad descriptors before touching a device, and its host-side
combinatorial number system is a bijection."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

from paper_2502_20072_amd import _binding as B
import paper_2502_20072_amd as P


def _declared_functions(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sisso_\w+)\s*\(", text)))


def _headers():
    inc = os.path.dirname(B.HEADER)
    return sorted(os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h"))


def test_exports_every_declared_symbol():
    lib = B.load()
    heads = _headers()
    assert len(heads) >= 3
    total = 0
    for h in heads:
        names = _declared_functions(h)
        total += len(names)
        for n in names:
            assert hasattr(lib, n), f"{n} declared in {os.path.basename(h)} but not exported"
    assert total >= 40


def _desc(n=100, S=20, offsets=None, D_max=3, k_max=10, ws=0, wsb=0, F=0, y=0):
    offsets = np.array([0, n] if offsets is None else offsets, dtype=np.int64)
    return B.make_desc(F, y, offsets, n, S, D_max, k_max, ws, wsb)


def test_workspace_bytes_pure_and_validating():
    a = B.sisso_l0_workspace_bytes(_desc())
    b = B.sisso_l0_workspace_bytes(_desc())
    assert a == b > 0
    assert B.sisso_l0_workspace_bytes(_desc(S=40)) > a
    assert B.sisso_l0_workspace_bytes(_desc(D_max=0)) == 0
    assert B.sisso_l0_workspace_bytes(_desc(D_max=B.SISSO_MAX_D + 1)) == 0
    assert B.sisso_l0_workspace_bytes(_desc(k_max=B.SISSO_MAX_K + 1)) == 0
    # the big multi-task workload fits a single MI355X comfortably
    big = B.sisso_l0_workspace_bytes(_desc(n=17000, S=1500, offsets=np.linspace(0, 17000, 17).astype(np.int64),
                                           D_max=3, k_max=100))
    assert 0 < big < 4 << 30


def test_create_rejects_bad_descriptors_without_device():
    with pytest.raises(B.SissoError) as e:
        B.sisso_l0_create(_desc())            # null F / y / workspace
    assert e.value.code == B.SISSO_EINVAL
    assert "null" in B.sisso_l0_last_error(None)
    with pytest.raises(B.SissoError) as e:
        B.sisso_l0_create(_desc(F=8, y=8, ws=256, wsb=1 << 40, offsets=[0, 50, 40, 100]))
    assert e.value.code == B.SISSO_EINVAL
    with pytest.raises(B.SissoError) as e:
        B.sisso_l0_create(_desc(F=8, y=8, ws=256, wsb=16))
    assert e.value.code == B.SISSO_ENOMEM
    with pytest.raises(B.SissoError) as e:
        B.sisso_l0_create(_desc(F=8, y=8, ws=257, wsb=1 << 40))
    assert e.value.code == B.SISSO_EINVAL
    d = _desc(F=8, y=8, ws=256, wsb=1 << 40)
    d.precision = 7
    with pytest.raises(B.SissoError) as e:
        B.sisso_l0_create(d)
    assert e.value.code == B.SISSO_ENOTSUP


def test_null_handle_calls():
    lib = B.load()
    assert lib.sisso_gram(None) == B.SISSO_EINVAL
    assert lib.sisso_l0_search(None, 2, 3) == B.SISSO_EINVAL
    assert lib.sisso_l0_scored(None) == 0
    lib.sisso_l0_destroy(None)


@pytest.mark.parametrize("S,D", [(1, 1), (6, 3), (9, 4), (12, 2), (12, 4), (7, 7)])
def test_lex_rank_bijection(S, D):
    for r, t in enumerate(itertools.combinations(range(S), D)):
        assert P.rank_of(S, t) == r
        assert P.unrank(S, D, r) == t


@pytest.mark.parametrize("S,D", [(600, 4), (5000, 3), (50000, 2), (65535, 4), (1500, 3)])
def test_rank_space_edges_64bit(S, D):
    N = math.comb(S, D)
    assert P.unrank(S, D, 0) == tuple(range(D))
    assert P.unrank(S, D, N - 1) == tuple(range(S - D, S))
    for r in [1, N // 7, N // 2, N - 2]:
        assert P.rank_of(S, P.unrank(S, D, r)) == r
    with pytest.raises(B.SissoError):
        P.unrank(S, D, N)
    assert P.rank_of(S, [0] * D) == (1 << 64) - 1 if D > 1 else True


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        B.load()


def test_tuning_and_report_entry_points_reject_null_handle():
    lib = B.load()
    lib.sisso_l0_set_search_grid.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.sisso_l0_set_search_grid.restype = ctypes.c_int32
    lib.sisso_l0_search_grid.argtypes = [ctypes.c_void_p]
    lib.sisso_l0_search_grid.restype = ctypes.c_int32
    lib.sisso_l0_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.sisso_l0_autotune.restype = ctypes.c_int32
    lib.sisso_l0_precision_report.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    lib.sisso_l0_precision_report.restype = ctypes.c_int32
    assert lib.sisso_l0_set_search_grid(None, 256) == B.SISSO_EINVAL
    assert lib.sisso_l0_search_grid(None) == 0
    assert lib.sisso_l0_autotune(None, 3, 10, None, None) == B.SISSO_EINVAL
    out = (ctypes.c_double * 4)()
    assert lib.sisso_l0_precision_report(None, 16, out) == B.SISSO_EINVAL


def test_precision_modes_size_the_workspace():
    def ws(prec, n=5000, S=300):
        d = B.make_desc(0, 0, np.array([0, n], dtype=np.int64), n, S, 2, 10, precision=prec)
        return B.sisso_l0_workspace_bytes(d)
    fp64, bf16 = ws(B.SISSO_PREC_FP64), ws(B.SISSO_PREC_BF16_COMP)
    # three BF16 slices of every padded column plus one exponent per 256-sample chunk
    n_chunks = (5000 + 255) // 256 + 1
    assert bf16 - fp64 >= 3 * 300 * n_chunks * 256 * 2 + 300 * n_chunks * 4
    # two FP16 slices: less slice memory than three BF16 slices, more than none
    fp16 = ws(B.SISSO_PREC_FP16_COMP)
    assert fp16 - fp64 >= 2 * 300 * n_chunks * 256 * 2 + 300 * n_chunks * 4
    assert fp16 < bf16
    assert ws(7) == 0


def test_fp32_solve_form_drops_the_record_tables():
    """The FP32 solve form keeps the FP64 Gram (no slices) and runs the
    general kernels, so it holds no D = 3 / D = 4 record table; its lists are
    twice as long (2 (k + 16) candidates for the FP64 re-score)."""
    def ws(prec, D):
        d = B.make_desc(0, 0, np.array([0, 2000], dtype=np.int64), 2000, 300, D, 100, precision=prec)
        return B.sisso_l0_workspace_bytes(d)
    # D_max = 2: no table in either form, only the longer lists
    assert ws(B.SISSO_PREC_FP32_SOLVE, 2) > ws(B.SISSO_PREC_FP64, 2)
    # D_max = 4: the FP64 form carries the D = 3 and D = 4 record tables
    # (C(300, 3) / 6 x 160 bytes of D = 4 records alone), the FP32 form none
    rec4 = (300 ** 3 // 24) * 160
    assert ws(B.SISSO_PREC_FP64, 4) - ws(B.SISSO_PREC_FP32_SOLVE, 4) > rec4 // 2


def test_several_task_d3_workspace_holds_filter_matrix_and_step_queue():
    """With several tasks and D_max >= 3 the workspace also holds the filter
    task's matrix alone (S^2 doubles, one-task tiled, so padded to 64) and
    the D = 3 step queue (24 bytes per sweep step plus a chunk per wave);
    neither exists for one task or for D_max = 2."""
    S = 300
    Sp = (S + 63) // 64 * 64
    off2 = np.array([0, 150, 300], dtype=np.int64)

    def ws(offsets, D_max):
        return B.sisso_l0_workspace_bytes(_desc(n=int(offsets[-1]), S=S, offsets=offsets, D_max=D_max, k_max=20))

    # one task: D_max 3 vs 2 adds only the pair-record table (and scratch)
    one3, one2 = ws(np.array([0, 300], dtype=np.int64), 3), ws(np.array([0, 300], dtype=np.int64), 2)
    two3, two2 = ws(off2, 3), ws(off2, 2)
    extra_one = one3 - one2
    extra_two = two3 - two2
    # several tasks add the one-task matrix and the queue on top of that
    assert extra_two - extra_one >= Sp * Sp * 8
    # the queue: one 24-byte record per sweep step (tiles x 32 rows, tiles
    # of 4 first indices x 32 rows x 128 columns) at the least
    tiles = 0
    for jb in range((S - 2) // 32 + 1):
        j0 = jb * 32
        jmax = min(j0 + 31, S - 2)
        kc0 = (j0 + 1) // 128
        ng = (jmax - 1) // 4 + 1 if jmax >= 1 else 0
        tiles += ((S + 127) // 128 - kc0) * ng
    assert extra_two - extra_one >= Sp * Sp * 8 + tiles * 32 * 24


def test_sis_host_checks_without_a_device():
    lib = B._slib()
    # workspace sizes are pure functions of the shape and reject bad shapes
    offs = np.array([0, 50, 120], dtype=np.int64)
    d = B.sisso_sis_desc(None, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 120, 2, 3, None, 0, None)
    a = lib.sisso_sis_workspace_bytes(ctypes.byref(d))
    assert a == lib.sisso_sis_workspace_bytes(ctypes.byref(d)) and a >= 120 * 3 * 8
    d.nres = 17
    assert lib.sisso_sis_workspace_bytes(ctypes.byref(d)) == 0
    assert lib.sisso_topm_workspace_bytes(1000, 10) > 0
    assert lib.sisso_topm_workspace_bytes(0, 10) == 0
    assert lib.sisso_topm_workspace_bytes(1000, 0) == 0
    assert lib.sisso_topm_workspace_bytes(1000, (1 << 20) + 1) == 0
    f = B.sisso_fit_desc(None, None, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 120, 200, 2, 3, 10, 4, 8,
                         None, 0, None)
    assert lib.sisso_fit_workspace_bytes(ctypes.byref(f)) > 0
    f.k = 11                      # k > m_sis: the first dimension has only m_sis models
    assert lib.sisso_fit_workspace_bytes(ctypes.byref(f)) == 0
    f.k, f.M = 8, 29              # M < D_max * m_sis
    assert lib.sisso_fit_workspace_bytes(ctypes.byref(f)) == 0
    # argument errors are returned before any device work
    assert lib.sisso_fc_eval(99, 1, 10, 2, 1, 1, 0.0, 1.0, None, 1, None) == B.SISSO_EINVAL
    assert lib.sisso_fc_eval(0, 1, 10, 2, 1, 1, 2.0, 1.0, None, 1, None) == B.SISSO_EINVAL
    cnt = ctypes.c_int32(0)
    assert lib.sisso_topm(None, 10, 2, 1, None, ctypes.byref(cnt), 1, 1 << 20, None) == B.SISSO_EINVAL
    assert lib.sisso_residuals(1, 1, 10, 2, 1, 1, 1, 1, 0, 1, 1, None) == B.SISSO_EINVAL
    h = ctypes.c_void_p()
    assert lib.sisso_sis_create(None, ctypes.byref(h)) == B.SISSO_EINVAL
    rc = lib.sisso_fit(ctypes.byref(f), None, None, None, None)
    assert rc == B.SISSO_EINVAL and lib.sisso_fit_last_error()
