"""The C ABI library loads, exports what include/sorsvd.h declares, and rejects bad
arguments on the host before anything is launched (CPU only: no compute calls)."""
import ctypes

import pytest

import paper_1804_00462_amd as P
from paper_1804_00462_amd import _lib

EINVAL, EWORKSPACE, EUNSUPPORTED = -1, -2, -7


@pytest.fixture(scope="module")
def clib():
    return P.load()


def test_exports_every_declared_symbol(clib):
    names = _lib.header_symbols()
    assert "sorsvd" in names and "sorsvd_workspace_bytes" in names
    for name in names:
        assert hasattr(clib, name), name
    assert set(names) == set(_lib._SIGS)  # the binding covers the whole header


def test_version_and_status_strings(clib):
    assert clib.sorsvd_version().startswith(b"sorsvd")
    assert clib.sorsvd_status_string(0) == b"ok"
    assert clib.sorsvd_status_string(EINVAL) == b"invalid argument"


def test_workspace_query_validates_shapes():
    assert P.workspace_bytes(1000, 800, 20, 0, P.SORSVD_F64) > 0
    assert P.workspace_bytes(800, 1000, 20, 2, P.SORSVD_F32) > 0
    assert P.workspace_bytes(10, 8, 0, 0, P.SORSVD_F64) == 0       # k < 1
    assert P.workspace_bytes(10, 8, 9, 0, P.SORSVD_F64) == 0       # k > min(m, n)
    assert P.workspace_bytes(10, 8, 3, -1, P.SORSVD_F64) == 0      # q < 0
    assert P.workspace_bytes(10, 8, 4, 0, P.SORSVD_F64, l=3) == 0  # l < k
    assert P.workspace_bytes(10, 8, 3, 0, 9) == 0                   # unknown dtype
    # workspace grows with the sketch width
    assert P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_F32) > P.workspace_bytes(5000, 4000, 16, 1, P.SORSVD_F32)
    # the pass-efficient core matrix keeps the last orbit product (n x LP FP64)
    assert (P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_F32, pass_efficient=1)
            == P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_F32) + 4000 * 64 * 8)
    # 16-bit A: the same, and with refinement the partial sums of the 2 LP-column
    # orbit product (without a device the split is the device-independent one)
    assert (P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_BF16, pass_efficient=1)
            == P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_BF16) + 4000 * 64 * 8)
    assert (P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_BF16, pass_efficient=1, refine=1)
            >= P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_BF16, refine=1) + 4000 * 64 * 8)


def test_fp16_workspace_and_unsupported_combinations(clib):
    # FP16 A shares the 16-bit plan and adds the 256-byte operand scale record
    assert (P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_F16, refine=1)
            == P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_BF16, refine=1) + 256)
    assert (P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_F16, pass_efficient=1, refine=1)
            == P.workspace_bytes(5000, 4000, 64, 1, P.SORSVD_BF16, pass_efficient=1, refine=1) + 256)

    def ws(t, col_exp):  # col_exp is only checked for null on the host
        o = _lib.Opts(col_exp=col_exp)
        return clib.sorsvd_workspace_bytes(3000, 2000, 32, 1, t, ctypes.byref(o))
    assert ws(P.SORSVD_F16, 64) == ws(P.SORSVD_F16, None) > 0
    for t in (P.SORSVD_F64, P.SORSVD_F32, P.SORSVD_BF16, P.SORSVD_DIAG):
        assert ws(t, 64) == 0  # column exponents are an FP16 option
    # no (k, q) predictor and no probe for FP16 A
    assert clib.sorsvd_probe_workspace_bytes(3000, 2000, P.SORSVD_F16) == 0
    assert clib.sorsvd_auto_workspace_bytes(3000, 2000, P.SORSVD_F16) == 0
    assert clib.sorsvd_step_workspace_bytes(3000, 2000, 32, P.SORSVD_F16) > 0


def test_pack_f16_rejects_bad_arguments_before_launch(clib):
    vp = ctypes.c_void_p
    assert clib.sorsvd_pack_f16(vp(1), 100, P.SORSVD_F64, 50, 101, vp(1), 101, vp(1), None) == EINVAL  # lda < n
    assert clib.sorsvd_pack_f16(vp(1), 101, P.SORSVD_F64, 50, 101, vp(1), 100, vp(1), None) == EINVAL  # ldo < n
    assert clib.sorsvd_pack_f16(vp(0), 101, P.SORSVD_F32, 50, 101, vp(1), 101, vp(1), None) == EINVAL  # null A
    assert clib.sorsvd_pack_f16(vp(1), 101, P.SORSVD_F32, 50, 101, vp(1), 101, vp(0), None) == EINVAL  # null e
    assert clib.sorsvd_pack_f16(vp(1), 101, P.SORSVD_BF16, 50, 101, vp(1), 101, vp(1), None) == EUNSUPPORTED
    assert clib.sorsvd_pack_f16(vp(0), 0, P.SORSVD_F64, 0, 0, vp(0), 0, vp(0), None) == 0  # empty: nothing to do


def _call(clib, A=1, lda=800, t=0, m=1000, n=800, k=20, q=0, U=1, ldu=20, S=1, V=1, ldv=20, ws=256, wsb=1 << 40,
          opts=None):
    vp = ctypes.c_void_p
    return clib.sorsvd(vp(A), lda, t, m, n, k, q, 1, vp(U), ldu, vp(S), vp(V), ldv, vp(ws), wsb, None,
                       ctypes.byref(opts) if opts is not None else None)


def test_sorsvd_rejects_bad_arguments_before_launch(clib):
    assert _call(clib, A=0) == EINVAL
    assert _call(clib, lda=799) == EINVAL
    assert _call(clib, ldu=19) == EINVAL
    assert _call(clib, ldv=19) == EINVAL
    assert _call(clib, k=0) == EINVAL
    assert _call(clib, k=801) == EINVAL
    assert _call(clib, q=-1) == EINVAL
    assert _call(clib, wsb=1024) == EWORKSPACE
    assert _call(clib, ws=257) == EINVAL           # misaligned workspace
    assert _call(clib, t=7) == EINVAL
    big = _lib.Opts(l=1100)
    assert _call(clib, m=2000, n=1500, lda=1500, k=200, ldu=200, ldv=200, opts=big) == EUNSUPPORTED  # l > 1024


def test_wide_sketches_have_a_workspace(clib):
    # widths up to 1024 (column-blocked passes, blocked QR factor and core SVD)
    for t in (P.SORSVD_F64, P.SORSVD_F32, P.SORSVD_BF16, P.SORSVD_F16):
        for l in (129, 200, 256, 300, 512, 700, 1024):
            o = _lib.Opts(l=l)
            assert clib.sorsvd_workspace_bytes(4000, 3000, min(l, 100), 1, t, ctypes.byref(o)) > 0, (t, l)
    o = _lib.Opts(l=1025)
    assert clib.sorsvd_workspace_bytes(4000, 3000, 100, 1, P.SORSVD_F64, ctypes.byref(o)) == 0


def test_step_entry_points_reject_bad_arguments(clib):
    vp = ctypes.c_void_p
    assert clib.sorsvd_step_qr(vp(1), 5, 6, vp(1), vp(1), vp(256), 1 << 40, None) == EINVAL  # l > rows
    assert clib.sorsvd_step_core_svd(vp(1), 8, 9, vp(1), vp(1), vp(1), 0, vp(256), 1 << 40, None) == EINVAL
    assert clib.sorsvd_step_sketch(vp(1), 10, 0, 20, 16, vp(1), 4, vp(1), vp(256), 16, None) == EWORKSPACE
    assert clib.sorsvd_philox_normal(1, 0, 0, -1, 3, vp(1), None) == EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError):
        _lib.load()


def _problems(specs):
    """sorsvd_problem array with placeholder (never dereferenced) device pointers."""
    arr = (_lib.Problem * len(specs))()
    for i, (m, n, k, l, q) in enumerate(specs):
        arr[i] = _lib.Problem(A=256, lda=n, m=m, n=n, k=k, l=l, q=q, reserved=0, seed=i, U=512, ldu=k,
                              S=768, V=1024, ldv=k)
    return arr


def _create(clib, specs, dtype=1, opts=None, count=None):
    h, nb = ctypes.c_void_p(), ctypes.c_size_t()
    arr = _problems(specs)
    st = clib.sorsvd_batch_create(len(specs) if count is None else count, arr, dtype,
                                  ctypes.byref(opts) if opts is not None else None, ctypes.byref(h),
                                  ctypes.byref(nb))
    return st, h, nb.value


def test_batch_plan_is_host_only_and_sized(clib):
    st, h, nb = _create(clib, [(300, 200, 10, 0, 1), (129, 517, 20, 40, 0)])
    assert st == 0 and h.value and nb > 0
    assert clib.sorsvd_batch_count(h) == 2
    cfg = (ctypes.c_int32 * 6)()
    assert clib.sorsvd_batch_get_config(h, cfg) == 0
    assert list(cfg[0::2]) == [1, 1, 1] and min(cfg[1::2]) >= 1
    # run / read_info before a workspace is bound, a too small or misaligned workspace
    assert clib.sorsvd_batch_run(h, ctypes.c_void_p(256), None) == EINVAL
    assert clib.sorsvd_batch_upload(h, ctypes.c_void_p(256), nb - 1, None) == EWORKSPACE
    assert clib.sorsvd_batch_upload(h, ctypes.c_void_p(264), nb, None) == EINVAL
    bad = (ctypes.c_int32 * 6)(3, 256, 1, 256, 1, 256)
    assert clib.sorsvd_batch_set_config(h, bad) == EINVAL
    good = (ctypes.c_int32 * 6)(2, 512, 1, 128, 2, 64)
    assert clib.sorsvd_batch_set_config(h, good) == 0
    assert clib.sorsvd_batch_get_config(h, cfg) == 0 and list(cfg) == [2, 512, 1, 128, 2, 64]
    clib.sorsvd_batch_destroy(h)
    # the workspace grows with the problems
    _, h2, nb2 = _create(clib, [(300, 200, 10, 0, 1), (129, 517, 20, 40, 0), (4000, 2000, 72, 0, 1)])
    assert nb2 > nb
    clib.sorsvd_batch_destroy(h2)
    # FP64 batches run 64-row tiles only
    _, h3, _ = _create(clib, [(300, 200, 10, 0, 1)], dtype=0)
    assert clib.sorsvd_batch_set_config(h3, good) == EINVAL
    clib.sorsvd_batch_destroy(h3)
    clib.sorsvd_batch_destroy(None)


def test_batch_create_rejects_bad_problems(clib):
    ok = (300, 200, 10, 0, 1)
    assert _create(clib, [ok], count=0)[0] == EINVAL
    assert _create(clib, [ok, (300, 200, 0, 0, 1)])[0] == EINVAL      # k < 1
    assert _create(clib, [ok, (300, 200, 201, 0, 1)])[0] == EINVAL    # k > min(m, n)
    assert _create(clib, [ok, (300, 200, 10, 9, 1)])[0] == EINVAL     # 0 < l < k
    assert _create(clib, [ok, (300, 200, 10, 201, 1)])[0] == EINVAL   # l > min(m, n)
    assert _create(clib, [ok, (300, 200, 10, 0, -1)])[0] == EINVAL    # q < 0
    assert _create(clib, [(300, 200, 10, 129, 0)])[0] == EUNSUPPORTED # padded l > 128
    assert _create(clib, [ok], dtype=2)[0] == EUNSUPPORTED            # BF16 batches
    assert _create(clib, [ok], opts=_lib.Opts(refine=1))[0] == EUNSUPPORTED
    arr = _problems([ok])
    arr[0].lda = 199
    h, nb = ctypes.c_void_p(), ctypes.c_size_t()
    assert clib.sorsvd_batch_create(1, arr, 1, None, ctypes.byref(h), ctypes.byref(nb)) == EINVAL
    arr = _problems([ok])
    arr[0].A = None
    assert clib.sorsvd_batch_create(1, arr, 1, None, ctypes.byref(h), ctypes.byref(nb)) == EINVAL


def test_batch_tuning_cache_is_read_at_create(clib, tmp_path, monkeypatch):
    specs = [(300, 200, 10, 0, 1), (129, 517, 20, 40, 0)]
    _, h, _ = _create(clib, specs)
    clib.sorsvd_batch_destroy(h)
    # key: dtype, count and the summed m n LP of the batch
    work = 300 * 200 * 16 + 129 * 517 * 48
    cache = tmp_path / "tune.txt"
    cache.write_text(f"t1_c2_w{work:.6e} 2 640 1 96 2 3200\nt1_c2_w1.000000e+00 1 1 1 1 1 1\n")
    monkeypatch.setenv("SORSVD_TUNE_CACHE", str(cache))
    _, h, _ = _create(clib, specs)
    cfg = (ctypes.c_int32 * 6)()
    clib.sorsvd_batch_get_config(h, cfg)
    assert list(cfg) == [2, 640, 1, 96, 2, 3200]
    clib.sorsvd_batch_destroy(h)
