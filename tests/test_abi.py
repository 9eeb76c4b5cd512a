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
    big = _lib.Opts(l=300)
    assert _call(clib, k=200, ldu=200, ldv=200, opts=big) == EUNSUPPORTED  # wider than this build's passes


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
