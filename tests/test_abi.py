"""Host-side checks of the C ABI library (no GPU needed, no compute calls).

The library must load, export every function include/vlbm.h declares, and
reject invalid parameters before touching a device.
"""
import ctypes
import os
import re

import pytest

import oracle
from paper_2504_15574_amd import vlbm as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vlbm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vlbm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2504_15574_amd import build
        build.build()
    return B.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("vlbm_create", "vlbm_init_fields", "vlbm_step", "vlbm_moments", "vlbm_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    bound = {name for name, _, _ in B.SIGNATURES}
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in bound, name


def test_params_struct_layout_matches_header():
    # uint32 + 3 int32, 5 doubles, 2 int32 (natural alignment) = 64 bytes
    assert ctypes.sizeof(B.vlbm_params) == 64


def test_invalid_parameters_are_rejected_on_the_host(lib):
    p = B.make_params(32, 64, 1e-3, 1e-3)
    assert B.vlbm_workspace_bytes(p) > 0
    bad = [B.make_params(2, 64, 1e-3, 1e-3), B.make_params(32, 63, 1e-3, 1e-3),
           B.make_params(32, 64, -1.0, 1e-3), B.make_params(32, 64, 1e-3, 0.0),
           B.make_params(32, 64, 1e-3, 1e-3, q=3)]
    for q in bad:
        assert B.vlbm_workspace_bytes(q) == 0
    out = ctypes.c_void_p()
    st = lib.vlbm_create(ctypes.byref(bad[0]), None, ctypes.c_void_p(256), 1 << 20, ctypes.byref(out))
    assert st == 1 and b"n_theta" in lib.vlbm_last_error()
    st = lib.vlbm_create(ctypes.byref(bad[4]), None, ctypes.c_void_p(256), 1 << 20, ctypes.byref(out))
    assert st == 2
    # a workspace that is too small is refused before any device call
    st = lib.vlbm_create(ctypes.byref(p), None, ctypes.c_void_p(256), 1024, ctypes.byref(out))
    assert st == 3
    st = lib.vlbm_create(ctypes.byref(p), None, ctypes.c_void_p(257), 1 << 40, ctypes.byref(out))
    assert st == 1


def test_workspace_size_scales_with_storage(lib):
    b64 = B.vlbm_workspace_bytes(B.make_params(256, 512, 1e-3, 1e-4, "f64"))
    b32 = B.vlbm_workspace_bytes(B.make_params(256, 512, 1e-3, 1e-4, "f32"))
    b16 = B.vlbm_workspace_bytes(B.make_params(256, 512, 1e-3, 1e-4, "f16"))
    n = 256 * 512
    assert b64 - b32 == 3 * 16 * n * 4
    assert b32 - b16 == 3 * 16 * n * 2


@pytest.mark.parametrize("nt,nph,tau", [(32, 64, 1e-3), (512, 1024, 5e-4), (2048, 4096, 1e-5),
                                        (64, 1, 2e-3)])
def test_suggest_dt_rule(lib, nt, nph, tau):
    p = B.make_params(nt, nph, tau, 1.0)
    assert B.vlbm_suggest_dt(p) == pytest.approx(oracle.suggest_dt(nt, nph, tau), rel=1e-14)


def test_missing_library_fails_loudly(tmp_path):
    saved = B._lib
    try:
        B._lib = None
        with pytest.raises(B.VlbmError):
            B.load(str(tmp_path / "nope.so"))
    finally:
        B._lib = saved
