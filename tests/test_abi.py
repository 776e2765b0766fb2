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
HEADERS = [os.path.join(ROOT, "include", h) for h in ("vlbm.h", "vlbm_closure.h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(vlbm_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


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
    from paper_2504_15574_amd import closure
    bound = {name for name, _, _ in B.SIGNATURES} | {name for name, _, _ in closure.SIGNATURES}
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
           B.make_params(32, 64, 1e-3, 1e-3, q=5)]
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


def test_fp32_quadrature_keeps_mass_and_momentum_identities(lib):
    # The reduced-precision kernels compute with FP32 nodes and weights moved by
    # a few ulps from the D2Q16 rule (App. A) so that the identities that make
    # BGK conserve mass and momentum hold on the FP32 values themselves.  Checked
    # here in exact rational arithmetic against the oracle's FP64 rule.
    from fractions import Fraction as Fr
    import numpy as np
    v, w, r = B.vlbm_quadrature_f32()
    v64, w1 = oracle.quadrature()
    w64 = np.outer(w1, w1).ravel()
    ulp = lambda x: np.spacing(np.float32(abs(x)))
    assert np.all(np.abs(v.astype(np.float64) - v64) <= 10 * np.array([ulp(x) for x in v64]))
    assert np.all(np.abs(w.astype(np.float64) - w64) <= 12 * np.array([ulp(x) for x in w64]))
    assert np.array_equal(v, -v[::-1])                          # symmetric nodes
    W = w.reshape(4, 4)
    assert np.array_equal(W, W.T) and np.array_equal(W, W[::-1, ::-1])
    m0 = sum(Fr(float(x)) for x in w) - 1
    m2 = sum(Fr(float(w[4 * a + b])) * Fr(float(v[a])) ** 2 for a in range(4) for b in range(4)) - 1
    assert abs(float(m0)) <= 2e-9 and float(m0) == r[0]
    assert abs(float(m2)) <= 2e-10 and float(m2) == r[1]
    # plain rounding of the FP64 rule misses the momentum identity by far more
    vr, wr = v64.astype(np.float32), w64.astype(np.float32)
    m2r = sum(Fr(float(wr[4 * a + b])) * Fr(float(vr[a])) ** 2 for a in range(4) for b in range(4)) - 1
    assert abs(float(m2r)) > 100 * abs(float(m2))
