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


# the largest grids whose population buffer (Q^2 planes) stays below 4 GiB,
# the reach of the kernels' 32-bit buffer offsets, per storage format
MAX_GRIDS = {"f64": (4095, 8192), "f32": (8191, 8192), "f16": (16383, 8192)}


@pytest.mark.parametrize("storage", sorted(MAX_GRIDS))
def test_largest_grid_is_accepted_and_one_more_row_is_not(lib, storage):
    nt, nph = MAX_GRIDS[storage]
    b = {"f64": 8, "f32": 4, "f16": 2}[storage]
    assert 16 * nt * nph * b < 2 ** 32 <= 16 * (nt + 1) * nph * b
    assert B.vlbm_workspace_bytes(B.make_params(nt, nph, 1e-5, 1e-7, storage)) > 0
    bad = B.make_params(nt + 1, nph, 1e-5, 1e-7, storage)
    assert B.vlbm_workspace_bytes(bad) == 0
    out = ctypes.c_void_p()
    st = lib.vlbm_create(ctypes.byref(bad), None, ctypes.c_void_p(256), 1 << 40, ctypes.byref(out))
    assert st == 2 and b"4 GiB" in lib.vlbm_last_error()


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
    # a few ulps from the D2Q16 rule (App. A): sum w = 1 holds exactly on the
    # FP32 values and the fourth moments sum w v^4 = 3, sum w vt^2 vp^2 = 1
    # nearly so; sum w v^2 - 1 is left to the equilibrium's coefficients.
    # Checked here in exact rational arithmetic against the oracle's FP64 rule.
    from fractions import Fraction as Fr
    import numpy as np
    v, w, r = B.vlbm_quadrature_f32()
    v64, w1 = oracle.quadrature()
    w64 = np.outer(w1, w1).ravel()
    ulp = lambda x: np.spacing(np.float32(abs(x)))
    assert np.all(np.abs(v.astype(np.float64) - v64) <= 10 * np.array([ulp(x) for x in v64]))
    assert np.all(np.abs(w.astype(np.float64) - w64) <= 42 * np.array([ulp(x) for x in w64]))
    assert np.array_equal(v, -v[::-1])                          # symmetric nodes
    W = w.reshape(4, 4)
    assert np.array_equal(W, W.T) and np.array_equal(W, W[::-1, ::-1])

    def moments(v, w):
        F = [[Fr(float(w[4 * a + b])), Fr(float(v[a])), Fr(float(v[b]))] for a in range(4) for b in range(4)]
        s0 = sum(x for x, _, _ in F)
        s2 = sum(x * p * p for x, p, _ in F)
        s4 = sum(x * p ** 4 for x, p, _ in F)
        s22 = sum(x * p * p * q * q for x, p, q in F)
        return s0, s2, s4, s22
    s0, s2, s4, s22 = moments(v, w)
    assert s0 == 1 and r[0] == 0.0
    assert float(s2 - 1) == r[1] and abs(r[1]) < 1e-6
    assert abs(float(s4 - 3)) <= 5e-8 and abs(float(s4 - 3) - r[2]) <= 1e-15
    assert abs(float(s22 - 1)) <= 5e-8 and abs(float(s22 - 1) - r[3]) <= 1e-15
    # plain rounding of the FP64 rule misses the fourth moment by far more
    _, _, s4r, _ = moments(v64.astype(np.float32), w64.astype(np.float32))
    assert abs(float(s4r - 3)) > 5 * abs(float(s4 - 3))
    # with P(xi) = xi/S2 + (xi^2 - S2 u^2)/2 + xi (xi^2 - g u^2)/6, g = (S4 + 3
    # S22) / (2 S2), the equilibrium's mass and momentum on this rule are exact
    # up to the anisotropy (S4 - 3 S22) u^3 / 12, for any u
    g = (s4 + 3 * s22) / (2 * s2)
    rng = np.random.default_rng(5)
    for _ in range(4):
        ut, up = (Fr(float(x)) for x in rng.normal(0, 0.1, 2))
        u2 = ut * ut + up * up
        mass = mt = 0
        for a in range(4):
            for b in range(4):
                wk, vt, vp = Fr(float(w[4 * a + b])), Fr(float(v[a])), Fr(float(v[b]))
                xi = vt * ut + vp * up
                f = wk * (1 + xi / s2 + (xi * xi - s2 * u2) / 2 + xi * (xi * xi - g * u2) / 6)
                mass += f
                mt += vt * f
        assert mass == 1
        bound = abs(float(s4 - 3 * s22)) * abs(float(ut)) * float(u2) / 12 * 1.01
        assert abs(float(mt - ut)) <= bound + 1e-30


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU; asked for more it says so and fails
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one MI355X" in (r.stdout + r.stderr) and "not supported" in (r.stdout + r.stderr)
