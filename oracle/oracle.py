"""ctypes binding of the plain-C FP64 vLBM oracle (``vlbm_oracle.c``).

Test infrastructure only: see the package docstring.  Arrays are numpy
float64, C-contiguous; populations are ``[Q*Q, n_theta, n_phi]`` with
``k = Q*k_theta + k_phi`` over ascending Gauss-Hermite nodes (Q = 4: D2Q16, the
default; Q = 3: D2Q9), fields are ``[n_theta, n_phi]``.  Functions that take
populations infer Q from their count; the others take ``q``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vlbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.or_set_q.argtypes = [ctypes.c_int]
        L.or_hermite.restype = ctypes.c_double
        L.or_hermite.argtypes = [ctypes.c_int, ctypes.c_double]
        L.or_quadrature.argtypes = [_dp, _dp]
        L.or_kernels.argtypes = [_dp, _dp]
        L.or_feq_thermal.argtypes = [ctypes.c_double] * 4 + [_dp]
        L.or_collision.argtypes = [_dp, ctypes.c_double, _dp]
        L.or_force.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp]
        L.or_weno5.restype = ctypes.c_double
        L.or_weno5.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_double]
        L.or_flux.restype = ctypes.c_double
        L.or_flux.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_double]
        L.or_rhs_s.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp,
                               ctypes.c_int]
        L.or_step_s.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                _dp, ctypes.c_int64, ctypes.c_int, _dp]
        L.or_init.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.or_moments.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.or_vorticity.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.or_diagnostics.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _use_q(q):
    if lib().or_set_q(int(q)):
        raise ValueError(f"quadrature order {q} (3 or 4)")
    return int(q)


def _q_of(npop):
    q = {9: 3, 16: 4}.get(int(npop))
    if q is None:
        raise ValueError(f"{npop} populations: expected 9 (Q = 3) or 16 (Q = 4)")
    return _use_q(q)


def hermite(n: int, x: float) -> float:
    return lib().or_hermite(n, x)


def quadrature(q=4):
    """Ascending nodes v[Q] and 1-D weights w[Q] of the Gauss-Hermite rule."""
    _use_q(q)
    v = np.zeros(4)
    w = np.zeros(4)
    lib().or_quadrature(_p(v), _p(w))
    return v[:q].copy(), w[:q].copy()


def kernels(q=4):
    """K^H and K~^H (QxQ, row k, column k')."""
    _use_q(q)
    K = np.zeros(16)
    Kt = np.zeros(16)
    lib().or_kernels(_p(K), _p(Kt))
    return K[:q * q].reshape(q, q), Kt[:q * q].reshape(q, q)


def feq(rho, ut, up, T=1.0, q=4):
    _use_q(q)
    out = np.zeros(16)
    lib().or_feq_thermal(rho, ut, up, T, _p(out))
    return out[:q * q].copy()


def collision(f16, tau):
    f16 = _arr(f16)
    q = _q_of(f16.size)
    out = np.zeros(16)
    lib().or_collision(_p(np.concatenate([f16, np.zeros(16 - f16.size)])), tau, _p(out))
    return out[:q * q].copy()


def force(f16, theta, R=1.0):
    f16 = _arr(f16)
    q = _q_of(f16.size)
    out = np.zeros(16)
    lib().or_force(_p(np.concatenate([f16, np.zeros(16 - f16.size)])), theta, R, _p(out))
    return out[:q * q].copy()


def weno5(h6, f6, direction, eps=1e-6):
    h6 = _arr(h6)
    f6 = _arr(f6)
    return lib().or_weno5(_p(h6), _p(f6), int(direction), eps)


SCHEMES = {"weno5": 0, "u1": 1, "u2": 2, "u3": 3}


def flux(scheme, h6, f6, direction, eps=1e-6):
    """Interface flux of a scheme (eqs. (fluxes_U1-3), (fluxes_W5)) from the six
    points s-2 .. s+3 around s+1/2."""
    h6 = _arr(h6)
    f6 = _arr(f6)
    return lib().or_flux(SCHEMES[scheme], _p(h6), _p(f6), int(direction), eps)


def rhs(f, R=1.0, tau=1e-3, eps=1e-6, threads=1, pole_fluxes=False, scheme="weno5",
        komissarov=False):
    f = _arr(f)
    npop, nt, np_ = f.shape
    _q_of(npop)
    L = np.zeros_like(f)
    fn = np.zeros((npop, np_)) if pole_fluxes else None
    fs = np.zeros((npop, np_)) if pole_fluxes else None
    rc = lib().or_rhs_s(nt, np_, R, tau, eps, SCHEMES[scheme], int(komissarov), _p(f), _p(L),
                        _p(fn), _p(fs), threads)
    if rc:
        raise ValueError("oracle rejected the grid")
    return (L, fn, fs) if pole_fluxes else L


def step(f, nsteps, R=1.0, tau=1e-3, dt=1e-3, eps=1e-6, threads=1, budget=False,
         scheme="weno5", komissarov=False):
    """Advance ``nsteps`` SSP-RK3 steps; returns the new populations (and the
    pole-flux mass budget when ``budget``).  ``scheme``: weno5, u1, u2, u3;
    ``komissarov``: the theta derivative of eq. (Komissarov_scheme)."""
    f = _arr(f).copy()
    npop, nt, np_ = f.shape
    _q_of(npop)
    b = np.zeros(1)
    rc = lib().or_step_s(nt, np_, R, tau, dt, eps, SCHEMES[scheme], int(komissarov), _p(f),
                         int(nsteps), threads, _p(b) if budget else None)
    if rc:
        raise ValueError("oracle rejected the grid")
    return (f, float(b[0])) if budget else f


def init(rho, ut, up, T=None, q=4):
    _use_q(q)
    rho, ut, up = _arr(rho), _arr(ut), _arr(up)
    nt, np_ = rho.shape
    Ta = _arr(T) if T is not None else None
    f = np.zeros((q * q, nt, np_))
    if lib().or_init(nt, np_, _p(rho), _p(ut), _p(up), _p(Ta), _p(f)):
        raise ValueError("oracle rejected the grid")
    return f


def moments(f):
    f = _arr(f)
    npop, nt, np_ = f.shape
    _q_of(npop)
    rho = np.zeros((nt, np_))
    ut = np.zeros_like(rho)
    up = np.zeros_like(rho)
    T = np.zeros_like(rho)
    lib().or_moments(nt, np_, _p(f), _p(rho), _p(ut), _p(up), _p(T))
    return rho, ut, up, T


def vorticity(ut, up, R=1.0):
    ut, up = _arr(ut), _arr(up)
    nt, np_ = ut.shape
    om = np.zeros_like(ut)
    lib().or_vorticity(nt, np_, R, _p(ut), _p(up), _p(om))
    return om


def diagnostics(f, R=1.0):
    f = _arr(f)
    npop, nt, np_ = f.shape
    _q_of(npop)
    out = np.zeros(8)
    lib().or_diagnostics(nt, np_, R, _p(f), _p(out))
    return out


def suggest_dt(n_theta, n_phi, tau, R=1.0):
    """Stability rule for the explicit scheme: the smallest of 0.2 dth, tau and
    half the phi-CFL limit of the row next to the pole (dropped for n_phi=1)."""
    dth = np.pi / n_theta
    vmax = np.sqrt(3.0 + np.sqrt(6.0))
    dt = min(0.2 * dth, tau)
    if n_phi > 1:
        dph = 2 * np.pi / n_phi
        dt = min(dt, 0.5 * R * np.sin(dth / 2) * dph / vmax)
    return dt
