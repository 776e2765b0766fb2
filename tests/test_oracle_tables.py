"""Pins of the oracle's velocity-space tables (Sec. III.A, III.C; Appendix A.2, A.3).

Each table is checked against something other than the oracle's own formula:
the values the paper prints, Gauss-Hermite exactness, and the exactness of the
Hermite-projected derivative on polynomials the Q=4 basis spans.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from golden_io import load_sections


def test_nodes_and_weights_match_printed_table():
    # Appendix A.2, Table "velocity_set_Q=4"
    v, w = oracle.quadrature()
    rows = load_sections("velocity_set_q4.txt")[None]
    assert np.all(np.diff(v) > 0)
    for avt, avp, wk in rows:
        for st, sp in itertools.product((-1, 1), repeat=2):
            it = int(np.argmin(np.abs(v - st * avt)))
            ip = int(np.argmin(np.abs(v - sp * avp)))
            assert abs(v[it] - st * avt) < 1e-15 and abs(v[ip] - sp * avp) < 1e-15
            assert w[it] * w[ip] == pytest.approx(wk, rel=1e-14)


def test_nodes_are_roots_of_H4():
    # Fig. "stencils": the nodes are the roots of H_4(x) = x^4 - 6x^2 + 3
    v, _ = oracle.quadrature()
    for x in v:
        assert abs(x ** 4 - 6 * x ** 2 + 3) < 1e-13
        assert abs(oracle.hermite(4, x)) < 1e-13


def test_gauss_hermite_exact_to_degree_7():
    # A Q-point Gauss rule for the weight exp(-v^2/2)/sqrt(2 pi) integrates
    # polynomials of degree <= 2Q-1 exactly: E[v^n] = (n-1)!! for even n, 0 odd.
    v, w = oracle.quadrature()
    for n in range(8):
        exact = 0.0 if n % 2 else float(np.prod(np.arange(n - 1, 0, -2))) if n else 1.0
        assert np.sum(w * v ** n) == pytest.approx(exact, abs=1e-13)
    # and misses degree 8 (E[v^8] = 105), which is what makes Q = 4 a 4-point rule
    assert abs(np.sum(w * v ** 8) - 105.0) > 1.0


def test_kernels_match_printed_matrices():
    # Appendix A.2, eqs. (Q4_Kk), (Q4_KKt)
    K, Kt = oracle.kernels()
    g = load_sections("kernels_q4.txt")
    Kp = np.array([r[0] for r in g["K"]]).reshape(4, 4)
    Ktp = np.array([r[0] for r in g["Kt"]]).reshape(4, 4)
    assert np.max(np.abs(K - Kp)) < 2e-15
    assert np.max(np.abs(Kt - Ktp)) < 5e-15


def test_kernel_identities_appendix_A3():
    # Appendix A.3: sum_k K_{k,k'} = sum_k Kt_{k,k'} = 0,
    # sum_k K_{k,k'} v_k = -1, sum_k Kt_{k,k'} v_k = -v_{k'}
    v, _ = oracle.quadrature()
    K, Kt = oracle.kernels()
    assert np.max(np.abs(K.sum(axis=0))) < 1e-14
    assert np.max(np.abs(Kt.sum(axis=0))) < 1e-14
    assert np.max(np.abs(v @ K + 1.0)) < 1e-14
    assert np.max(np.abs(v @ Kt + v)) < 1e-14


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_kernels_differentiate_spanned_polynomials_exactly(deg):
    # Eqs. (df): for f(v) = omega(v) p(v) with deg p <= 2, the projected derivative
    # is exact because d/dv[omega p] = omega (p' - v p) stays in the span of
    # H_0..H_3; on the nodes f_k = w_k p(v_k) (eq. (f_disc)), so
    #   sum_k' K_{k,k'} w_k' p(v_k') = w_k (p'(v_k) - v_k p(v_k))
    #   sum_k' Kt_{k,k'} w_k' p(v_k') = w_k d/dv[v p](v_k) - w_k v_k^2 p(v_k)
    rng = np.random.default_rng(deg)
    c = rng.normal(size=deg + 1)
    p = np.polynomial.Polynomial(c)
    v, w = oracle.quadrature()
    K, Kt = oracle.kernels()
    fk = w * p(v)
    want = w * (p.deriv()(v) - v * p(v))
    assert np.max(np.abs(K @ fk - want)) < 1e-13
    vp = np.polynomial.Polynomial([0, 1]) * p
    want_t = w * (vp.deriv()(v) - v * vp(v))
    assert np.max(np.abs(Kt @ fk - want_t)) < 1e-13


def test_hermite_polynomials_low_orders():
    # eq. (hermite_polynomials) in 1-D: H0 = 1, H1 = x, H2 = x^2 - 1, H3 = x^3 - 3x
    for x in (-1.7, 0.3, 2.2):
        assert oracle.hermite(0, x) == 1.0
        assert oracle.hermite(1, x) == x
        assert oracle.hermite(2, x) == pytest.approx(x * x - 1, abs=1e-15)
        assert oracle.hermite(3, x) == pytest.approx(x ** 3 - 3 * x, abs=1e-14)
        assert oracle.hermite(5, x) == pytest.approx(x ** 5 - 10 * x ** 3 + 15 * x, abs=1e-12)
    assert math.isclose(oracle.hermite(-1, 0.5), 0.0)
