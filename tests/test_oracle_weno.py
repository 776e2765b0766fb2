"""Pins of the oracle's WENO-5 interface flux (Sec. III.E, eqs. fluxes_W5,
WENO5_delta, WENO5_sigma).

Checked against textbook properties of finite-difference WENO-5 rather than
against a retyped copy of the formula: the linear (ideal-weight) limit is the
fifth-order upwind flux, every candidate reproduces the primitive-based
interface value of a quadratic exactly (so any weights do), the ideal weights
reproduce quartics, and a jump switches the weights to the smooth stencil.
"""
import numpy as np
import pytest

import oracle

rng = np.random.default_rng(7)


def test_ideal_weight_limit_is_upwind5():
    # f constant -> all smoothness indicators vanish -> weights = (1, 6, 3)/10;
    # the flux becomes (2 h_{s-2} - 13 h_{s-1} + 47 h_s + 27 h_{s+1} - 3 h_{s+2})/60
    for _ in range(20):
        h = rng.normal(size=6)
        f = np.full(6, 0.37)
        want = (2 * h[0] - 13 * h[1] + 47 * h[2] + 27 * h[3] - 3 * h[4]) / 60
        assert oracle.weno5(h, f, +1) == pytest.approx(want, rel=1e-13, abs=1e-15)
        want_m = (2 * h[5] - 13 * h[4] + 47 * h[3] + 27 * h[2] - 3 * h[1]) / 60
        assert oracle.weno5(h, f, -1) == pytest.approx(want_m, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("direction", [+1, -1])
def test_quadratic_flux_exact_for_any_weights(direction):
    # For h(j) quadratic, the function H whose cell averages are h is
    # H(x) = h(x) - h''/24, and each 3-point candidate gives H(s+1/2) exactly, so
    # the WENO flux is H(s+1/2) whatever f (and hence the weights) is.
    for _ in range(20):
        a, b, c = rng.normal(size=3)
        j = np.arange(-2, 4, dtype=float)          # points s-2 .. s+3, s = 0
        h = a + b * j + c * j * j
        f = rng.normal(size=6)                      # arbitrary smoothness data
        H = a + b * 0.5 + c * 0.25 - 2 * c / 24.0
        assert oracle.weno5(h, f, direction) == pytest.approx(H, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("direction", [+1, -1])
def test_ideal_weights_differentiate_quartics_exactly(direction):
    # Fifth-order property: with ideal weights, F_{s+1/2} - F_{s-1/2} = p'(s)
    # exactly for any polynomial p of degree <= 4 sampled at the points.
    for _ in range(10):
        p = np.polynomial.Polynomial(rng.normal(size=5))
        j = np.arange(-3, 4, dtype=float)          # s-3 .. s+3 with s = 0
        h = p(j)
        f = np.ones(7)
        Fp = oracle.weno5(h[1:7], f[1:7], direction)  # interface +1/2: points -2..3
        Fm = oracle.weno5(h[0:6], f[0:6], direction)  # interface -1/2: points -3..2
        assert Fp - Fm == pytest.approx(p.deriv()(0.0), rel=1e-11, abs=1e-12)


def test_weights_finite_when_smoothness_vanishes():
    h = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    f = np.zeros(6)
    val = oracle.weno5(h, f, +1, eps=1e-6)
    assert np.isfinite(val)


def test_jump_selects_the_smooth_stencil():
    # A jump between s and s+1: only candidate 1 (points s-2..s) is smooth, its
    # weight dominates and the flux is the upwind value, not an overshoot.
    f = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
    assert abs(oracle.weno5(f, f, +1)) < 1e-6
    # mirrored: upwind from the right takes the right state
    assert oracle.weno5(f, f, -1) == pytest.approx(1.0, abs=1e-6)


def test_smoothness_indicator_uses_f_not_h():
    # The indicators are printed in terms of f: with f constant and h rough,
    # the weights stay ideal (upwind-5 value), while the same rough data used
    # as f move them away from it.
    h = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
    lin = (2 * h[0] - 13 * h[1] + 47 * h[2] + 27 * h[3] - 3 * h[4]) / 60
    assert oracle.weno5(h, np.ones(6), +1) == pytest.approx(lin, abs=1e-15)
    assert abs(oracle.weno5(h, h, +1) - lin) > 0.1
