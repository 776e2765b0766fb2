"""Pins of the oracle's upwind fluxes (U1, U2, U3) and of the Komissarov form of
the theta derivative (Sec. III.E, eqs. (fluxes_U1-3), (Komissarov_scheme),
(Komissarov_sin_cos)).  CPU only."""
import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads as W

V, W1 = oracle.quadrature()
WK = np.outer(W1, W1).reshape(16)
ORDER = {"u1": 1, "u2": 2, "u3": 3, "weno5": 5}


def _rest(nt, nph):
    return np.broadcast_to(WK[:, None, None], (16, nt, nph)).copy()


@pytest.mark.parametrize("scheme", ["u1", "u2", "u3"])
def test_flux_difference_is_exact_up_to_the_scheme_order(scheme):
    # Conservative finite differences: (F_{s+1/2} - F_{s-1/2}) / dx equals h'(x_s)
    # exactly for polynomials of degree <= p and not for degree p + 1, for both
    # upwind directions (the negative one reads the mirrored stencil).
    p = ORDER[scheme]
    x = np.arange(-3, 5, dtype=float)        # points s-3 .. s+4 around s = 0
    for direction in (1, -1):
        for deg in range(0, p + 2):
            h = x ** deg
            Fp = oracle.flux(scheme, h[1:7], np.zeros(6), direction)   # interface s+1/2
            Fm = oracle.flux(scheme, h[0:6], np.zeros(6), direction)   # interface s-1/2
            exact = deg * 0.0 ** (deg - 1) if deg > 0 else 0.0
            if deg <= p:
                assert abs((Fp - Fm) - exact) < 1e-12, (direction, deg)
            else:
                assert abs((Fp - Fm) - exact) > 1e-3, (direction, deg)


def test_upwind_fluxes_read_only_the_upwind_side():
    # U1 takes the upwind cell value: h_s for v > 0, h_{s+1} for v < 0
    h = np.array([1.0, 2.0, 3.0, 5.0, 8.0, 13.0])
    assert oracle.flux("u1", h, np.zeros(6), 1) == 3.0
    assert oracle.flux("u1", h, np.zeros(6), -1) == 5.0
    assert oracle.flux("u2", h, np.zeros(6), 1) == 1.5 * 3.0 - 0.5 * 2.0
    assert oracle.flux("u3", h, np.zeros(6), -1) == pytest.approx(3.0 / 3 + 5.0 * 5 / 6 - 8.0 / 6)


@pytest.mark.parametrize("scheme,ratio", [("u1", 2.0), ("u2", 2.0), ("u3", 8.0)])
def test_rest_state_residual_order_standard_form(scheme, ratio):
    # Standard form: the rest-state residual falls with the flux order at the
    # interior rows, but in the pole rows the division by R sin(theta_s) ~ dth/2
    # costs one order.  U2 is first order there: its O(dth^3) interface error
    # becomes O(dth) (why the paper favours the Komissarov form for low orders).
    res = [np.abs(oracle.rhs(_rest(nt, 1), scheme=scheme)).max() for nt in (16, 32, 64)]
    for a, b in zip(res, res[1:]):
        assert 0.85 * ratio < a / b < 1.15 * ratio


@pytest.mark.parametrize("scheme", ["u1", "u2", "u3", "weno5"])
def test_komissarov_form_is_exactly_well_balanced(scheme):
    # Any consistent flux reconstructs the constant v w rho0 exactly, and
    # (sin th_{s+1/2} - sin th_{s-1/2}) / (cos th_{s-1/2} - cos th_{s+1/2}) =
    # cot th_s exactly, which the inertial force on w rho0 cancels: the rest
    # state is steady to rounding, at every resolution.
    for nt in (8, 16, 64):
        L = oracle.rhs(_rest(nt, 4), scheme=scheme, komissarov=True)
        assert np.abs(L).max() < 1e-12


def test_komissarov_pole_fluxes_vanish_and_mass_is_conserved():
    # sin(th) = 0 at both pole interfaces: no flux leaves through the poles, and
    # the band-area-weighted mass sum_s (cos th_{s-1/2} - cos th_{s+1/2}) sum f
    # is conserved to rounding by every step.
    nt, nph = 12, 16
    rho, ut, up, T = W.random_state(nt, nph, seed=21, du=0.05, dT=0.05, smooth=False)
    f0 = oracle.init(rho, ut, up, T)
    _, fn, fs = oracle.rhs(f0, pole_fluxes=True, scheme="u3", komissarov=True)
    assert np.all(fn == 0.0) and np.all(fs == 0.0)
    dth = np.pi / nt
    band = np.cos(np.arange(nt) * dth) - np.cos((np.arange(nt) + 1) * dth)
    mass = lambda f: (band[:, None] * f.sum(axis=0)).sum()
    f = oracle.step(f0, 20, tau=2e-3, dt=5e-4, scheme="u3", komissarov=True)
    assert abs(mass(f) - mass(f0)) < 1e-14 * mass(f0)


@pytest.mark.parametrize("scheme", ["u2", "weno5"])
def test_komissarov_sound_mode_converges_at_second_order(scheme):
    # The l = 2 density mode of C1 against its closed form: with the Komissarov
    # form the error falls ~4x per refinement whatever the flux order (the paper
    # states the form cannot exceed second order).
    tau, dt, n = 1e-3, 1e-3, 500
    errs = []
    for nt in (16, 32, 64):
        rho, ut, up, T = W.sound_wave_p2(nt, 1)
        f = oracle.step(oracle.init(rho, ut, up), n, tau=tau, dt=dt, scheme=scheme,
                        komissarov=True)
        r = oracle.moments(f)[0]
        th, _ = W.grid(nt, 1)
        p2 = 0.5 * (3 * np.cos(th) ** 2 - 1)
        a = ((r[:, 0] - 1) * np.sin(th) * p2).sum() / (np.sin(th) * p2 * p2).sum()
        errs.append(abs(a - cf.density_mode_amplitude(2, tau, n * dt, 1e-3)) / 1e-3)
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5


def test_weno5_default_is_unchanged():
    # or_rhs / or_step without a scheme are the WENO-5 standard form
    rho, ut, up, T = W.random_state(10, 12, seed=22, du=0.05)
    f = oracle.init(rho, ut, up, T)
    assert np.array_equal(oracle.rhs(f), oracle.rhs(f, scheme="weno5", komissarov=False))
