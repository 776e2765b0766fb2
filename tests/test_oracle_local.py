"""Pins of the oracle's cell-local physics: equilibrium, BGK, inertial force.

Sec. III.B (eq. feq_Q=4), Sec. III.C / eq. (Lf) and Appendix A.3-A.4.  The
checks are moment identities that follow from the continuous kinetic theory,
not re-evaluations of the oracle's own expressions.
"""
import numpy as np
import pytest

import oracle

V, W1 = oracle.quadrature()
VT = np.repeat(V, 4)          # v_theta of population k = 4 kt + kp
VP = np.tile(V, 4)            # v_phi
WK = np.outer(W1, W1).reshape(16)


def _moms(f):
    n = f.sum()
    return n, (f * VT).sum(), (f * VP).sum()


@pytest.mark.parametrize("rho,ut,up,T", [(1.0, 0.0, 0.0, 1.0), (1.3, 0.1, -0.2, 1.0),
                                         (0.7, -0.05, 0.3, 1.0), (1.5, 0.02, 0.01, 1.2),
                                         (1.1, 0.2, 0.1, 0.9)])
def test_equilibrium_reproduces_moments_up_to_third_order(rho, ut, up, T):
    # Appendix A.4: with Q = 4 the discrete equilibrium has the moments of a
    # Maxwellian exactly up to order 3:  n, n u, rho u u + p delta,
    # rho uuu + p (u delta)_sym, with p = rho T.
    f = oracle.feq(rho, ut, up, T)
    u = np.array([ut, up])
    vv = np.stack([VT, VP])
    p = rho * T
    assert f.sum() == pytest.approx(rho, rel=1e-14)
    assert np.allclose(vv @ f, rho * u, rtol=0, atol=1e-14)
    M2 = np.einsum("ak,bk,k->ab", vv, vv, f)
    assert np.allclose(M2, rho * np.outer(u, u) + p * np.eye(2), rtol=0, atol=1e-14)
    M3 = np.einsum("ak,bk,ck,k->abc", vv, vv, vv, f)
    I = np.eye(2)
    want = rho * np.einsum("a,b,c->abc", u, u, u) + p * (
        np.einsum("a,bc->abc", u, I) + np.einsum("b,ca->abc", u, I) + np.einsum("c,ab->abc", u, I))
    assert np.allclose(M3, want, rtol=0, atol=1e-14)
    # temperature as the second central moment: sum f |v-u|^2 = 2 n T (D = 2)
    assert (f * ((VT - ut) ** 2 + (VP - up) ** 2)).sum() == pytest.approx(2 * rho * T, rel=1e-13)


def test_equilibrium_is_truncated_maxwellian():
    # eq. (feq_disc): f^eq_k = w_k f_M(v_k)/omega(v_k); the order-3 truncation
    # misses only O(u^4) terms, so at |u| = 1e-3 the two agree to ~1e-12 w_k.
    rho, ut, up = 1.0, 1e-3, -7e-4
    f = oracle.feq(rho, ut, up)
    exact = rho * WK * np.exp(-((VT - ut) ** 2 + (VP - up) ** 2) / 2) / np.exp(-(VT ** 2 + VP ** 2) / 2)
    assert np.max(np.abs(f - exact) / WK) < 1e-11
    # and the error really is fourth order: doubling u multiplies it by ~16
    f2 = oracle.feq(rho, 2 * ut, 2 * up)
    exact2 = rho * WK * np.exp(-((VT - 2 * ut) ** 2 + (VP - 2 * up) ** 2) / 2) / np.exp(-(VT ** 2 + VP ** 2) / 2)
    r = np.max(np.abs(f2 - exact2) / WK) / np.max(np.abs(f - exact) / WK)
    assert 12 < r < 20


def test_rest_equilibrium_is_the_weights():
    assert np.allclose(oracle.feq(1.0, 0.0, 0.0), WK, rtol=0, atol=1e-16)


def test_bgk_conserves_mass_and_momentum_per_cell():
    # Sec. III.B: 1 and v are collision invariants of BGK with this f^eq
    rng = np.random.default_rng(3)
    for _ in range(20):
        f = WK * (1 + 0.3 * rng.uniform(-1, 1, 16))
        C = oracle.collision(f, 2e-3)
        scale = np.abs(C).max()
        assert abs(C.sum()) < 1e-14 * scale * 16
        assert abs((C * VT).sum()) < 1e-14 * scale * 16
        assert abs((C * VP).sum()) < 1e-14 * scale * 16
        # and relaxes toward the equilibrium of the same moments
        n, jt, jp = _moms(f)
        feq = oracle.feq(n, jt / n, jp / n)
        assert np.allclose(C, -(f - feq) / 2e-3, rtol=1e-12, atol=0)


@pytest.mark.parametrize("theta", [0.1, 0.7, 1.5, 2.9])
def test_force_moments_on_random_populations(theta):
    # The inertial term of eq. (Boltzmann_eq_sphere) integrated against 1, v and
    # |v|^2 (Appendix A.3, eqs. (quad_cons_df_moments)):
    #   sum G = 0,
    #   sum v_th G =  (cot/R) sum f v_ph^2,
    #   sum v_ph G = -(cot/R) sum f v_th v_ph,
    #   sum |v|^2 G = 0  (no work done by the geometric force).
    rng = np.random.default_rng(int(theta * 10))
    R = 1.7
    cot = np.cos(theta) / np.sin(theta) / R
    for _ in range(10):
        f = WK * (1 + 0.5 * rng.uniform(-1, 1, 16))
        G = oracle.force(f, theta, R)
        s = np.abs(G).max() + 1e-300
        assert abs(G.sum()) < 1e-14 * s * 16
        assert (G * VT).sum() == pytest.approx(cot * (f * VP ** 2).sum(), rel=1e-13, abs=1e-16)
        assert (G * VP).sum() == pytest.approx(-cot * (f * VT * VP).sum(), rel=1e-13, abs=1e-16)
        assert abs((G * (VT ** 2 + VP ** 2)).sum()) < 1e-13 * s * 16


def test_force_on_equilibrium_gives_centrifugal_and_coriolis_terms():
    # For f = f^eq(rho, u): momentum source = (cot/R) (rho u_ph^2 + p, -rho u_th u_ph),
    # the geometric terms of eqs. (sph_Dudt) / (sph_dtau) with p = rho.
    rho, ut, up, th = 1.2, 0.05, -0.08, 0.9
    f = oracle.feq(rho, ut, up)
    G = oracle.force(f, th, 1.0)
    cot = np.cos(th) / np.sin(th)
    assert (G * VT).sum() == pytest.approx(cot * (rho * up * up + rho), rel=1e-13)
    assert (G * VP).sum() == pytest.approx(-cot * rho * ut * up, rel=1e-12)


def test_force_vanishes_at_equator():
    f = WK * 1.1
    assert np.max(np.abs(oracle.force(f, np.pi / 2, 1.0))) < 1e-15
