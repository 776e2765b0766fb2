"""Pins of the oracle's whole update against closed forms and exact invariants.

Sec. III.D-III.G (grid, flux-form advection, pole and periodic ghosts, SSP-RK3)
and the analytic solutions of Appendix B.  Sizes keep the CPU time of the
whole file to tens of seconds.
"""
import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads as W
from golden_io import load_sections

V, W1 = oracle.quadrature()
WK = np.outer(W1, W1).reshape(16)
THREADS = 4


def _rest(nt, nph):
    return np.broadcast_to(WK[:, None, None], (16, nt, nph)).copy()


# ------------------------------------------------------------ rest state
def test_rest_state_residual_is_fifth_order_and_phi_exact():
    # At rest the collision vanishes exactly, the phi fluxes cancel exactly and
    # the theta advection (sin theta carried in the flux) balances the inertial
    # force up to the WENO-5 truncation: max|L| falls ~32x per refinement.
    res = []
    for nt in (16, 32, 64):
        L1 = oracle.rhs(_rest(nt, 1))
        L8 = oracle.rhs(_rest(nt, 8))
        assert np.array_equal(L8, np.repeat(L1, 8, axis=2))
        res.append(np.abs(L1).max())
    assert 28 < res[0] / res[1] < 36
    assert 28 < res[1] / res[2] < 36


def test_pole_flux_at_rest_leading_order():
    # With ideal weights the theta flux through the pole interface (sin = 0)
    # is the upwind-5 reconstruction of h_j = v w sin(theta_j) over ghost rows
    # with negative sin: to leading order -|v_kt| w_k dth^5 / 60 on both poles.
    nt = 64
    dth = np.pi / nt
    _, fn, fs = oracle.rhs(_rest(nt, 2), pole_fluxes=True)
    want = -np.abs(np.repeat(V, 4)) * WK * dth ** 5 / 60
    assert np.allclose(fn[:, 0], want, rtol=2e-3)
    assert np.allclose(fs[:, 0], want, rtol=2e-3)


# ------------------------------------------------------------ ghosts / pole
def _rigid_rotation_x(nt, nph, omega):
    # u = omega x_hat x r: u_theta = -omega sin(phi), u_phi = -omega cos(th) cos(phi),
    # with the isothermal (c_s = 1) density that balances the centripetal
    # acceleration, rho = exp(omega^2 r_perp^2 / 2), r_perp^2 = y^2 + z^2.
    th, ph = W.grid(nt, nph)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    rperp2 = np.sin(TH) ** 2 * np.sin(PH) ** 2 + np.cos(TH) ** 2
    return (np.exp(omega ** 2 * rperp2 / 2), -omega * np.sin(PH),
            -omega * np.cos(TH) * np.cos(PH))


def test_rotation_through_the_poles_is_smooth_steady_state():
    # A balanced rigid rotation about the x axis crosses both poles and is a
    # steady state.  With the full velocity inversion at phi + pi its residual
    # (beyond the rest-state one) converges at fifth order; a flip of the theta
    # component alone would leave an O(omega/dth) error in the pole rows.
    # omega is small so that the O(omega^3 cot th) Hermite-truncation residual
    # of the force in the pole rows stays below the discretisation error.
    res = []
    for nt in (16, 32, 64):
        rho, ut, up = _rigid_rotation_x(nt, 2 * nt, 1e-4)
        L = oracle.rhs(oracle.init(rho, ut, up), threads=THREADS)
        L0 = oracle.rhs(_rest(nt, 2 * nt), threads=THREADS)
        res.append(np.abs(L - L0).max())
    assert res[0] / res[1] > 20 and res[1] / res[2] > 10
    assert res[2] < 1e-10


def test_phi_uniform_state_stays_bitwise_phi_uniform():
    rho, ut, up, T = W.random_state(16, 8, seed=1, du=0.02)
    # make it axisymmetric
    rho, ut, up = (np.repeat(a[:, :1], 8, axis=1) for a in (rho, ut, up))
    f = oracle.step(oracle.init(rho, ut, up), 5, tau=1e-3, dt=5e-4)
    assert np.array_equal(f, np.repeat(f[:, :, :1], 8, axis=2))
    f1 = oracle.step(oracle.init(rho[:, :1], ut[:, :1], up[:, :1]), 5, tau=1e-3, dt=5e-4)
    assert np.array_equal(f[:, :, :1], f1)


# ------------------------------------------------------------ conservation
def test_mass_budget_identity():
    # sum_k of the collision and of the force vanish per cell and the phi fluxes
    # telescope around the circle, so the discrete mass
    #   M = R^2 dth dph sum sin(th_s) sum_k f_k
    # changes only by the theta fluxes through the two pole interfaces.
    nt, nph, R = 12, 16, 1.3
    rho, ut, up, T = W.random_state(nt, nph, seed=4, du=0.05)
    f0 = oracle.init(rho, ut, up)
    th, _ = W.grid(nt, nph)
    dA = R * R * (np.pi / nt) * (2 * np.pi / nph) * np.sin(th)[None, :, None]
    f1, budget = oracle.step(f0, 3, R=R, tau=2e-3, dt=1e-3, budget=True)
    dM = (dA * f1).sum() - (dA * f0).sum()
    assert abs(budget) > 1e-12                      # the pole fluxes do not vanish
    assert abs(dM - budget) < 1e-14 * (dA * f0).sum()


def test_bgk_and_force_leave_cell_mass_untouched():
    # Per cell, L summed over k is the flux divergence alone.  On a phi-uniform
    # state the phi part is exactly zero, so sum_k L_k sin(theta) dth summed over
    # theta telescopes to the two pole fluxes.
    nt = 16
    rho, ut, up, T = W.random_state(nt, 1, seed=5, du=0.05)
    f = oracle.init(rho, ut, up)
    # tau = 1 keeps the round-off of the (vanishing) collision sum small
    L, fn, fs = oracle.rhs(f, tau=1.0, pole_fluxes=True)
    th, _ = W.grid(nt, 1)
    terms = L.sum(axis=0)[:, 0] * np.sin(th) * (np.pi / nt)
    scale = (np.abs(L).sum(axis=0)[:, 0] * np.sin(th)).sum() * (np.pi / nt)
    assert abs(terms.sum() + (fs.sum() - fn.sum())) < 1e-14 * scale


# ------------------------------------------------------------ time stepping
def test_ssp_rk3_is_third_order_in_time():
    # A non-equilibrium perturbation with zero mass and momentum relaxes at rate
    # 1/tau; at fixed grid, successive halvings of dt shrink the change of the
    # end state by 2^3.
    nt = 8
    rho, ut, up, T = W.random_state(nt, 1, seed=2, du=0.02)
    f0 = oracle.init(rho, ut, up)
    rng = np.random.default_rng(0)
    g = rng.normal(size=(16, nt, 1)) * WK[:, None, None] * 0.05
    vt, vp = np.repeat(V, 4), np.tile(V, 4)
    B = np.stack([np.ones(16), vt, vp])                # project out 1, v_th, v_ph
    for s in range(nt):
        c = np.linalg.lstsq(B.T, g[:, s, 0], rcond=None)[0]
        g[:, s, 0] -= B.T @ c
    f0 = f0 + g
    tau, T_end = 1e-3, 4e-3
    ends = [oracle.step(f0, int(round(T_end / dt)), tau=tau, dt=dt) for dt in (2.5e-4, 1.25e-4, 6.25e-5)]
    r = np.abs(ends[0] - ends[1]).max() / np.abs(ends[1] - ends[2]).max()
    assert 7.0 < r < 9.0


# ------------------------------------------------------------ closed forms
def test_sound_mode_c1_matches_closed_form_and_converges():
    # rho = 1 + 1e-3 P_2(cos th) at rest; the l = 2 density mode oscillates with
    # lambda^2 = 6, gamma = nu (lambda^2 - 1), omega^2 = 6 - gamma^2
    # (eq. (sound_damping_coeffs) with nu_v = nu).  500 steps, t = 0.5.
    tau, dt, n = 1e-3, 1e-3, 500
    errs = []
    for nt in (16, 32):
        rho, ut, up, T = W.sound_wave_p2(nt, 1)
        f = oracle.step(oracle.init(rho, ut, up), n, tau=tau, dt=dt)
        r, _, _, _ = oracle.moments(f)
        th, _ = W.grid(nt, 1)
        p2 = 0.5 * (3 * np.cos(th) ** 2 - 1)
        a = ((r[:, 0] - 1) * np.sin(th) * p2).sum() / (np.sin(th) * p2 * p2).sum()
        errs.append(abs(a - cf.density_mode_amplitude(2, tau, n * dt, 1e-3)) / 1e-3)
    assert errs[1] < 5e-6
    assert errs[0] / errs[1] > 50


@pytest.mark.slow
def test_c1_full_grid_equals_axisymmetric_run():
    # The configured C1 grid (32 x 64) run for 500 steps: phi-uniform data stay
    # bitwise uniform, so it must equal the N_phi = 1 run exactly.
    tau, dt, n = 1e-3, 1e-3, 500
    assert oracle.suggest_dt(32, 64, tau) == pytest.approx(1e-3)
    rho, ut, up, T = W.sound_wave_p2(32, 64)
    f = oracle.step(oracle.init(rho, ut, up), n, tau=tau, dt=dt, threads=THREADS)
    f1 = oracle.step(oracle.init(rho[:, :1], ut[:, :1], up[:, :1]), n, tau=tau, dt=dt)
    assert np.array_equal(f, np.repeat(f1, 64, axis=2))


def test_single_shear_mode_decays_at_kappa():
    # u_phi = V0 sin(th) G^e_1(th): one even shear mode, V(t) = V0 exp(-kappa t),
    # kappa = 2n(2n+3) nu = 10 nu (eq. (shear_kappaen)).  t = 2.
    tau, dt, T, V0 = 1e-3, 1e-3, 2.0, 1e-5
    k = cf.shear_kappa(1, "e", tau)
    prof = []
    for nt in (32, 64):
        th, _ = W.grid(nt, 1)
        G = cf.shear_G(1, "e", th)
        up = (V0 * np.sin(th) * G)[:, None]
        f = oracle.step(oracle.init(np.ones((nt, 1)), np.zeros((nt, 1)), up),
                        int(T / dt), tau=tau, dt=dt, threads=THREADS)
        _, a, b, _ = oracle.moments(f)
        ratio = cf.project_shear(b[:, 0], th, G) / cf.project_shear(up[:, 0], th, G)
        prof.append(np.abs(b[:, 0] - up[:, 0] * np.exp(-k * T)).max() / V0)
        if nt == 64:
            assert abs(ratio - np.exp(-k * T)) < 2e-5
            assert np.abs(a).max() < 1e-3 * V0          # no sound wave excited
    assert prof[0] / prof[1] > 16                       # at least fourth order


def test_rigid_rotation_mode_is_undamped():
    # The n = 0 shear mode (u_phi = Omega sin th) has kappa = 0 (Sec. IV.B).
    tau, dt, Om = 1e-3, 1e-3, 1e-5
    err = []
    for nt in (32, 64):
        th, _ = W.grid(nt, 1)
        up = (Om * np.sin(th))[:, None]
        f = oracle.step(oracle.init(np.ones((nt, 1)), np.zeros((nt, 1)), up), 1000,
                        tau=tau, dt=dt, threads=THREADS)
        _, _, b, _ = oracle.moments(f)
        err.append(np.abs(b - up).max() / Om)
    assert err[1] < 1e-5
    assert err[0] / err[1] > 24


def test_paper_shear_amplitudes_from_constant_profile():
    # eq. (shear_ampl): projections of u_phi = V0 on G^e_n; the grid projection of
    # this trigonometric-polynomial integrand is exact, so it must reproduce the
    # printed values (pins the closed forms the other tests use).
    printed = [r[0] for r in load_sections("axisymmetric_amplitudes.txt")["shear"]]
    th, _ = W.grid(64, 1)
    for n, want in enumerate(printed):
        got = cf.project_shear(np.ones(64), th, cf.shear_G(n, "e", th))
        assert got == pytest.approx(want, rel=1e-12)
        assert cf.shear_v_even_const(n) == pytest.approx(want, rel=1e-13)


def test_paper_sound_amplitudes_from_parabolic_profile():
    # Sec. IV.A: frak-u_n = int u_theta0 F^e_n for u_theta0 = U0 (pi - th) th
    printed = [r[0] for r in load_sections("axisymmetric_amplitudes.txt")["sound"]]
    th, _ = W.grid(4096, 1)
    for n, want in enumerate(printed, start=1):
        got = cf.project_sound((np.pi - th) * th, th, cf.sound_F(n, "e", th))
        assert got == pytest.approx(want, rel=1e-6)


def test_closed_form_modes_are_orthonormal_and_match_legendre():
    th = (np.arange(20000) + 0.5) * np.pi / 20000
    dth = np.pi / 20000
    for n in range(4):
        for m in range(4):
            g = np.sum(np.sin(th) ** 3 * cf.shear_G(n, "e", th) * cf.shear_G(m, "e", th)) * dth
            assert g == pytest.approx(1.0 if n == m else 0.0, abs=1e-6)
    # printed explicit forms: G^e_0 = sqrt(3)/2, G^e_2 = sqrt(165)/128 (15 + 28 cos2 + 21 cos4);
    # the printed G^e_1 prefactor sqrt(21/32) is a misprint for sqrt(21/128)
    assert np.allclose(cf.shear_G(0, "e", th), np.sqrt(3) / 2)
    assert np.allclose(cf.shear_G(1, "e", th), np.sqrt(21 / 128) * (3 + 5 * np.cos(2 * th)))
    assert np.allclose(cf.shear_G(2, "e", th),
                       np.sqrt(165) / 128 * (15 + 28 * np.cos(2 * th) + 21 * np.cos(4 * th)))
    # printed sound mode F^e_1 = sqrt(3)/2 sin^2
    assert np.allclose(cf.sound_F(1, "e", th), np.sqrt(3) / 2 * np.sin(th) ** 2)
    # F^o_1/sin th is proportional to dP_2/d th: the C1 density mode is sound mode o,1
    f = cf.sound_F(1, "o", th) / np.sin(th)
    dp2 = -3 * np.cos(th) * np.sin(th)
    c = f[100] / dp2[100]
    assert np.allclose(f, c * dp2, atol=1e-12)
    assert cf.sound_lambda2(1, "o") == 6


# ------------------------------------------------------------ diagnostics
def test_vorticity_of_rigid_rotation():
    # u_phi = Omega sin th -> omega = 2 Omega cos th (eq. for the vorticity, Sec. IV.D)
    nt, nph = 64, 8
    th, _ = W.grid(nt, nph)
    up = np.repeat((0.3 * np.sin(th))[:, None], nph, axis=1)
    om = oracle.vorticity(np.zeros_like(up), up)
    assert np.abs(om - 0.6 * np.cos(th)[:, None]).max() < 1e-5


def test_vorticity_of_a_spherical_harmonic_converges_at_fourth_order():
    # Streamfunction psi = P_3^2(cos th) cos(2 phi) with P_3^2(x) = 15 x (1 - x^2):
    # u_th = -(1/sin th) d psi/d phi, u_phi = d psi/d th (R = 1), whose vorticity
    # is the Laplacian of psi, -l (l + 1) psi = -12 psi (Sec. IV.D).  The
    # oracle's central differences (with the pole-mirrored rows) must approach
    # it at fourth order, including the rows next to the poles.
    def err(nt):
        nph = 2 * nt
        th, ph = W.grid(nt, nph)
        T, P = np.meshgrid(th, ph, indexing="ij")
        x = np.cos(T)
        p32, dp32 = 15 * x * (1 - x * x), 15 * (1 - 3 * x * x)
        psi = p32 * np.cos(2 * P)
        ut = 2 * p32 * np.sin(2 * P) / np.sin(T)
        up = -np.sin(T) * dp32 * np.cos(2 * P)
        om = oracle.vorticity(ut, up)
        return np.abs(om + 12 * psi).max() / np.abs(12 * psi).max()
    e1, e2 = err(32), err(64)
    assert e1 < 2e-3
    assert e1 / e2 > 12                                 # 16 for fourth order


def test_diagnostics_of_rest_state():
    nt, nph, R = 16, 8, 1.0
    d = oracle.diagnostics(_rest(nt, nph) * 1.2, R)
    dth = np.pi / nt
    # midpoint sum of sin over the cell centres: sum sin((s+1/2)dth) = 1/sin(dth/2)
    assert d[0] == pytest.approx(2 * np.pi * 1.2 * dth / np.sin(dth / 2), rel=1e-13)
    assert d[1] == pytest.approx(d[0], rel=1e-13)      # sum f |v|^2 / 2 = n T with T = 1
    assert abs(d[2]) < 1e-30 and abs(d[3]) < 1e-15 and d[4] == 0.0 and d[5] < 1e-15
    assert d[6] == pytest.approx(1.2) and d[7] == pytest.approx(1.2)
