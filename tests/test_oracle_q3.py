"""Pins of the oracle's Q = 3 (D2Q9) model: App. A.1 (velocity set, weights,
kernels, eq. (feq_Q=3)) and the whole update against the same closed forms as
Q = 4.  CPU only."""
import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads as W
from golden_io import load_sections

V, W1 = oracle.quadrature(3)
WK = np.outer(W1, W1).reshape(9)


def test_velocity_set_matches_printed_table():
    rows = load_sections("velocity_set_q3.txt")[None]
    assert np.allclose(V, [-np.sqrt(3), 0, np.sqrt(3)], atol=1e-15)
    for at, ap, w in rows:
        for kt in range(3):
            for kp in range(3):
                if (np.isclose(abs(V[kt]), at) and np.isclose(abs(V[kp]), ap)) or \
                   (np.isclose(abs(V[kt]), ap) and np.isclose(abs(V[kp]), at)):
                    assert WK[3 * kt + kp] == pytest.approx(w, rel=1e-14)
    assert WK.sum() == pytest.approx(1.0, rel=1e-15)
    # nodes are the roots of H_3 and the rule integrates degree <= 5 exactly
    assert np.allclose([oracle.hermite(3, v) for v in V], 0, atol=1e-14)
    for p, m in [(0, 1), (2, 1), (4, 3)]:
        assert (W1 * V ** p).sum() == pytest.approx(m, rel=1e-14)


def test_kernels_match_printed_matrices():
    K, Kt = oracle.kernels(3)
    g = load_sections("kernels_q3.txt")
    assert np.allclose(K.reshape(-1), np.array(g["K"]).reshape(-1), atol=1e-14)
    assert np.allclose(Kt.reshape(-1), np.array(g["Kt"]).reshape(-1), atol=1e-14)


def test_equilibrium_moments_to_second_order():
    for rho, ut, up in [(1.1, 0.05, -0.03), (0.9, -0.2, 0.1)]:
        f = oracle.feq(rho, ut, up, q=3)
        vt, vp = np.repeat(V, 3), np.tile(V, 3)
        assert f.sum() == pytest.approx(rho, rel=1e-14)
        assert (f * vt).sum() == pytest.approx(rho * ut, rel=1e-13)
        assert (f * vp).sum() == pytest.approx(rho * up, rel=1e-13)
        assert (f * vt * vt).sum() == pytest.approx(rho * (ut * ut + 1), rel=1e-13)
        assert (f * vt * vp).sum() == pytest.approx(rho * ut * up, rel=1e-12, abs=1e-15)


def test_force_moment_identities():
    rng = np.random.default_rng(1)
    f = rng.random(9)
    th = 0.7
    G = oracle.force(f, th)
    vt, vp = np.repeat(V, 3), np.tile(V, 3)
    cot = np.cos(th) / np.sin(th)
    assert abs(G.sum()) < 1e-14
    assert (vt * G).sum() == pytest.approx(cot * (f * vp * vp).sum(), rel=1e-13)
    assert (vp * G).sum() == pytest.approx(-cot * (f * vt * vp).sum(), rel=1e-13)


def test_rest_state_fifth_order_and_komissarov_exact():
    res = [np.abs(oracle.rhs(np.broadcast_to(WK[:, None, None], (9, nt, 1)).copy())).max()
           for nt in (16, 32, 64)]
    assert 28 < res[0] / res[1] < 36 and 28 < res[1] / res[2] < 36
    for nt in (16, 64):
        L = oracle.rhs(np.broadcast_to(WK[:, None, None], (9, nt, 2)).copy(), komissarov=True)
        assert np.abs(L).max() < 1e-12


def test_sound_and_shear_modes_match_closed_forms():
    tau, dt, n = 1e-3, 1e-3, 500
    errs = []
    for nt in (16, 32):
        rho, ut, up, T = W.sound_wave_p2(nt, 1)
        f = oracle.step(oracle.init(rho, ut, up, q=3), n, tau=tau, dt=dt)
        r = oracle.moments(f)[0]
        th, _ = W.grid(nt, 1)
        p2 = 0.5 * (3 * np.cos(th) ** 2 - 1)
        a = ((r[:, 0] - 1) * np.sin(th) * p2).sum() / (np.sin(th) * p2 * p2).sum()
        errs.append(abs(a - cf.density_mode_amplitude(2, tau, n * dt, 1e-3)) / 1e-3)
    assert errs[1] < 1e-5 and errs[0] / errs[1] > 20
    # one even shear mode decays at kappa = 10 nu (t = 2)
    V0, Tend = 1e-5, 2.0
    nt = 64
    th, _ = W.grid(nt, 1)
    G = cf.shear_G(1, "e", th)
    up = (V0 * np.sin(th) * G)[:, None]
    f = oracle.step(oracle.init(np.ones((nt, 1)), np.zeros((nt, 1)), up, q=3), int(Tend / dt),
                    tau=tau, dt=dt, threads=4)
    _, a, b, _ = oracle.moments(f)
    ratio = cf.project_shear(b[:, 0], th, G) / cf.project_shear(up[:, 0], th, G)
    assert abs(ratio - np.exp(-cf.shear_kappa(1, "e", tau) * Tend)) < 2e-6


def test_pole_mirror_inverts_both_components():
    # Population k = 3 kt + kp mirrors to 8 - k = (2 - kt, 2 - kp): v -> -v
    for k in range(9):
        kt, kp = divmod(k, 3)
        assert V[2 - kt] == -V[kt] and V[2 - kp] == -V[kp]
