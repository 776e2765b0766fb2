"""Initial macroscopic fields on the cell-centred latitude-longitude grid.

Every generator returns ``(rho, u_theta, u_phi, T)``, float64 arrays of shape
``[n_theta, n_phi]`` (phi fastest).  ``u_theta``/``u_phi`` are the orthonormal
(vielbein) components.  Cell centres are theta_s = (s+1/2) pi/N_theta and
phi_q = (q+1/2) 2 pi/N_phi (the 1-based grid of Sec. III.D shifted to 0-based).

Random states draw from ``numpy.random.default_rng(seed)`` in a fixed order so
that a seed names a field exactly.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grid", "rest_state", "sound_wave_p2", "sound_wave_parabolic", "shear_wave_const",
    "random_vorticity_state", "turbulence_state", "shock_state", "random_state",
    "sh_synthesis",
]


def grid(n_theta: int, n_phi: int):
    th = (np.arange(n_theta) + 0.5) * np.pi / n_theta
    ph = (np.arange(n_phi) + 0.5) * 2.0 * np.pi / n_phi
    return th, ph


def _fields(n_theta, n_phi):
    z = np.zeros((n_theta, n_phi))
    return np.ones_like(z), z.copy(), z.copy(), np.ones_like(z)


def rest_state(n_theta: int, n_phi: int, rho0: float = 1.0):
    rho, ut, up, T = _fields(n_theta, n_phi)
    return rho * rho0, ut, up, T


def sound_wave_p2(n_theta: int, n_phi: int, amp: float = 1e-3):
    """Fluid at rest with rho = 1 + amp * P_2(cos theta) (the l = 2 density mode)."""
    th, _ = grid(n_theta, n_phi)
    rho, ut, up, T = _fields(n_theta, n_phi)
    p2 = 0.5 * (3.0 * np.cos(th) ** 2 - 1.0)
    rho += amp * p2[:, None]
    return rho, ut, up, T


def sound_wave_parabolic(n_theta: int, n_phi: int, U0: float = 1e-5):
    """u_theta = U0 (pi - theta) theta, rho = 1 (the sound-wave initial state of Sec. IV.A)."""
    th, _ = grid(n_theta, n_phi)
    rho, ut, up, T = _fields(n_theta, n_phi)
    ut += (U0 * (np.pi - th) * th)[:, None]
    return rho, ut, up, T


def shear_wave_const(n_theta: int, n_phi: int, V0: float = 1e-5):
    """u_phi = V0 everywhere, rho = 1 (the shear-wave initial state of Sec. IV.B)."""
    rho, ut, up, T = _fields(n_theta, n_phi)
    up += V0
    return rho, ut, up, T


def _legendre_columns(lmax: int, m: int, th: np.ndarray):
    """Orthonormal associated Legendre functions Pbar_l^m(cos th), l = m..lmax, and
    their theta derivatives (so that Y_lm = Pbar_l^m * trig(m phi) is orthonormal on
    the unit sphere, with the sqrt(2) of real harmonics applied by the caller)."""
    x = np.cos(th)
    s = np.sin(th)
    # Pbar_m^m by the diagonal recurrence
    p = np.full_like(th, np.sqrt(1.0 / (4.0 * np.pi)))
    for mm in range(1, m + 1):
        p = -np.sqrt((2.0 * mm + 1.0) / (2.0 * mm)) * s * p
    P = np.zeros((lmax - m + 1, th.size))
    P[0] = p
    if lmax > m:
        P[1] = np.sqrt(2.0 * m + 3.0) * x * p
    for l in range(m + 2, lmax + 1):
        a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
        P[l - m] = a * (x * P[l - m - 1] - b * P[l - m - 2])
    dP = np.zeros_like(P)
    for l in range(m, lmax + 1):
        prev = P[l - m - 1] if l > m else 0.0
        c = np.sqrt((2.0 * l + 1.0) * (l * l - m * m) / (2.0 * l - 1.0)) if l > m else 0.0
        dP[l - m] = (l * x * P[l - m] - c * prev) / s
    return P, dP


def sh_synthesis(coef: dict, n_theta: int, n_phi: int, lmax: int):
    """Evaluate psi = sum a_lm Y_lm (real orthonormal harmonics) and its derivatives.

    ``coef[(l, m)]`` for m in -l..l (m < 0: sin(|m| phi), m > 0: cos(m phi)).
    Returns psi, d psi/d theta, d psi/d phi on the grid.  Each order m is
    summed over l in theta first; the phi dependence is then synthesised with
    one inverse real FFT per field (direct sums when n_phi <= 2 lmax)."""
    th, ph = grid(n_theta, n_phi)
    use_fft = n_phi > 2 * lmax
    nf = n_phi // 2 + 1
    spec = [np.zeros((n_theta, nf), complex) for _ in range(3)] if use_fft else None
    out = [np.zeros((n_theta, n_phi)) for _ in range(3)]
    dph = 2.0 * np.pi / n_phi
    for m in range(0, lmax + 1):
        P, dP = _legendre_columns(lmax, m, th)
        lc = np.arange(m, lmax + 1)
        r2 = 1.0 if m == 0 else np.sqrt(2.0)
        ac = r2 * np.array([coef.get((l, m), 0.0) for l in lc])
        as_ = r2 * np.array([coef.get((l, -m), 0.0) for l in lc]) if m > 0 else np.zeros(lc.size)
        A, B = ac @ P, as_ @ P          # psi = sum_m A_m cos(m phi) + B_m sin(m phi)
        dA, dB = ac @ dP, as_ @ dP
        if use_fft:
            # cos/sin(m phi_q) with phi_q = (q + 1/2) dph -> coefficient of e^{i m q dph}
            sh = np.exp(0.5j * m * dph)
            w = n_phi if m == 0 else 0.5 * n_phi
            spec[0][:, m] += w * (A - 1j * B) * sh
            spec[1][:, m] += w * (dA - 1j * dB) * sh
            spec[2][:, m] += w * 1j * m * (A - 1j * B) * sh
        else:
            cm, sm = np.cos(m * ph), np.sin(m * ph)
            out[0] += np.outer(A, cm) + np.outer(B, sm)
            out[1] += np.outer(dA, cm) + np.outer(dB, sm)
            out[2] += m * (np.outer(-A, sm) + np.outer(B, cm))
    if use_fft:
        out = [np.fft.irfft(sp, n=n_phi, axis=1) for sp in spec]
    return out[0], out[1], out[2]


def _velocity_from_streamfunction(dth, dph, th, R=1.0):
    # u = r_hat x grad psi: u_theta = -(1/(R sin th)) d_phi psi, u_phi = (1/R) d_theta psi
    ut = -dph / (R * np.sin(th)[:, None])
    up = dth / R
    return ut, up


def random_vorticity_state(n_theta: int, n_phi: int, seed: int = 0, lmax: int = 16,
                           amp: float = 1e-4, shear: float = 1e-3, R: float = 1.0):
    """Shear wave u_phi = shear * dP_1(cos th)/d th plus a toroidal flow whose
    vorticity is sum_{l=1..lmax} sum_m b_lm Y_lm, b_lm ~ N(0, amp^2)
    (draws in l ascending, m = -l..l order); rho = T = 1."""
    rng = np.random.default_rng(seed)
    coef = {}
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            b = rng.normal(0.0, amp)
            coef[(l, m)] = -b * R * R / (l * (l + 1.0))     # streamfunction coefficient
    th, _ = grid(n_theta, n_phi)
    _, dth, dph = sh_synthesis(coef, n_theta, n_phi, lmax)
    ut, up = _velocity_from_streamfunction(dth, dph, th, R)
    up = up + (-shear * np.sin(th))[:, None]
    rho, _, _, T = _fields(n_theta, n_phi)
    return rho, ut, up, T


def turbulence_state(n_theta: int, n_phi: int, seed: int = 0, lmax: int = 256,
                     urms: float = 0.05, slope: float = -3.0, R: float = 1.0):
    """Decaying-turbulence initial state: streamfunction sum_{l=1..lmax} a_lm Y_lm with
    a_lm ~ N(0, s_l^2), s_l^2 = 2 E(l) / (l(l+1)(2l+1)), E(l) = l^slope, rescaled to an
    area-weighted rms |u| of ``urms``; rho = T = 1."""
    rng = np.random.default_rng(seed)
    coef = {}
    for l in range(1, lmax + 1):
        sl = np.sqrt(2.0 * l ** slope / (l * (l + 1.0) * (2.0 * l + 1.0)))
        for m in range(-l, l + 1):
            coef[(l, m)] = rng.normal(0.0, sl)
    th, _ = grid(n_theta, n_phi)
    _, dth, dph = sh_synthesis(coef, n_theta, n_phi, lmax)
    ut, up = _velocity_from_streamfunction(dth, dph, th, R)
    wgt = np.sin(th)[:, None] * np.ones((1, n_phi))
    rms = np.sqrt((wgt * (ut ** 2 + up ** 2)).sum() / wgt.sum())
    ut *= urms / rms
    up *= urms / rms
    rho, _, _, T = _fields(n_theta, n_phi)
    return rho, ut, up, T


def shock_state(n_theta: int, n_phi: int, theta0: float, rho_in: float = 1.5,
                T_in: float = 1.2):
    """Axisymmetric discontinuity: rho = rho_in, T = T_in for theta < theta0, else 1; u = 0."""
    th, _ = grid(n_theta, n_phi)
    rho, ut, up, T = _fields(n_theta, n_phi)
    inside = (th < theta0)[:, None]
    rho = np.where(inside, rho_in, 1.0) * np.ones((1, n_phi))
    T = np.where(inside, T_in, 1.0) * np.ones((1, n_phi))
    return rho, ut, up, T


def random_state(n_theta: int, n_phi: int, seed: int = 0, drho: float = 0.05,
                 du: float = 0.05, dT: float = 0.0, smooth: bool = True):
    """A generic 2-D state for parity tests.  ``smooth``: a few random low-order
    Fourier modes in (theta, phi); otherwise independent uniform noise per cell
    (rough data that drive the WENO weights far from the ideal ones)."""
    rng = np.random.default_rng(seed)
    th, ph = grid(n_theta, n_phi)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    out = []
    for amp in (drho, du, du, dT):
        if smooth:
            fld = np.zeros_like(TH)
            for _ in range(4):
                a, b, c = rng.normal(size=3)
                kt, kp = rng.integers(1, 4), rng.integers(0, 3)
                fld += a * np.cos(kt * TH + b) * np.cos(kp * PH + c)
            fld *= amp / 4.0
        else:
            fld = amp * rng.uniform(-1.0, 1.0, size=TH.shape)
        out.append(fld)
    rho = 1.0 + out[0]
    ut, up = out[1], out[2]
    T = 1.0 + out[3]
    if n_phi == 1:
        ut = ut.copy()
    return rho, ut, up, T
