"""Closed-form solutions of the linearised Navier-Stokes equations on the sphere.

Written from the paper's Appendix B (axisymmetric sound and shear waves) and
used only by the tests, to pin the CPU oracle.  Units: R = 1 unless given,
c_s = 1 (isothermal, T0 = 1), nu = tau and nu_v = nu (Chapman-Enskog result of
Appendix A.4: eta = zeta = tau p).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gamma, rgamma


def jacobi(n: int, a: float, b: float, x):
    """Jacobi polynomial P_n^(a,b)(x) from the explicit series, eq. (Jacobi_series).
    1/Gamma vanishes at the poles, which makes a = -1 well defined."""
    x = np.asarray(x, dtype=float)
    pref = gamma(a + n + 1) / (math.factorial(n) * gamma(a + b + n + 1))
    tot = np.zeros_like(x)
    for m in range(n + 1):
        tot = tot + math.comb(n, m) * gamma(a + b + n + m + 1) * rgamma(a + m + 1) * ((x - 1) / 2) ** m
    return pref * tot


# ---------------------------------------------------------------- sound waves
def sound_F(n: int, parity: str, th):
    """Angular functions of the acoustic modes, eqs. (sound_Fen), (sound_Fon)."""
    c2 = np.cos(2 * th)
    if parity == "e":
        return (-1) ** n * math.sqrt(n * (4 * n - 1) / (2 * n - 1)) * jacobi(n, -1, -0.5, c2)
    return (-1) ** n * np.cos(th) * math.sqrt(n * (4 * n + 1) / (2 * n + 1)) * jacobi(n, -1, 0.5, c2)


def sound_lambda2(n: int, parity: str) -> float:
    """Eigenvalues, eq. (sound_lambda_aux)."""
    return 2 * n * (2 * n - 1) if parity == "e" else 2 * n * (2 * n + 1)


def sound_gamma_omega(lam2: float, nu: float, nu_v: float | None = None, R: float = 1.0,
                      cs: float = 1.0):
    """Damping and frequency, eq. (sound_damping_coeffs)."""
    nu_v = nu if nu_v is None else nu_v
    g = nu * lam2 / (2 * R * R) * ((lam2 - 2) / lam2 + nu_v / nu)
    w = math.sqrt(lam2 * cs * cs / (R * R) - g * g)
    return g, w


def sound_amplitude(frak_u: float, lam2: float, nu: float, t):
    """U_n(t) for an initial state with zero density gradient, eq. (sound_amplitudes)."""
    g, w = sound_gamma_omega(lam2, nu)
    t = np.asarray(t, dtype=float)
    return frak_u * np.exp(-g * t) * (np.cos(w * t) - g / w * np.sin(w * t))


def density_mode_amplitude(l: int, nu: float, t, a0: float = 1.0):
    """Amplitude of a Legendre density mode rho = 1 + a(t) P_l(cos th) started at
    rest: lambda^2 = l(l+1) and the damped-oscillator solution with a'(0) = 0
    (the continuity equation gives d rho/dt = 0 when u = 0)."""
    g, w = sound_gamma_omega(l * (l + 1.0), nu)
    t = np.asarray(t, dtype=float)
    return a0 * np.exp(-g * t) * (np.cos(w * t) + g / w * np.sin(w * t))


# ---------------------------------------------------------------- shear waves
def shear_G(n: int, parity: str, th):
    """Angular functions of the shear modes, eqs. (shear_Gen), (shear_Gon)."""
    c2 = np.cos(2 * th)
    if parity == "e":
        return math.sqrt((2 * n + 1) * (4 * n + 3) / (4 * (n + 1))) * jacobi(n, 1, -0.5, c2)
    return math.sqrt((2 * n + 3) * (4 * n + 5) / (4 * (n + 1))) * np.cos(th) * jacobi(n, 1, 0.5, c2)


def shear_kappa(n: int, parity: str, nu: float, R: float = 1.0) -> float:
    """Damping rates, eqs. (shear_kappaen), (shear_kappaon)."""
    if parity == "e":
        return nu / R ** 2 * 2 * n * (2 * n + 3)
    return 2 * nu / R ** 2 * (2 * n + 1) * (n + 2)


def shear_v_even_const(n: int) -> float:
    """v^e_n / V0 for u_phi(0) = V0: the general term printed after eq. (shear_ampl)."""
    return (math.pi * math.sqrt((2 * n + 1) * (4 * n + 3)) / (4 * (n + 1) ** 1.5)
            * (math.comb(2 * n, n) / 4 ** n) ** 2)


def toroidal_kappa(l: int, nu: float, R: float = 1.0) -> float:
    """Decay rate of a degree-l toroidal (shear) mode: nu (l-1)(l+2)/R^2, which is
    kappa^e_n at l = 2n+1 and kappa^o_n at l = 2n+2."""
    return nu * (l - 1) * (l + 2) / R ** 2


# ---------------------------------------------------------------- projections
def project_shear(up_theta, th, G):
    """V_n = int_0^pi d th sin^2 th u_phi G_n (eq. (shear_veon)), midpoint rule."""
    dth = th[1] - th[0]
    return float(np.sum(np.sin(th) ** 2 * up_theta * G) * dth)


def project_sound(ut_theta, th, F):
    """U_n = int_0^pi d th u_theta F_n (eq. (sound_uncos)), midpoint rule."""
    dth = th[1] - th[0]
    return float(np.sum(ut_theta * F) * dth)
