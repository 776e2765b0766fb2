"""Validation tooling for the GPU vLBM (host numpy, not on the solver's path).

* ``euler_axisym``: the inviscid isothermal Euler equations for axisymmetric
  flows (App. D): U = (rho, rho u_theta), flux F = (rho u, rho (u^2 + c_s^2)),
  source (0, rho c_s^2 cot(theta) / R); the theta derivative as the difference
  of F sin(theta) at the cell interfaces over R dth sin(theta_s); interface
  fluxes by characteristic flux splitting: at each interface the Jacobian's
  left eigenvectors (at the mean state of the two cells) project the point
  fluxes of the six-point stencil, each characteristic flux is reconstructed
  by WENO-5 (eqs. (fluxes_W5)-(WENO5_sigma)) upwind of its eigenvalue
  u +- c_s, and the right eigenvectors map back; pole ghosts mirror rho and
  negate u_theta; SSP-RK3 time stepping (Sec. III.G).
* Rankine-Hugoniot relations of an axisymmetric discontinuity (Sec. IV.C,
  eqs. (Rankine-Hugoniot), (shock_gen), (RH_primary)).
* Rotated frames (App. C): coordinates, scalars and orthonormal velocity
  components of a frame rotated by alpha about the y axis, eqs. (transf),
  (transf_inv), (transf_u).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Euler solver (App. D)
def _weno5_pos(f, eps):
    """WENO-5 reconstruction at s+1/2 from f[..., 0:5] = f_{s-2..s+2} (upwind
    from the left); smoothness indicators from the same values."""
    f0, f1, f2, f3, f4 = (f[..., i] for i in range(5))
    F1 = f0 / 3 - 7 * f1 / 6 + 11 * f2 / 6
    F2 = -f1 / 6 + 5 * f2 / 6 + f3 / 3
    F3 = f2 / 3 + 5 * f3 / 6 - f4 / 6
    s1 = 13 / 12 * (f0 - 2 * f1 + f2) ** 2 + 0.25 * (f0 - 4 * f1 + 3 * f2) ** 2
    s2 = 13 / 12 * (f1 - 2 * f2 + f3) ** 2 + 0.25 * (f1 - f3) ** 2
    s3 = 13 / 12 * (f2 - 2 * f3 + f4) ** 2 + 0.25 * (3 * f2 - 4 * f3 + f4) ** 2
    a1, a2, a3 = 0.1 / (eps + s1) ** 2, 0.6 / (eps + s2) ** 2, 0.3 / (eps + s3) ** 2
    return (a1 * F1 + a2 * F2 + a3 * F3) / (a1 + a2 + a3)


def _ghosts(rho, m, ng=3):
    """Pole ghosts: rho_{-j} = rho_{j-1}, u_{-j} = -u_{j-1} (and the south pole)."""
    rg = np.concatenate([rho[:ng][::-1], rho, rho[-ng:][::-1]])
    mg = np.concatenate([-m[:ng][::-1], m, -m[-ng:][::-1]])
    return rg, mg


def euler_rhs(rho, m, R=1.0, cs=1.0, eps=1e-6):
    """dU/dt of the axisymmetric Euler equations on the cell-centred theta grid."""
    N = rho.size
    dth = np.pi / N
    th = (np.arange(N) + 0.5) * dth
    rg, mg = _ghosts(rho, m)
    ug = mg / rg
    Fr, Fm = mg, mg * ug + cs * cs * rg                 # point fluxes
    # interfaces i = 0..N between cells i-1 and i (ghost-padded index i + 2 is cell i-1)
    idx = np.arange(N + 1)[:, None] + np.arange(6)[None, :]       # stencil s-2 .. s+3
    ui = 0.5 * (ug[idx[:, 2]] + ug[idx[:, 3]])                     # mean state of the two cells
    lp, lm = ui + cs, ui - cs
    # left eigenvectors L+- = (c -+ u, +-1) / (2c): characteristic point fluxes
    Qp = ((cs - ui)[:, None] * Fr[idx] + Fm[idx]) / (2 * cs)
    Qm = ((cs + ui)[:, None] * Fr[idx] - Fm[idx]) / (2 * cs)

    def upwind(Q, lam):
        left = _weno5_pos(Q[:, 0:5], eps)
        right = _weno5_pos(Q[:, 5:0:-1], eps)          # mirror stencil s+3 .. s-1
        return np.where(lam >= 0, left, right)

    qp, qm = upwind(Qp, lp), upwind(Qm, lm)
    # right eigenvectors R+- = (1, u +- c)
    Fr_i = qp + qm
    Fm_i = lp * qp + lm * qm
    si = np.sin(np.minimum(np.arange(N + 1), N - np.arange(N + 1)) * dth)   # 0 at both poles
    div = lambda F: (F[1:] * si[1:] - F[:-1] * si[:-1]) / (R * dth * np.sin(th))
    drho = -div(Fr_i)
    dm = -div(Fm_i) + rho * cs * cs / (R * np.tan(th))
    return drho, dm


def euler_axisym(rho, u, t_end, R=1.0, cs=1.0, cfl=0.4, eps=1e-6, times=()):
    """Advance (rho, u_theta) on N cells to t_end with SSP-RK3; returns the final
    (rho, u) and the states at the requested times (dict t -> (rho, u))."""
    rho = np.asarray(rho, dtype=float).copy()
    m = rho * np.asarray(u, dtype=float)
    N = rho.size
    dth = np.pi / N
    t, out = 0.0, {}
    pending = sorted(times)
    while t < t_end - 1e-15:
        dt = cfl * R * dth / (np.abs(m / rho).max() + cs)
        stop = min([t_end] + [x for x in pending if x > t + 1e-15])
        dt = min(dt, stop - t)
        a1, b1 = euler_rhs(rho, m, R, cs, eps)
        r1, m1 = rho + dt * a1, m + dt * b1
        a2, b2 = euler_rhs(r1, m1, R, cs, eps)
        r2, m2 = 0.75 * rho + 0.25 * (r1 + dt * a2), 0.75 * m + 0.25 * (m1 + dt * b2)
        a3, b3 = euler_rhs(r2, m2, R, cs, eps)
        rho = rho / 3 + 2 / 3 * (r2 + dt * a3)
        m = m / 3 + 2 / 3 * (m2 + dt * b3)
        t += dt
        while pending and abs(t - pending[0]) < 1e-12:
            out[pending.pop(0)] = (rho.copy(), m / rho)
    return rho, m / rho, out


# ---------------------------------------------------------------------------
# Rankine-Hugoniot relations (Sec. IV.C)
def rh_primary(rho_n, rho_s, cs=1.0):
    """Primary shock into fluid at rest (u_S = 0): (u_N, shock speed R dtheta_d/dt)."""
    u_n = cs * (np.sqrt(rho_n / rho_s) - np.sqrt(rho_s / rho_n))
    return u_n, rho_n * u_n / (rho_n - rho_s)


def rh_post_shock(speed, rho_s, cs=1.0):
    """State north of a shock moving at `speed` into fluid at rest of density
    rho_S: (rho_N, u_N)."""
    return rho_s * (speed / cs) ** 2, (speed ** 2 - cs ** 2) / speed


def shock_front(theta, rho, theta_min=0.0, halo=5):
    """Polar angle of a south-moving front: the steepest descent of rho south of
    theta_min, refined to where rho crosses the mean of the values `halo` cells
    on either side (linear interpolation between cells).  Small precursors
    ahead of the front (kinetic modes that outrun a shock) do not move it."""
    theta, rho = np.asarray(theta), np.asarray(rho)
    g = np.diff(rho)
    g[theta[:-1] < theta_min] = 0.0
    i = int(np.argmin(g))
    lo, hi = max(i - halo + 1, 0), min(i + halo, rho.size - 1)
    level = 0.5 * (rho[lo] + rho[hi])
    j = lo
    while j < hi and rho[j + 1] > level:
        j += 1
    r0, r1 = rho[j], rho[j + 1]
    return theta[j] + (level - r0) / (r1 - r0) * (theta[j + 1] - theta[j])


# ---------------------------------------------------------------------------
# Rotated frames (App. C): frame ' is the original rotated by alpha about y
def to_original(th_p, ph_p, alpha):
    """(theta, phi) of the point with rotated-frame coordinates (theta', phi'),
    eq. (transf_inv)."""
    x = np.cos(alpha) * np.sin(th_p) * np.cos(ph_p) - np.sin(alpha) * np.cos(th_p)
    y = np.sin(th_p) * np.sin(ph_p)
    z = np.sin(alpha) * np.sin(th_p) * np.cos(ph_p) + np.cos(alpha) * np.cos(th_p)
    return np.arccos(np.clip(z, -1, 1)), np.arctan2(y, x) % (2 * np.pi)


def velocity_to_rotated(th, ph, th_p, ph_p, ut, up, alpha):
    """Orthonormal components (u_theta', u_phi') in the rotated frame of a
    velocity with components (u_theta, u_phi) at the same point, eq. (transf_u)."""
    c = np.cos(alpha) * np.sin(th) + np.sin(alpha) * np.cos(th) * np.cos(ph)
    d = np.sin(alpha) * np.sin(ph)
    s = np.sin(th_p)
    return (c * ut - d * up) / s, (d * ut + c * up) / s
