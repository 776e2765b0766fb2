"""The paper's axisymmetric sound- and shear-wave benchmarks run on the GPU path.

Sec. IV.A: u_theta(0) = U0 (pi - theta) theta, rho = 1, u_phi = 0; the even
sound modes U^e_n(t) = int u_theta F^e_n dtheta follow eq. (sound_amplitudes)
with the printed amplitudes frak-u_n.  Sec. IV.B: u_phi(0) = V0, rho = 1,
u_theta = 0; the even shear modes V^e_n(t) = int sin^2 theta u_phi G^e_n dtheta
decay as v^e_n exp(-kappa^e_n t), eq. (shear_kappaen), with the printed v^e_n.
Both are run with N_phi = 1 (the flows are axisymmetric) at several N_theta as
one batched ensemble, sampled at even intervals, and compared with the closed
forms through the time-integrated relative error of eq. (l2_err).  The
projections are midpoint sums over the cell centres (eq. (rot_UV_aux) at
N_phi = 1).
"""
from __future__ import annotations

import numpy as np

import closed_forms as cf
from golden_io import load_sections
import workloads as W

AMPL = load_sections("axisymmetric_amplitudes.txt")


def closed_form(kind: str, n: int, nu: float, t, amp: float):
    """U^e_n(t) (sound, n >= 1) or V^e_n(t) (shear, n >= 0) for the paper's
    initial profiles of amplitude `amp`."""
    t = np.asarray(t, dtype=float)
    if kind == "sound":
        frak = AMPL["sound"][n - 1][0] * amp
        return cf.sound_amplitude(frak, cf.sound_lambda2(n, "e"), nu, t)
    v = AMPL["shear"][n][0] * amp
    return v * np.exp(-cf.shear_kappa(n, "e", nu) * t)


def _initial(kind, nt, amp):
    return W.sound_wave_parabolic(nt, 1, amp) if kind == "sound" else W.shear_wave_const(nt, 1, amp)


def _project(kind, nt, ut, up, modes):
    th, _ = W.grid(nt, 1)
    if kind == "sound":
        return [cf.project_sound(ut[:, 0], th, cf.sound_F(n, "e", th)) for n in modes]
    return [cf.project_shear(up[:, 0], th, cf.shear_G(n, "e", th)) for n in modes]


def amplitude_series(kind, n_thetas, tau, dt, t_end, samples, modes, amp=1e-5,
                     scheme="weno5", komissarov=False):
    """Run the benchmark at every N_theta in one ensemble (FP64 storage) and
    return (times, {N_theta: amplitudes[len(times), len(modes)]})."""
    from paper_2504_15574_amd import Ensemble, Solver
    steps_total = int(round(t_end / dt))
    per = steps_total // samples
    assert per * samples == steps_total, "t_end / dt must split into the samples"
    sols = []
    for nt in n_thetas:
        s = Solver(nt, 1, tau, dt, storage="f64", scheme=scheme, komissarov=komissarov)
        s.init_fields(*_initial(kind, nt, amp))
        sols.append(s)
    ens = Ensemble(sols)
    amps = {nt: [] for nt in n_thetas}

    def sample():
        for nt, s in zip(n_thetas, sols):
            _, ut, up = s.moments(with_T=False)
            amps[nt].append(_project(kind, nt, ut, up, modes))

    sample()
    ens.capture(per)
    for _ in range(samples):
        ens.replay()
        sample()
    ens.release()
    for s in sols:
        s.close()
    times = np.arange(samples + 1) * per * dt
    return times, {nt: np.array(a) for nt, a in amps.items()}


def l2_errors(kind, times, amps, modes, nu, amp=1e-5):
    """eq. (l2_err) per mode: sqrt(int |U_sim - U_th|^2 dt / int |U_th|^2 dt)
    over the sampled interval (trapezoidal rule)."""
    out = {}
    for nt, a in amps.items():
        row = []
        for j, n in enumerate(modes):
            th = closed_form(kind, n, nu, times, amp)
            num = np.trapezoid((a[:, j] - th) ** 2, times)
            den = np.trapezoid(th ** 2, times)
            row.append(float(np.sqrt(num / den)))
        out[nt] = row
    return out


def orders(errs, n_thetas):
    """Observed orders log2(e_N / e_2N) between consecutive resolutions."""
    e = np.array([errs[nt] for nt in n_thetas])
    return np.log(e[:-1] / e[1:]) / np.log(np.array(n_thetas[1:]) / np.array(n_thetas[:-1]))[:, None]
