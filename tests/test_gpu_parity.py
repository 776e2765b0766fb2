"""GPU (HIP) path vs the CPU FP64 oracle, through the C ABI.

Element-by-element comparisons on seeded inputs at sizes the oracle finishes
in seconds, spanning several 15 x 16 tiles with ragged tails in theta and phi,
the axisymmetric (n_phi = 1) case and the pole rows, and at the full C2 and
benchmark grids.  FP64 storage must agree with the oracle to 1e-12 relative,
both of max |f| and of the deviation scale max |f - w rho0| (plus the
oracle's own rounding, see _assert_parity); the reduced-precision formats
report their error as a number and are held to bounds derived from their
unit round-off.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    from paper_2504_15574_amd import load
    load()


def _solver(nt, nph, tau, dt, storage="f64", **kw):
    from paper_2504_15574_amd import Solver
    return Solver(nt, nph, tau, dt, storage=storage, **kw)


V, W1 = oracle.quadrature()
WK = np.outer(W1, W1).reshape(16)


def _errs(fg, fr, rho0=1.0):
    dev = fr - WK[:, None, None] * rho0
    ad = np.abs(fg - fr).max()
    return ad / np.abs(fr).max(), ad / max(np.abs(dev).max(), 1e-300)


def _assert_parity(fg, fr, steps, rho0=1.0, what=""):
    """FP64 parity with the oracle, element by element, in two forms:
    - relative to the populations: max |f_gpu - f_oracle| <= 1e-12 max |f|;
    - relative to the flow: max |f_gpu - f_oracle| <= 1e-12 max |f - w rho0|
      plus what the oracle's own rounding accounts for.  The oracle updates f
      itself (~0.2) and rounds it at ulp(max f) several times per stage, and
      at small amplitudes and many steps those roundings add up (nearly the
      same increment added to nearly the same value every stage); the GPU
      stores f - w rho0 and rounds at that scale.  The allowance is 12 ulp(max
      f) per step (4 per stage); the cases here use 0.1 - 0.7 of it."""
    ad = np.abs(fg - fr).max()
    fmax = np.abs(fr).max()
    dev = np.abs(fr - WK[:, None, None] * rho0).max()
    allow = 12 * steps * np.spacing(fmax)
    print(f"  {what}max |diff| {ad:.2e}: {ad / fmax:.2e} of max |f|, {ad / dev:.2e} of the deviation "
          f"scale; oracle rounding allowance {allow:.2e}", flush=True)
    assert ad <= 1e-12 * fmax
    assert ad <= 1e-12 * dev + allow


def _run_both(state, nt, nph, tau, dt, n, storage="f64", R=1.0):
    rho, ut, up, T = state
    print(f"[case] {storage} {nt}x{nph} tau={tau} dt={dt} steps={n}", flush=True)
    s = _solver(nt, nph, tau, dt, storage, radius=R)
    s.init_fields(rho, ut, up, T)
    s.step(n)
    fg = s.populations()
    s.close()
    fr = oracle.step(oracle.init(rho, ut, up, T), n, R=R, tau=tau, dt=dt, threads=THREADS)
    return fg, fr


def test_init_matches_oracle_equilibrium():
    st = W.random_state(20, 34, seed=3, du=0.1, dT=0.1)
    s = _solver(20, 34, 1e-3, 1e-4)
    s.init_fields(*st)
    fg = s.populations()
    fr = oracle.init(*st)
    assert np.abs(fg - fr).max() < 1e-15
    r, a, b, T = s.moments()
    rr, ar, br, Tr = oracle.moments(fr)
    assert np.abs(r - rr).max() < 1e-14
    assert np.abs(a - ar).max() < 1e-14 and np.abs(b - br).max() < 1e-14
    assert np.abs(T - Tr).max() < 1e-13
    # the thermal initial state reproduces its own T (order-3 Hermite projection)
    assert np.abs(T - st[3]).max() < 1e-13


@pytest.mark.parametrize("nt,nph,seed,smooth", [
    (26, 50, 1, False),      # ragged in theta (26 = 15 + 11) and phi (50 = 3*16 + 2)
    (22, 192, 2, True),      # twelve phi tiles
    (37, 1, 3, False),       # axisymmetric, odd n_theta
    (8, 130, 4, False),      # one partial tile row; every row is a pole row
    (3, 2, 5, False),        # the smallest grid: every ghost row maps back into the grid
    (5, 18, 6, False),       # n_phi below TQ + 3: columns wrap with the integer modulo
    (6, 20, 7, False),       # n_phi = 20: the one-fold column wrap
    (48, 64, 8, True),       # interior tiles (halo inside the grid) beside boundary tiles
])
def test_f64_parity_random_states(nt, nph, seed, smooth):
    st = W.random_state(nt, nph, seed=seed, du=0.05, dT=0.05, smooth=smooth)
    tau = 2e-3
    dt = oracle.suggest_dt(nt, nph, tau)
    fg, fr = _run_both(st, nt, nph, tau, dt, 12)
    _assert_parity(fg, fr, 12)


def test_f64_parity_c1_sound_wave_full():
    # C1: 32 x 64, nu = tau = 1e-3, dt = 1e-3, 500 steps, rho = 1 + 1e-3 P2(cos th)
    st = W.sound_wave_p2(32, 64)
    fg, fr = _run_both(st, 32, 64, 1e-3, 1e-3, 500)
    _assert_parity(fg, fr, 500, what="C1 ")
    # phi-uniform data stay bitwise phi-uniform on the GPU too
    assert np.array_equal(fg, np.repeat(fg[:, :, :1], 64, axis=2))


def test_f64_parity_random_vorticity_2d():
    # C2-type state (shear wave + random toroidal vorticity, l <= 16) at 64 x 128
    st = W.random_vorticity_state(64, 128, seed=0, lmax=16, amp=1e-2, shear=1e-2)
    tau = 5e-4
    dt = oracle.suggest_dt(64, 128, tau)
    fg, fr = _run_both(st, 64, 128, tau, dt, 50)
    _assert_parity(fg, fr, 50, what="C2-type ")


def test_f64_radius_and_rho0():
    st = W.random_state(16, 64, seed=9, drho=0.1, du=0.05)
    rho, ut, up, T = st
    rho = rho * 1.7
    s = _solver(16, 64, 3e-3, 1e-3, "f64", radius=2.5, rho0=1.7)
    s.init_fields(rho, ut, up)
    s.step(10)
    fg = s.populations()
    s.close()
    fr = oracle.step(oracle.init(rho, ut, up), 10, R=2.5, tau=3e-3, dt=1e-3, threads=THREADS)
    _assert_parity(fg, fr, 10, rho0=1.7)


def test_stage_launch_count_and_determinism():
    st = W.random_state(24, 96, seed=5, du=0.05, smooth=False)
    outs = []
    for _ in range(2):
        s = _solver(24, 96, 2e-3, 5e-4)
        s.init_fields(*st)
        s.step(7)
        from paper_2504_15574_amd import vlbm_stage_launches
        assert vlbm_stage_launches(s.ctx) == 21
        outs.append(s.populations())
        s.close()
    assert np.array_equal(outs[0], outs[1])    # no LDS race: bitwise repeatable


def test_checkpoint_resume_continues_the_run():
    st = W.random_state(16, 64, seed=6, du=0.05)
    a = _solver(16, 64, 2e-3, 5e-4)
    a.init_fields(*st)
    a.step(20)
    straight = a.populations()
    b = _solver(16, 64, 2e-3, 5e-4)
    b.init_fields(*st)
    b.step(10)
    ck = b.populations()
    c = _solver(16, 64, 2e-3, 5e-4)
    c.set_populations(ck)
    c.step(10)
    resumed = c.populations()
    for x in (a, b, c):
        x.close()
    assert np.abs(resumed - straight).max() < 1e-15


def test_diagnostics_and_vorticity_match_oracle():
    st = W.random_vorticity_state(48, 96, seed=2, lmax=8, amp=1e-2, shear=1e-2)
    s = _solver(48, 96, 1e-3, 1e-4, radius=1.3)
    s.init_fields(*st)
    s.step(3)
    d = s.diagnostics()
    om = s.vorticity()
    f = s.populations()
    r, a, b, T = s.moments()
    s.close()
    dr = oracle.diagnostics(f, 1.3)
    assert np.allclose(d[[0, 1, 2, 3]], dr[[0, 1, 2, 3]], rtol=1e-12, atol=1e-18)
    assert d[4] == 0 and dr[4] == 0
    assert np.allclose(d[5:], dr[5:], rtol=1e-13)
    omr = oracle.vorticity(a, b, 1.3)
    assert np.abs(om - omr).max() <= 1e-12 * np.abs(omr).max()


def test_device_field_entry_points_refuse_short_tensors():
    # The kernels write n_theta x n_phi values through a device pointer, so
    # the binding refuses a tensor of another size or type before any launch.
    import torch
    from paper_2504_15574_amd import VlbmError
    from paper_2504_15574_amd.closure import vlbm_box_filter
    s = _solver(16, 32, 1e-3, 1e-4)
    s.init_fields(*W.random_state(16, 32, seed=12, du=0.05))
    good = [torch.empty(16, 32, dtype=torch.float64, device="cuda") for _ in range(3)]
    s.moments_device(*good)
    short = torch.empty(16, 31, dtype=torch.float64, device="cuda")
    for call in (lambda: s.moments_device(good[0], short, good[2]),
                 lambda: s.vorticity_device(short),
                 lambda: s.init_fields_device(short, good[1], good[2]),
                 lambda: s.correct_moments_device(good[0], good[1], short),
                 lambda: s.moments_device(good[0].float(), good[1], good[2])):
        with pytest.raises(VlbmError):
            call()
    f = torch.zeros(2 * 8 * 16, dtype=torch.float64, device="cuda")
    c = torch.zeros(2 * 4 * 8 - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(VlbmError):
        vlbm_box_filter(8, 16, 2, 2, f, f, f, c, c, c)
    torch.cuda.synchronize()
    r, a, b, _ = s.moments()
    s.close()
    assert np.array_equal(good[0].cpu().numpy(), r)


def test_unstable_run_is_detected():
    # dt = 4 tau exceeds the SSP-RK3 stability limit of the stiff BGK term
    # (|dt/tau| < 2.51 on the negative real axis): the run blows up and the
    # diagnostics report non-finite populations instead of silently continuing.
    st = W.random_state(16, 32, seed=7, du=0.05, smooth=False)
    s = _solver(16, 32, 1e-3, 4e-3)
    s.init_fields(*st)
    s.step(400)
    d = s.diagnostics(raise_unstable=False)
    from paper_2504_15574_amd import VlbmError
    with pytest.raises(VlbmError):
        s.diagnostics()
    s.close()
    assert d[4] > 0


@pytest.mark.parametrize("storage,bound", [("f32", 2e-5), ("f16", 5e-3)])
def test_reduced_precision_error_vs_oracle(storage, bound):
    # Deviation storage: the error is reported relative to the deviation scale
    # max |f - w rho0| (the part of f that carries the flow).
    st = W.random_vorticity_state(64, 128, seed=1, lmax=12, amp=2e-2, shear=2e-2)
    tau = 5e-4
    dt = oracle.suggest_dt(64, 128, tau)
    fg, fr = _run_both(st, 64, 128, tau, dt, 30, storage)
    rel, reldev = _errs(fg, fr)
    print(f"  {storage}: max rel {rel:.2e}, deviation-relative {reldev:.2e}")
    assert reldev < bound


# ---------------------------------------------------------------- full sizes
@pytest.mark.parametrize("nt,nph,tau,steps,maker", [
    (512, 1024, 5e-4, 3, "vorticity"),      # the C2 grid (shear wave + random vorticity)
    (2048, 4096, 1e-5, 1, "turbulence"),    # the benchmark grid, one full step
])
def test_f64_parity_full_size(nt, nph, tau, steps, maker):
    # Full-size parity in the launch configuration bench.py times: every cell of
    # every population is compared with the CPU oracle (OpenMP over rows).
    if maker == "vorticity":
        st = W.random_vorticity_state(nt, nph, seed=0, lmax=16, amp=1e-4, shear=1e-3)
    else:
        st = W.turbulence_state(nt, nph, seed=0, lmax=256, urms=0.05)
    dt = oracle.suggest_dt(nt, nph, tau)
    fg, fr = _run_both(st, nt, nph, tau, dt, steps)
    _assert_parity(fg, fr, steps, what=f"{nt}x{nph} ")


def _degree_energy(om, th, lmax):
    """sum_m |<om, Y_lm>|^2 per degree l (midpoint rule in theta, FFT in phi),
    with associated Legendre functions from scipy, independent of the input
    generator's recurrence."""
    from scipy.special import lpmv
    from math import factorial
    nph = om.shape[1]
    Z = np.fft.rfft(om, axis=1) * (2 * np.pi / nph)
    wq = np.sin(th) * (th[1] - th[0])
    E = np.zeros(lmax + 1)
    for m in range(lmax + 1):
        for l in range(max(m, 1), lmax + 1):
            nrm = np.sqrt((2 * l + 1) / (4 * np.pi) * factorial(l - m) / factorial(l + m))
            c = (nrm * lpmv(m, l, np.cos(th)) * wq) @ Z[:, m]
            E[l] += (1 if m == 0 else 2) * abs(c) ** 2
    return E


def test_c2_full_run_decays_at_the_viscous_rates():
    # The C2 workload run to its end: 512 x 1024, tau = 5e-4 (nu = tau), 2000
    # steps of a rigid rotation u_phi = -1e-3 sin th plus random toroidal flow
    # (vorticity sum_{l<=16} b_lm Y_lm, b_lm ~ N(0, 1e-8)), FP64 and FP32 store.
    # Closed forms (Sec. IV.B; App. B): the n = 0 shear mode (rigid rotation)
    # is undamped, and a degree-l toroidal mode decays at kappa_l =
    # nu (l-1)(l+2) — rigid rotation only turns it (Rossby-Haurwitz), so the
    # per-degree energy E_l (sum over m) falls as exp(-2 kappa_l t_eff).  Runs
    # start at equilibrium, where the viscous stress builds up as
    # 1 - exp(-t/tau) (BGK relaxation), so t_eff = t - tau (1 - exp(-t/tau)).
    # Nonlinear transfer between degrees (amplitude 1e-4) is left out of the
    # closed form: the measured decrements must agree with it to 1 % (FP64)
    # or 2 % (FP32, plus its rounding noise).  FP32 vorticity within 1e-4 of
    # FP64 after the whole run.
    import closed_forms as cf
    from paper_2504_15574_amd import Solver
    nt, nph, tau, steps, lmax = 512, 1024, 5e-4, 2000, 16
    st = W.random_vorticity_state(nt, nph, seed=0, lmax=lmax, amp=1e-4, shear=1e-3)
    th, _ = W.grid(nt, nph)
    G0 = cf.shear_G(0, "e", th)
    om_end = {}
    for storage, rel_tol, rot_tol, l1_tol in (("f64", 0.01, 1e-9, 1e-8), ("f32", 0.02, 1e-7, 1e-7)):
        print(f"[case] C2 {storage} {nt}x{nph} tau={tau} steps={steps}", flush=True)
        s = Solver(nt, nph, tau, storage=storage)
        s.init_fields(*st)
        om0 = s.vorticity()
        s.step(steps)
        om1 = s.vorticity()
        _, _, up1 = s.moments(with_T=False)
        t = steps * s.dt
        s.close()
        om_end[storage] = om1
        V0 = cf.project_shear(st[2].mean(axis=1), th, G0)
        V1 = cf.project_shear(up1.mean(axis=1), th, G0)
        E0, E1 = _degree_energy(om0, th, lmax), _degree_energy(om1, th, lmax)
        dec = -0.5 * np.log(E1[1:] / E0[1:])                  # degrees 1..lmax
        t_eff = t - tau * (1.0 - np.exp(-t / tau))
        want = np.array([cf.toroidal_kappa(l, tau) * t_eff for l in range(2, lmax + 1)])
        rel = np.abs(dec[1:] / want - 1.0)
        print(f"  {storage}: rigid rotation {V1 / V0 - 1:.2e}, l = 1 decrement {dec[0]:.2e}, "
              f"l = 2..{lmax} decrement vs closed form max rel {rel.max():.2e}")
        assert abs(V1 / V0 - 1.0) < rot_tol
        assert abs(dec[0]) < l1_tol                           # l = 1 (tilted rotation): undamped
        assert rel.max() < rel_tol
        assert t > 10 * tau                                   # well past the initial layer
    w = np.sin(th)[:, None]
    d = om_end["f32"] - om_end["f64"]
    err = np.sqrt((w * d * d).sum() / (w * om_end["f64"] ** 2).sum())
    print(f"  FP32 vs FP64 vorticity after {steps} steps: {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_reduced_precision_full_size_properties(storage):
    # At the benchmark size the reduced formats stay finite, conserve the
    # rest-state structure and track the FP64 run: after 20 steps the
    # area-weighted velocity error is below 1e-5 (f32) / 1e-3 (f16).
    from paper_2504_15574_amd import Solver
    nt, nph, tau = 2048, 4096, 1e-5
    st = W.turbulence_state(nt, nph, seed=0, lmax=256, urms=0.05)
    res = {}
    for s in ("f64", storage):
        sol = Solver(nt, nph, tau, storage=s)
        sol.init_fields(*st)
        sol.step(20)
        d = sol.diagnostics()
        res[s] = (sol.moments(with_T=False), d)
        sol.close()
    (r64, a64, b64), d64 = res["f64"]
    (r, a, b), d = res[storage]
    th, _ = W.grid(nt, nph)
    w = np.sin(th)[:, None]
    du = np.sqrt((w * ((a - a64) ** 2 + (b - b64) ** 2)).sum() / (w * (a64 ** 2 + b64 ** 2)).sum())
    print(f"  {storage}: u rel L2 {du:.2e}, mass {d[0]:.15e} vs {d64[0]:.15e}")
    assert du < (1e-5 if storage == "f32" else 1e-3)
    assert abs(d[0] - d64[0]) < 1e-6 * d64[0]


@pytest.mark.parametrize("storage,bound", [("f32", 1e-5), ("f16", 2e-2)])
def test_reduced_precision_long_run_has_no_rounding_drift(storage, bound):
    # 2000 steps (6000 rounded stage outputs per population).  Unbiased rounding
    # accumulates like a random walk, about sqrt(6000) ~ 80 ulp of the stored
    # deviation; rounding to nearest of a nearly constant increment errs the
    # same way every step and would reach ~1500 ulp (measured without the
    # dithered store and the moment-exact FP32 quadrature: u error 9e-5 in FP32,
    # 7e-2 in FP16).  The bounds sit between the two regimes.
    from paper_2504_15574_amd import Solver
    nt, nph, tau = 32, 64, 1e-3
    st = W.random_state(nt, nph, seed=3, du=0.05)
    res = {}
    for s in ("f64", storage):
        sol = Solver(nt, nph, tau, storage=s)
        sol.init_fields(*st)
        sol.step(2000)
        res[s] = sol.moments(with_T=False)
        sol.close()
    th, _ = W.grid(nt, nph)
    w = np.sin(th)[:, None]
    (r64, a64, b64), (r, a, b) = res["f64"], res[storage]
    du = np.sqrt((w * ((a - a64) ** 2 + (b - b64) ** 2)).sum() / (w * (a64 ** 2 + b64 ** 2)).sum())
    print(f"  {storage}: u rel L2 after 2000 steps {du:.2e}")
    assert du < bound


def test_fp32_store_meets_the_benchmark_precision_gate():
    # The benchmark grid (2048 x 4096, tau = 1e-5, turbulence with rms |u| =
    # 0.05), FP32 store against FP64 after 1000 steps from the same initial
    # state: area-weighted relative L2 of rho, u and vorticity within 1e-4.
    from paper_2504_15574_amd import Solver
    nt, nph, tau = 2048, 4096, 1e-5
    st = W.turbulence_state(nt, nph, seed=0, lmax=256, urms=0.05)
    res = {}
    for s in ("f64", "f32"):
        sol = Solver(nt, nph, tau, storage=s)
        sol.init_fields(*st)
        sol.step(1000)
        res[s] = (sol.moments(with_T=False), sol.vorticity())
        sol.close()
    th, _ = W.grid(nt, nph)
    w = np.sin(th)[:, None]
    rel = lambda x, y: np.sqrt((w * (x - y) ** 2).sum() / (w * y ** 2).sum())
    (r64, a64, b64), o64 = res["f64"]
    (r, a, b), o = res["f32"]
    e = {"rho": rel(r, r64), "u": np.sqrt((rel(a, a64) ** 2 * (w * a64 ** 2).sum() +
                                            rel(b, b64) ** 2 * (w * b64 ** 2).sum()) /
                                           (w * (a64 ** 2 + b64 ** 2)).sum()),
         "vorticity": rel(o, o64)}
    print("  " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert all(v <= 1e-4 for v in e.values()), e
    # The density fluctuation rho - 1 is 1.2e-9 rms at this time (the flow is
    # nearly incompressible and the initial pressure imbalance has had a sixth
    # of a cell's sound crossing), far below what FP32 deviations resolve: the
    # stored populations carry ~0.02 with an ulp of 1.9e-9, and 16 dithered
    # roundings per stage add an unbiased noise to the mass.  Its error is
    # therefore stated, and bounded by that noise: a random walk of 3 x 1000
    # stages of 16 roundings of at most 1/2 ulp (uniform, variance ulp^2 / 12).
    w1 = w * np.ones_like(r)
    w1 /= w1.sum()
    drho = np.sqrt((w1 * (r - r64) ** 2).sum())
    fluct = np.sqrt((w1 * (r64 - 1.0) ** 2).sum())
    ulp = np.spacing(np.float32(0.02))
    walk = np.sqrt(3 * 1000 * 16 / 12.0) * ulp
    print(f"  rho - 1: FP64 rms {fluct:.2e}, FP32 rms error {drho:.2e} "
          f"({drho / fluct:.1f} of the fluctuation; rounding-noise bound {walk:.2e})")
    assert drho <= walk


# the largest grids whose population buffer stays below 4 GiB (the reach of the
# kernels' 32-bit buffer offsets; one more row is rejected on the host)
MAX_GRIDS = {"f64": (4095, 8192), "f32": (8191, 8192), "f16": (16383, 8192)}


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_largest_grids_match_a_two_column_run(storage):
    # A phi-uniform state stays phi-uniform, and its phi flux differences are
    # exactly zero, so every column of the largest grid must evolve like the
    # same rows on 2 columns (same dt): bit for bit in FP64 (checked against
    # the oracle on the 2 columns), within the dithered rounding otherwise.
    # Every halo and pole address of the largest grids is exercised, up to
    # the last population's last row.
    from paper_2504_15574_amd import Solver
    nt, nph = MAX_GRIDS[storage]
    th = (np.arange(nt) + 0.5) * np.pi / nt
    rho = (1.0 + 0.01 * np.sin(3 * th))[:, None]
    ut = (0.02 * np.cos(2 * th) * np.sin(th))[:, None]
    up = (0.03 * np.sin(th) + 0.01 * np.sin(5 * th))[:, None]
    tau = 1e-3
    dt = oracle.suggest_dt(nt, nph, tau)
    print(f"[case] {storage} {nt}x{nph} dt={dt:.3e}", flush=True)
    small = Solver(nt, 2, tau, dt, storage=storage)
    small.init_fields(rho, ut, up)
    small.step(1)
    ms = small.moments(with_T=False)
    if storage == "f64":
        fs = small.populations()
        fr = oracle.step(oracle.init(*(np.repeat(a, 2, axis=1) for a in (rho, ut, up))), 1, tau=tau, dt=dt,
                         threads=THREADS)
        assert np.abs(fs - fr).max() <= 1e-12 * np.abs(fr).max()
    small.close()
    big = Solver(nt, nph, tau, dt, storage=storage)
    big.init_fields(rho, ut, up)
    big.step(1)
    mb = big.moments(with_T=False)
    big.close()
    tol = {"f64": 0.0, "f32": 1e-6, "f16": 1e-4}[storage]
    for a, b in zip(mb, ms):
        ref = b[:, :1]
        assert np.abs(b[:, 1:] - ref).max() <= tol
        assert np.abs(a - ref).max() <= tol, storage
