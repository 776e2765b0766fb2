"""Upwind fluxes U1, U2, U3 and the Komissarov theta derivative on the GPU,
against the FP64 oracle (Sec. III.E, eqs. (fluxes_U1-3), (Komissarov_scheme))."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
THREADS = 8


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    from paper_2504_15574_amd import load
    load()


CASES = [(26, 50, 1, False), (37, 1, 2, True), (23, 70, 3, False)]


@pytest.mark.parametrize("scheme", ["u1", "u2", "u3", "weno5"])
@pytest.mark.parametrize("komissarov", [False, True])
@pytest.mark.parametrize("nt,nph,seed,smooth", CASES)
def test_scheme_parity_with_oracle(scheme, komissarov, nt, nph, seed, smooth):
    from paper_2504_15574_amd import Solver
    tau = 2e-3
    st = W.random_state(nt, nph, seed=seed, du=0.05, dT=0.05, smooth=smooth)
    dt = oracle.suggest_dt(nt, nph, tau)
    s = Solver(nt, nph, tau, dt, scheme=scheme, komissarov=komissarov)
    s.init_fields(*st)
    s.step(5)
    fg = s.populations()
    s.close()
    fr = oracle.step(oracle.init(*st), 5, tau=tau, dt=dt, threads=THREADS, scheme=scheme,
                     komissarov=komissarov)
    assert np.abs(fg - fr).max() <= 1e-12 * np.abs(fr).max()


def test_general_kernel_gives_the_default_bits():
    # A WENO-5 run batched with a U3 run goes through the general kernel
    # variant; it must give the same bits as the WENO-5 run stepped alone.
    from paper_2504_15574_amd import Ensemble, Solver
    st = W.random_state(30, 64, seed=4, du=0.05, smooth=False)
    a = Solver(30, 64, 2e-3, storage="f32")
    b = Solver(30, 64, 2e-3, storage="f32")
    c = Solver(20, 32, 2e-3, storage="f32", scheme="u3", komissarov=True)
    for s in (a, b, c):
        s.init_fields(*W.random_state(s.n_theta, s.n_phi, seed=4, du=0.05, smooth=False))
    Ensemble([a, c]).step(4)
    b.step(4)
    assert np.array_equal(a.populations(), b.populations())
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_komissarov_rest_state_is_steady_and_mass_exact(storage):
    from paper_2504_15574_amd import Solver
    nt, nph = 48, 96
    s = Solver(nt, nph, 2e-3, scheme="u3", komissarov=True, storage=storage)
    s.init_fields(*W.rest_state(nt, nph))
    f0 = s.populations()
    s.step(50)
    assert np.abs(s.populations() - f0).max() < (1e-14 if storage == "f64" else 1e-7)
    s.close()
    # band-area-weighted mass of a rough state is conserved to rounding
    st = W.random_state(nt, nph, seed=8, du=0.05, dT=0.05, smooth=False)
    s = Solver(nt, nph, 2e-3, scheme="u3", komissarov=True)
    s.init_fields(*st)
    dth = np.pi / nt
    band = np.cos(np.arange(nt) * dth) - np.cos((np.arange(nt) + 1) * dth)
    mass = lambda f: (band[:, None] * f.sum(axis=0)).sum()
    m0 = mass(s.populations())
    s.step(30)
    assert abs(mass(s.populations()) - m0) < 1e-13 * m0
    s.close()


def test_unknown_advection_is_rejected():
    from paper_2504_15574_amd import vlbm as B
    p = B.make_params(16, 32, 1e-3, 1e-3)
    for adv in (4, 0x200, 0x103 | 0x400):
        p.advection = adv
        assert B.vlbm_workspace_bytes(p) == 0


def test_diagnostics_and_vorticity_do_not_depend_on_the_flux_form():
    # The Komissarov form uses a flux function without sin(theta); the area
    # element of the diagnostics and the metric of the vorticity are those of
    # the sphere in every form, so the same populations give the same numbers.
    from paper_2504_15574_amd import Solver
    st = W.random_vorticity_state(32, 64, seed=4, lmax=6, amp=1e-2, shear=1e-2)
    std = Solver(32, 64, 2e-3, 5e-4)
    std.init_fields(*st)
    f = std.populations()
    std.set_populations(f)        # both contexts encode the same FP64 populations
    kom = Solver(32, 64, 2e-3, 5e-4, scheme="u3", komissarov=True)
    kom.set_populations(f)
    d0, d1 = std.diagnostics(), kom.diagnostics()
    o0, o1 = std.vorticity(), kom.vorticity()
    std.close()
    kom.close()
    assert np.array_equal(d0, d1)
    assert np.array_equal(o0, o1)


def _upwind_bits(nt, nph, storage, scheme, komissarov, tile, steps):
    from paper_2504_15574_amd import Solver
    from paper_2504_15574_amd.vlbm import vlbm_set_tile_shape
    s = Solver(nt, nph, 2e-3, storage=storage, scheme=scheme, komissarov=komissarov)
    vlbm_set_tile_shape(s.ctx, *tile)
    s.init_fields(*W.random_state(nt, nph, seed=11, du=0.05, dT=0.05, smooth=False))
    s.step(steps)
    f = s.populations()
    s.close()
    return f


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("scheme,komissarov", [("u1", False), ("u2", True), ("u3", False), ("u3", True)])
def test_upwind_rounds_kernel_gives_the_per_population_kernel_bits(storage, scheme, komissarov):
    # D2Q16 upwind runs on 15 x 16 tiles take the population-rounds kernel, on
    # 7 x 32 tiles the per-population kernel: same fluxes, same order of
    # accumulation, same bits (a ragged grid with pole and wrap tiles)
    print(f"[case] upwind rounds vs per-population {storage} {scheme} kom={komissarov}", flush=True)
    a = _upwind_bits(61, 96, storage, scheme, komissarov, (15, 16), 6)
    b = _upwind_bits(61, 96, storage, scheme, komissarov, (7, 32), 6)
    assert np.isfinite(a).all() and np.array_equal(a, b)


@pytest.mark.parametrize("komissarov", [False, True])
def test_upwind_direct_to_lds_form_gives_the_per_population_kernel_bits(komissarov):
    # 512 x 1024 has 2240 tiles of 15 x 16: a single FP32 run takes the rounds
    # kernel's direct-to-LDS form
    print(f"[case] upwind direct-to-LDS vs per-population kom={komissarov}", flush=True)
    a = _upwind_bits(512, 1024, "f32", "u3", komissarov, (15, 16), 3)
    b = _upwind_bits(512, 1024, "f32", "u3", komissarov, (7, 32), 3)
    assert np.isfinite(a).all() and np.array_equal(a, b)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batched_upwind_runs_equal_one_by_one(storage):
    # upwind runs of two sizes and all three schemes in one batched launch (the
    # rounds kernel's run lookup) against each run stepped alone
    print(f"[case] batched upwind {storage}", flush=True)
    from paper_2504_15574_amd import Ensemble, Solver
    specs = [(45, 64, "u3", True), (30, 96, "u1", False), (45, 64, "u2", True), (61, 32, "u3", False)]

    def fresh():
        runs = []
        for i, (nt, nph, scheme, kom) in enumerate(specs):
            s = Solver(nt, nph, 2e-3, storage=storage, scheme=scheme, komissarov=kom)
            s.init_fields(*W.random_state(nt, nph, seed=20 + i, du=0.05, dT=0.05, smooth=False))
            runs.append(s)
        return runs

    alone = fresh()
    for s in alone:
        s.step(5)
    together = fresh()
    ens = Ensemble(together)
    ens.step(5)
    for a, b in zip(alone, together):
        fa, fb = a.populations(), b.populations()
        assert np.isfinite(fa).all() and np.array_equal(fa, fb)
    ens.release()
    for s in alone + together:
        s.close()
