"""Ensembles: many independent runs advanced by shared stage launches.

A batched launch covers the tiles of several contexts; every cell runs the same
arithmetic as in a single-context launch, so batched and one-by-one stepping
must agree bit for bit.  HIP-graph replays of recorded steps must equal eager
stepping, also with other work queued between replays.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    from paper_2504_15574_amd import load
    load()


def _runs(storage, specs, seed=0):
    from paper_2504_15574_amd import Solver
    rng = np.random.default_rng(seed)
    out = []
    for nt, nph in specs:
        tau = float(rng.uniform(1e-3, 5e-3))
        s = Solver(nt, nph, tau, storage=storage)
        s.init_fields(*W.random_state(nt, nph, seed=int(rng.integers(1 << 30)), du=0.05,
                                      dT=0.05, smooth=False))
        out.append(s)
    return out


SPECS = [(32, 64), (32, 64), (48, 96), (20, 1), (16, 130), (64, 128)]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_batched_equals_one_by_one_bitwise(storage):
    from paper_2504_15574_amd import Ensemble, vlbm_stage_launches
    a = _runs(storage, SPECS, seed=1)
    b = _runs(storage, SPECS, seed=1)
    ens = Ensemble(a)
    ens.step(7)
    for s in b:
        s.step(7)
    for x, y in zip(a, b):
        assert vlbm_stage_launches(x.ctx) == 21
        assert np.array_equal(x.populations(), y.populations())
    for s in a + b:
        s.close()


@pytest.mark.parametrize("shape", [(511, 1000), (512, 1024)])
def test_direct_to_lds_form_gives_the_register_form_bits(shape):
    # A single FP32 run of at least 2048 15 x 16 tiles takes the rounds
    # kernel's direct-to-LDS form; inside a batch the same run takes the
    # register form.  Ragged edges (511 x 1000: 35 x 63 tiles), pole rows and
    # the phi wrap all go through the direct loads' folded addresses.
    from paper_2504_15574_amd import Ensemble
    nt, nph = shape
    a = _runs("f32", [shape, (16, 32)], seed=5)
    b = _runs("f32", [shape], seed=5)
    assert ((nt + 14) // 15) * ((nph + 15) // 16) >= 2048
    Ensemble(a).step(6)
    b[0].step(6)
    assert np.array_equal(a[0].populations(), b[0].populations())
    for s in a + b:
        s.close()


def test_more_than_64_runs_split_into_launches():
    from paper_2504_15574_amd import Ensemble
    specs = [(8, 16)] * 40 + [(12, 32)] * 30
    a = _runs("f32", specs, seed=2)
    b = _runs("f32", specs, seed=2)
    Ensemble(a).step(3)
    for s in b:
        s.step(3)
    for x, y in zip(a, b):
        assert np.array_equal(x.populations(), y.populations())
    for s in a + b:
        s.close()


def test_graph_replays_match_eager_steps():
    # Record 4 steps once, replay three times with eager work (moment and
    # population read-backs, an eager step of another run) between the replays;
    # every replay must leave the same state as eager stepping.
    from paper_2504_15574_amd import Ensemble
    specs = [(32, 64), (48, 96), (16, 32)]
    g = _runs("f32", specs, seed=3)
    e = _runs("f32", specs, seed=3)
    other = _runs("f32", [(24, 48)], seed=4)[0]
    ens_g, ens_e = Ensemble(g), Ensemble(e)
    ens_g.capture(4)
    for rep in range(3):
        ens_g.replay()
        ens_e.step(4)
        other.step(1)
        _ = g[0].moments()
        for x, y in zip(g, e):
            assert np.array_equal(x.populations(), y.populations()), f"replay {rep}"
    ens_g.release()
    for s in g + e + [other]:
        s.close()


def test_graph_replays_of_the_direct_to_lds_form_match_eager_steps():
    # A graph of one FP32 run of 512 x 1024 (2240 15 x 16 tiles) records the
    # rounds kernel's direct-to-LDS form; its replays, with eager work between
    # them, must equal eager stepping of the same run (which takes that form too).
    from paper_2504_15574_amd import Ensemble
    g = _runs("f32", [(512, 1024)], seed=6)
    e = _runs("f32", [(512, 1024)], seed=6)
    other = _runs("f32", [(24, 48)], seed=7)[0]
    ens_g = Ensemble(g)
    ens_g.capture(3)
    for rep in range(3):
        ens_g.replay()
        e[0].step(3)
        other.step(1)
        _ = g[0].moments()
        assert np.array_equal(g[0].populations(), e[0].populations()), f"replay {rep}"
    ens_g.release()
    for s in g + e + [other]:
        s.close()


def test_batch_argument_errors():
    from paper_2504_15574_amd import VlbmError, vlbm_step_batch
    a = _runs("f32", [(16, 32)], seed=5)[0]
    b = _runs("f64", [(16, 32)], seed=5)[0]
    with pytest.raises(VlbmError):
        vlbm_step_batch([a.ctx, b.ctx], 1)          # mixed storage formats
    with pytest.raises(VlbmError):
        vlbm_step_batch([a.ctx, a.ctx], 1)          # the same run twice
    with pytest.raises(VlbmError):
        vlbm_step_batch([], 1)
    a.close()
    b.close()


def test_shock_state_parity_with_oracle():
    # The ensemble's initial state: rho = 1.5, T = 1.2 inside theta0, at rest
    # (temperature enters through the order-3 projection); WENO meets the jump.
    from paper_2504_15574_amd import Solver
    nt, nph, tau = 64, 128, 2e-3
    st = W.shock_state(nt, nph, theta0=np.pi / 4)
    dt = oracle.suggest_dt(nt, nph, tau)
    s = Solver(nt, nph, tau, dt)
    s.init_fields(*st)
    s.step(20)
    fg = s.populations()
    s.close()
    fr = oracle.step(oracle.init(*st), 20, tau=tau, dt=dt, threads=8)
    assert np.abs(fg - fr).max() <= 1e-12 * np.abs(fr).max()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_tile_shapes_give_identical_bits(storage):
    # 7 x 32 tiles against the default 15 x 16, single and batched launches
    from paper_2504_15574_amd import Ensemble
    specs = [(26, 50), (37, 1), (32, 64), (20, 130)]
    a = _runs(storage, specs, seed=11)
    b = _runs(storage, specs, seed=11)
    Ensemble(a, tile=(7, 32)).step(5)
    for s in b:
        s.step(5)
    for x, y in zip(a, b):
        assert np.array_equal(x.populations(), y.populations())
    for s in a + b:
        s.close()


def test_wide_tiles_match_the_oracle():
    from paper_2504_15574_amd import Solver, vlbm_set_tile_shape
    nt, nph, tau = 23, 70, 2e-3
    st = W.random_state(nt, nph, seed=12, du=0.05, dT=0.05, smooth=False)
    dt = oracle.suggest_dt(nt, nph, tau)
    s = Solver(nt, nph, tau, dt)
    vlbm_set_tile_shape(s.ctx, 7, 32)
    s.init_fields(*st)
    s.step(6)
    fg = s.populations()
    s.close()
    fr = oracle.step(oracle.init(*st), 6, tau=tau, dt=dt, threads=8)
    assert np.abs(fg - fr).max() <= 1e-12 * np.abs(fr).max()


def test_tile_shape_errors_and_autotuner():
    from paper_2504_15574_amd import Ensemble, VlbmError, vlbm_set_tile_shape, vlbm_step_batch
    a, b = _runs("f32", [(16, 32), (16, 32)], seed=13)
    with pytest.raises(VlbmError):
        vlbm_set_tile_shape(a.ctx, 8, 32)
    vlbm_set_tile_shape(a.ctx, 7, 32)
    with pytest.raises(VlbmError):
        vlbm_step_batch([a.ctx, b.ctx], 1)          # mixed tile shapes
    ens = Ensemble([a, b])
    times = ens.autotune(steps=2)
    assert len(times) == 6 and ens.tile in Ensemble.TILES     # one grid size: no per-size choice
    with pytest.raises(ValueError):
        ens.configure("all", {(16, 32): (7, 32)})           # per-size tiles need "by_size"
    a.close()
    b.close()


def test_autotuner_per_size_tiles_keep_the_bits():
    # Two grid sizes: the tuner also tries each size's own fastest tile shape;
    # whatever it picks, the runs match the same runs stepped one by one.
    from paper_2504_15574_amd import Ensemble
    sizes = [(16, 32), (30, 64), (16, 32), (30, 64)]
    runs = _runs("f32", sizes, seed=17)
    ref = _runs("f32", sizes, seed=17)
    ens = Ensemble(runs)
    times = ens.autotune(steps=2)
    assert len(times) in (6, 7) and all(v > 0 for v in times.values())
    ens.configure("by_size", {(16, 32): (7, 32), (30, 64): (15, 16)})
    assert ens.tile_name() == "16x32:7x32,30x64:15x16"
    ens.step(3)
    for s, r in zip(runs, ref):                           # the same number of steps one by one
        r.step(round((s.t - r.t) / r.dt))
        assert np.array_equal(s.populations(), r.populations())
    for s in runs + ref:
        s.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_persistent_launch_equals_one_by_one_bitwise(storage):
    # one cooperative launch carries all 7 steps of the six runs (grid
    # barriers between the RK stages); every cell must equal stepping each run
    # alone, and the step counters (dither phase) must advance the same way
    from paper_2504_15574_amd import Ensemble, vlbm_stage_launches
    a = _runs(storage, SPECS, seed=21)
    b = _runs(storage, SPECS, seed=21)
    Ensemble(a).step(7, persistent=True)
    for s in b:
        s.step(7)
    for x, y in zip(a, b):
        assert vlbm_stage_launches(x.ctx) == 21
        assert np.array_equal(x.populations(), y.populations())
    Ensemble(a).step(2, persistent=True)           # a second launch continues the runs
    for s in b:
        s.step(2)
    for x, y in zip(a, b):
        assert np.array_equal(x.populations(), y.populations())
    for s in a + b:
        s.close()


def test_persistent_launch_many_runs_and_wide_tiles():
    from paper_2504_15574_amd import Ensemble
    specs = [(8, 16)] * 40 + [(12, 32)] * 30 + [(37, 70)]
    a = _runs("f32", specs, seed=22)
    b = _runs("f32", specs, seed=22)
    Ensemble(a, tile=(7, 32)).step(3, persistent=True)
    for s in b:
        s.step(3)
    for x, y in zip(a, b):
        assert np.array_equal(x.populations(), y.populations())
    for s in a + b:
        s.close()


def test_persistent_launch_rejects_other_kernels():
    from paper_2504_15574_amd import Solver, VlbmError, vlbm_step_batch_persistent
    s9 = Solver(16, 32, 2e-3, q=3)
    sk = Solver(16, 32, 2e-3, komissarov=True)
    for s in (s9, sk):
        s.init_fields(*W.random_state(16, 32, seed=1, du=0.05))
        with pytest.raises(VlbmError):
            vlbm_step_batch_persistent([s.ctx], 1)
        s.close()


def test_persistent_barrier_wait_gives_up_with_an_error():
    # A spin limit of 0 makes every barrier wait give up at once: the kernel
    # still runs to its end, and the call reports the undefined state.  The
    # default limit then steps correctly again.
    from paper_2504_15574_amd import VlbmError, vlbm_set_barrier_spin_limit, vlbm_step_batch_persistent
    a = _runs("f32", [(32, 64), (48, 96)], seed=23)
    b = _runs("f32", [(32, 64), (48, 96)], seed=23)
    vlbm_set_barrier_spin_limit(0)
    try:
        with pytest.raises(VlbmError):
            vlbm_step_batch_persistent([s.ctx for s in a], 2)
    finally:
        vlbm_set_barrier_spin_limit(1 << 20)
    c = _runs("f32", [(32, 64), (48, 96)], seed=23)
    vlbm_step_batch_persistent([s.ctx for s in c], 2)
    for s in b:
        s.step(2)
    for x, y in zip(c, b):
        assert np.array_equal(x.populations(), y.populations())
    for s in a + b + c:
        s.close()


def test_persistent_graph_replays_match_eager_steps():
    # one persistent launch per replay, recorded in a HIP graph; eager work
    # between the replays; every replay must equal eager stepping
    from paper_2504_15574_amd import Ensemble
    specs = [(32, 64), (48, 96), (16, 32)]
    g = _runs("f32", specs, seed=24)
    e = _runs("f32", specs, seed=24)
    other = _runs("f32", [(24, 48)], seed=25)[0]
    ens_g, ens_e = Ensemble(g), Ensemble(e)
    ens_g.capture(4, persistent=True)
    for rep in range(3):
        ens_g.replay()
        ens_g.check()
        ens_e.step(4)
        other.step(1)
        _ = g[0].moments()
        for x, y in zip(g, e):
            assert np.array_equal(x.populations(), y.populations()), f"replay {rep}"
    ens_g.release()
    for s in g + e + [other]:
        s.close()


def test_graph_check_reports_a_persistent_launch_that_gave_up():
    # The spin limit is recorded with the launch: a graph captured with a limit
    # of 0 gives up at its first barrier on every replay (the kernel still runs
    # to its end) and vlbm_graph_check says so; a per-stage graph checks clean.
    from paper_2504_15574_amd import Ensemble, VlbmError, vlbm_set_barrier_spin_limit
    runs = _runs("f32", [(32, 64), (16, 32)], seed=26)
    ens = Ensemble(runs)
    ens.capture(2)
    ens.replay()
    ens.check()
    vlbm_set_barrier_spin_limit(0)
    try:
        ens.capture(2, persistent=True)
    finally:
        vlbm_set_barrier_spin_limit(1 << 20)
    ens.replay()
    with pytest.raises(VlbmError):
        ens.check()
    ens.release()
    for s in runs:
        s.close()


def test_ensemble_refuses_work_after_a_run_is_closed():
    # The ensemble's launch groups and graphs hold the runs' contexts; once a
    # run is closed every call that would use them raises instead.
    from paper_2504_15574_amd import Ensemble, VlbmError
    runs = _runs("f32", [(32, 64), (16, 32)], seed=27)
    ens = Ensemble(runs)
    ens.step(1)
    ens.capture(1)
    runs[1].close()
    for call in (lambda: ens.step(1), lambda: ens.replay(), lambda: ens.check(),
                 lambda: ens.capture(1), lambda: ens.autotune(1)):
        with pytest.raises(VlbmError):
            call()
    ens.release()
    runs[0].close()



@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("nt,nph,seed", [(8, 130, 3), (3, 2, 4), (64, 96, 5), (48, 20, 6), (5, 18, 7)])
def test_tile_shapes_give_the_same_bits_on_pole_and_small_grids(storage, nt, nph, seed):
    # 15 x 16 tiles run the population-round kernel, 7 x 32 tiles the
    # one-population-at-a-time kernel; both evaluate every flux with the same
    # arithmetic and accumulate each cell in the same order.  Grids where
    # every row is a pole row, the smallest grid, interior tiles, the one-fold
    # and the integer-modulo column wraps.
    from paper_2504_15574_amd import Solver, vlbm_set_tile_shape
    st = W.random_state(nt, nph, seed=seed, du=0.05, dT=0.05, smooth=False)
    out = []
    for shape in ((15, 16), (7, 32)):
        s = Solver(nt, nph, 2e-3, storage=storage)
        vlbm_set_tile_shape(s.ctx, *shape)
        s.init_fields(*st)
        s.step(6)
        out.append(s.populations())
        s.close()
    assert np.array_equal(out[0], out[1])
