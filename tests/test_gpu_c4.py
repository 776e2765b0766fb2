"""The batched-ensemble workload at its stated size, bit for bit.

64 independent runs (32 at 128 x 256, 32 at 256 x 512), D2Q16, FP32 deviation
store, each an axisymmetric shock at rest (Sec. IV.C): rho = 1.5, T = 1.2 for
theta < theta0, else rho = T = 1, with nu = tau ~ U[1e-4, 1e-2] and theta0 ~
U[pi/6, pi/3] drawn per run in run order from seed 0, dt per run from the
stability rule; 400 steps.  About 23 000 tiles of 15 x 16 cells make up one
stage, so in the persistent launch every workgroup works through many tiles
per stage.  Each form -- one launch per run, batched launches, one persistent
launch, and that persistent launch replayed from a HIP graph -- must leave
every run's populations identical, bit for bit, to stepping it alone.
"""
import hashlib

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 400


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    from paper_2504_15574_amd import load
    load()


def _specs():
    rng = np.random.default_rng(0)
    out = []
    for i in range(64):
        nt, nph = (128, 256) if i < 32 else (256, 512)
        nu = float(rng.uniform(1e-4, 1e-2))
        th0 = float(rng.uniform(np.pi / 6, np.pi / 3))
        out.append((nt, nph, nu, th0))
    return out


def _fresh_runs(specs):
    from paper_2504_15574_amd import Solver
    runs = []
    for nt, nph, nu, th0 in specs:
        s = Solver(nt, nph, nu, storage="f32")
        s.init_fields(*W.shock_state(nt, nph, th0, rho_in=1.5, T_in=1.2))
        runs.append(s)
    return runs


def _digests(runs):
    out = []
    for s in runs:
        f = s.populations()
        assert np.isfinite(f).all()
        out.append(hashlib.sha256(f.tobytes()).hexdigest())
    return out


def _close(runs):
    import torch
    for s in runs:
        s.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_c4_forms_equal_one_by_one_bitwise():
    from paper_2504_15574_amd import Ensemble
    specs = _specs()
    assert sum(n_t * n_p for n_t, n_p, _, _ in specs) == 5242880
    print("[case] C4 one run per launch", flush=True)
    ref_runs = _fresh_runs(specs)
    for s in ref_runs:
        s.step(STEPS)
    ref = _digests(ref_runs)
    _close(ref_runs)

    def check(form, advance):
        print(f"[case] C4 {form}", flush=True)
        runs = _fresh_runs(specs)
        ens = Ensemble(runs)
        advance(ens)
        got = _digests(runs)
        ens.release()
        _close(runs)
        bad = [i for i, (a, b) in enumerate(zip(got, ref)) if a != b]
        assert not bad, f"{form}: runs {bad} differ from stepping them alone"

    check("batched, tuned grouping and per-size tiles",
          lambda e: (e.configure("by_size", {(128, 256): (15, 16), (256, 512): (7, 32)}),
                     e.step(STEPS)))
    check("batched, one launch for all runs", lambda e: e.step(STEPS))
    check("persistent, one launch", lambda e: e.step(STEPS, persistent=True))

    def graph(e):
        e.capture(STEPS, persistent=True)
        e.replay()
        e.check()

    check("persistent launch replayed from a HIP graph", graph)
