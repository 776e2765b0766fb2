"""The D2Q9 model (Q = 3, App. A.1) on the GPU against the FP64 oracle."""
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


@pytest.mark.parametrize("nt,nph,seed,smooth", [(26, 50, 1, False), (37, 1, 2, True), (20, 130, 3, False)])
@pytest.mark.parametrize("scheme,komissarov", [("weno5", False), ("u3", True), ("u1", False)])
def test_d2q9_parity_with_oracle(nt, nph, seed, smooth, scheme, komissarov):
    from paper_2504_15574_amd import Solver
    tau = 2e-3
    st = W.random_state(nt, nph, seed=seed, du=0.05, dT=0.05, smooth=smooth)
    dt = oracle.suggest_dt(nt, nph, tau)
    s = Solver(nt, nph, tau, dt, q=3, scheme=scheme, komissarov=komissarov)
    s.init_fields(*st)
    f0 = s.populations()
    s.step(5)
    fg = s.populations()
    r, a, b, T = s.moments()
    s.close()
    fi = oracle.init(*st, q=3)
    assert np.abs(f0 - fi).max() <= 1e-14 * np.abs(fi).max()
    fr = oracle.step(fi, 5, tau=tau, dt=dt, threads=THREADS, scheme=scheme, komissarov=komissarov)
    assert fg.shape == (9, nt, nph)
    assert np.abs(fg - fr).max() <= 1e-12 * np.abs(fr).max()
    rr, ar, br, Tr = oracle.moments(fr)
    assert np.abs(r - rr).max() < 1e-13 and np.abs(a - ar).max() < 1e-12 and np.abs(T - Tr).max() < 1e-12


@pytest.mark.parametrize("storage,bound", [("f32", 2e-5), ("f16", 5e-3)])
def test_d2q9_reduced_precision(storage, bound):
    from paper_2504_15574_amd import Solver
    st = W.random_vorticity_state(64, 128, seed=1, lmax=12, amp=2e-2, shear=2e-2)
    tau = 5e-4
    dt = oracle.suggest_dt(64, 128, tau)
    s = Solver(64, 128, tau, dt, storage=storage, q=3)
    s.init_fields(*st)
    s.step(30)
    fg = s.populations()
    s.close()
    fr = oracle.step(oracle.init(*st, q=3), 30, tau=tau, dt=dt, threads=THREADS)
    V, W1 = oracle.quadrature(3)
    dev = fr - np.outer(W1, W1).reshape(9)[:, None, None]
    assert np.abs(fg - fr).max() <= bound * np.abs(dev).max()


def test_d2q9_batches_and_diagnostics():
    from paper_2504_15574_amd import Ensemble, Solver, VlbmError, vlbm_step_batch
    st = W.random_state(24, 48, seed=5, du=0.05, smooth=False)
    a = Solver(24, 48, 2e-3, q=3, storage="f32")
    b = Solver(24, 48, 2e-3, q=3, storage="f32")
    c = Solver(24, 48, 2e-3, q=4, storage="f32")
    for s in (a, b, c):
        s.init_fields(*st)
    with pytest.raises(VlbmError):
        vlbm_step_batch([a.ctx, c.ctx], 1)          # mixed quadrature orders
    Ensemble([a]).step(3)
    b.step(3)
    assert np.array_equal(a.populations(), b.populations())
    d = Solver(24, 48, 2e-3, q=3)
    d.init_fields(*st)
    d.step(2)
    f = d.populations()
    dg = d.diagnostics()
    assert np.allclose(dg, oracle.diagnostics(f), rtol=1e-12, atol=1e-15)
    _, ut, up, _ = oracle.moments(f)
    assert np.abs(d.vorticity() - oracle.vorticity(ut, up)).max() < 1e-10
    for s in (a, b, c, d):
        s.close()
