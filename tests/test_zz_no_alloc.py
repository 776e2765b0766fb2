"""The no-allocation entry point vlbm_diagnostics_static, through the C ABI,
against vlbm_diagnostics on the same state (two calls in a row, the second on
a smaller grid), plus its argument checks."""
import numpy as np
import pytest

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


def _compare(d_ctx, d_static):
    # sums (mass, energies, angular momentum): the two reductions differ only
    # in where rho0 enters (deviations vs full populations) and in the last bit
    # of sin(theta); extrema and the non-finite count agree to rounding
    assert np.allclose(d_static[[0, 1, 2, 3]], d_ctx[[0, 1, 2, 3]], rtol=1e-12, atol=1e-18)
    assert d_static[4] == d_ctx[4] == 0
    assert np.allclose(d_static[5:], d_ctx[5:], rtol=1e-13)


def test_static_diagnostics_match_the_context_diagnostics():
    import torch
    from paper_2504_15574_amd import Solver, vlbm_diagnostics_static, vlbm_get_populations
    stream = torch.cuda.current_stream()
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    for nt, nph, storage, R, seed in ((64, 128, "f64", 1.0, 1), (24, 48, "f32", 1.7, 2)):
        print(f"[case] static diagnostics {storage} {nt}x{nph} R={R}", flush=True)
        s = Solver(nt, nph, 2e-3, storage=storage, radius=R, stream=stream)
        s.init_fields(*W.random_state(nt, nph, seed=seed, du=0.05, dT=0.05))
        s.step(5)
        d_ctx = s.diagnostics()
        f = torch.empty(16 * nt * nph, dtype=torch.float64, device="cuda")
        vlbm_get_populations(s.ctx, f.data_ptr(), 1)
        out.fill_(-1.0)
        vlbm_diagnostics_static(nt, nph, 4, R, f.data_ptr(), out.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        _compare(d_ctx, out.cpu().numpy())
        # a non-finite population is counted
        f[3 * nt * nph + 5] = float("nan")
        vlbm_diagnostics_static(nt, nph, 4, R, f.data_ptr(), out.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        assert out[4].item() == 1.0
        s.close()


def test_static_diagnostics_reject_bad_arguments():
    import torch
    from paper_2504_15574_amd import VlbmError, vlbm_diagnostics_static
    f = torch.zeros(16 * 8 * 16, dtype=torch.float64, device="cuda")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    with pytest.raises(VlbmError, match="static scratch"):
        vlbm_diagnostics_static(122875, 2, 4, 1.0, f.data_ptr(), out.data_ptr())
    with pytest.raises(VlbmError):
        vlbm_diagnostics_static(8, 16, 5, 1.0, f.data_ptr(), out.data_ptr())
    with pytest.raises(VlbmError):
        vlbm_diagnostics_static(8, 16, 4, 1.0, 0, out.data_ptr())
    with pytest.raises(VlbmError):
        vlbm_diagnostics_static(8, 16, 4, -1.0, f.data_ptr(), out.data_ptr())
