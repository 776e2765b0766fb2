"""The learned closure end to end on the GPU: fine runs generate the training
data, the library's kernels train the network, and on held-out seeds the
coarse run with the closure tracks the filtered fine run better than the plain
coarse run, at a small fraction of the fine run's cost."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    from paper_2504_15574_amd import load
    load()


def test_trained_closure_beats_the_plain_coarse_run():
    from paper_2504_15574_amd.closure_train import Config, run
    cfg = Config(intervals=40, iters=1000, train_seeds=list(range(1000, 1016)),
                 eval_seeds=list(range(2000, 2004)))
    res = run(cfg, log=print)
    c, n = res["coarse"], res["closure"]
    last = lambda r, key: r["errors"][key][-1][1]
    print(f"  vorticity rel L2: coarse {last(c, 'vorticity'):.3f}, closure {last(n, 'vorticity'):.3f}")
    print(f"  spectrum |log10| : coarse {last(c, 'spectrum_dex'):.4f}, closure {last(n, 'spectrum_dex'):.4f}")
    print(f"  cost: fine / closure run = {n['cost_ratio_fine_over_this']:.1f}")
    assert res["loss_first_last"][1] < 0.3 * res["loss_first_last"][0]
    assert last(n, "vorticity") < 0.8 * last(c, "vorticity")
    assert last(n, "u") < 0.8 * last(c, "u")
    assert last(n, "spectrum_dex") < 0.5 * last(c, "spectrum_dex")
    assert n["cost_ratio_fine_over_this"] >= 10.0
