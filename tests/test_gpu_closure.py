"""Learned-closure kernels against the FP64 closure oracle (GPU).

Each convolution is checked on its own, fed with the GPU's own bf16 inputs and
the bf16-rounded weights, so that only the FP32 accumulation order separates
the two sides; the whole network's gradient is then checked end to end
against the oracle in FP64, to the accuracy bf16 activations allow.
"""
import numpy as np
import pytest

import oracle
from oracle import closure_oracle as CO
from paper_2504_15574_amd.closure import LAYERS

CIN = LAYERS[0][1][0]      # the network's input channels (rho - 1, u_theta, u_phi, T - 1)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)
    from paper_2504_15574_amd import load
    load()


def _setup(H, W, Bt, seed):
    import torch
    from paper_2504_15574_amd.closure import ClosureNet, f64_to_bf16_bits
    rng = np.random.default_rng(seed)
    net = ClosureNet(H, W, Bt, seed=seed)
    params = CO.init_params(rng, cin=CIN)
    params = [p + 0.05 * rng.normal(size=p.shape) for p in params]
    net.set_params(params)
    x = np.zeros((Bt, H, W, 8))
    x[..., :CIN] = rng.normal(size=(Bt, H, W, CIN))
    xb = torch.from_numpy(f64_to_bf16_bits(x).reshape(-1)).cuda()
    net.x[: xb.numel()].copy_(xb)
    return net, rng


def _f32(t, shape):
    return t.cpu().numpy()[: int(np.prod(shape))].reshape(shape).astype(np.float64)


def _b16(t, shape):
    from paper_2504_15574_amd.closure import bf16_to_f64
    return bf16_to_f64(t)[: int(np.prod(shape))].reshape(shape)


GRIDS = [(8, 16, 1, 0), (12, 32, 3, 1), (2, 16, 2, 2)]


@pytest.mark.parametrize("H,W,Bt,seed", GRIDS)
def test_each_convolution_matches_the_oracle(H, W, Bt, seed):
    import torch
    net, _ = _setup(H, W, Bt, seed)
    net.forward(Bt)
    torch.cuda.synchronize()
    nbr, cross = CO.neighbours(H, W)
    pb = net.bf16_params()
    x = _b16(net.x, (Bt, H, W, 8))[..., :CIN]
    ins = [x, _b16(net.a[0], (Bt, H, W, 32)), _b16(net.a[1], (Bt, H, W, 32))]
    for li, co in enumerate((32, 32, 16)):
        z = _f32(net.z[li], (Bt, H, W, co))
        ref = CO.conv_forward(ins[li], pb[2 * li], pb[2 * li + 1], nbr, cross,
                              (1, 2) if li == 0 else ())
        rco = ref.shape[-1]
        scale = np.abs(ref).max()
        assert np.abs(z[..., :rco] - ref).max() <= 2e-6 * scale, li
        assert np.all(z[..., rco:] == 0.0)
        a = _b16(net.a[li], (Bt, H, W, co))
        from paper_2504_15574_amd.closure import f64_to_bf16_bits
        want = f64_to_bf16_bits(np.maximum(z, 0) if li < 2 else z).view(np.uint16)
        got = net.a[li].cpu().numpy()[: want.size].view(np.uint16).reshape(want.shape)
        assert np.array_equal(got, want), li


@pytest.mark.parametrize("H,W,Bt,seed", GRIDS)
def test_loss_and_each_gradient_match_the_oracle(H, W, Bt, seed):
    import torch
    net, rng = _setup(H, W, Bt, seed)
    tgt = rng.normal(size=(Bt, H, W, 3))
    tg = torch.from_numpy(tgt.astype(np.float32).reshape(-1)).cuda()
    net.forward(Bt)
    loss = net.loss(Bt, tg)
    net.backward(Bt)
    torch.cuda.synchronize()
    nbr, cross = CO.neighbours(H, W)
    pb = net.bf16_params()
    z3 = _f32(net.z[2], (Bt, H, W, 16))[..., :3]
    lref, gref = CO.loss_and_grad(z3, tgt, H)
    assert abs(loss - lref) <= 1e-5 * lref
    dz3 = _b16(net.dz[2], (Bt, H, W, 16))
    assert np.abs(dz3[..., :3] - gref).max() <= 4e-3 * np.abs(gref).max()
    assert np.all(dz3[..., 3:] == 0)
    ins = [_b16(net.x, (Bt, H, W, 8))[..., :CIN], _b16(net.a[0], (Bt, H, W, 32)),
           _b16(net.a[1], (Bt, H, W, 32))]
    dzs = [_b16(net.dz[0], (Bt, H, W, 32)), _b16(net.dz[1], (Bt, H, W, 32)), dz3[..., :3]]
    zs = [_f32(net.z[0], (Bt, H, W, 32)), _f32(net.z[1], (Bt, H, W, 32))]
    for li, (ci, co) in enumerate(((8, 32), (32, 32), (32, 16))):
        dx, dw, db = CO.conv_backward(ins[li], pb[2 * li], dzs[li], nbr, cross,
                                      (1, 2) if li == 0 else ())
        gw = net.gw[li].cpu().numpy().reshape(co, 9, ci).astype(np.float64)
        rco, rci = dw.shape[0], dw.shape[2]
        assert np.abs(gw[:rco, :, :rci] - dw).max() <= 1e-5 * np.abs(dw).max(), li
        assert np.all(gw[rco:] == 0) and np.all(gw[:, :, rci:] == 0)
        gb = net.gb[li].cpu().numpy().astype(np.float64)
        assert np.abs(gb[:rco] - db).max() <= 1e-5 * max(np.abs(db).max(), 1e-30), li
        if li > 0:
            want = dx * (zs[li - 1] > 0)
            got = dzs[li - 1]
            assert np.abs(got - want).max() <= 4e-3 * np.abs(want).max(), li


def test_network_gradient_matches_the_oracle_end_to_end():
    import torch
    H, W, Bt = 10, 32, 2
    net, rng = _setup(H, W, Bt, 7)
    tgt = 0.1 * rng.normal(size=(Bt, H, W, 3))
    tg = torch.from_numpy(tgt.astype(np.float32).reshape(-1)).cuda()
    net.forward(Bt)
    net.loss(Bt, tg)
    net.backward(Bt)
    torch.cuda.synchronize()
    nbr, cross = CO.neighbours(H, W)
    pb = net.bf16_params()
    x = _b16(net.x, (Bt, H, W, 8))[..., :CIN]
    z, cache = CO.net_forward(pb, x, nbr, cross)
    _, dz = CO.loss_and_grad(z, tgt, H)
    grads = CO.net_backward(pb, cache, dz, nbr, cross)
    for li, ((ci, co), (rci, rco)) in enumerate(LAYERS):
        gw = net.gw[li].cpu().numpy().reshape(co, 9, ci)[:rco, :, :rci]
        gb = net.gb[li].cpu().numpy()[:rco]
        rw = np.linalg.norm(gw - grads[2 * li]) / np.linalg.norm(grads[2 * li])
        rb = np.linalg.norm(gb - grads[2 * li + 1]) / np.linalg.norm(grads[2 * li + 1])
        print(f"  layer {li}: weight-gradient rel L2 {rw:.2e}, bias {rb:.2e}")
        assert rw < 3e-2 and rb < 3e-2


def test_adam_matches_the_oracle():
    import torch
    H, W, Bt = 8, 16, 1
    net, rng = _setup(H, W, Bt, 3)
    tg = torch.from_numpy(rng.normal(size=H * W * 3 * Bt).astype(np.float32)).cuda()
    p0 = [t.cpu().numpy().astype(np.float64) for t in net.master]
    for step in (1, 2):
        net.forward(Bt)
        net.loss(Bt, tg)
        net.backward(Bt)
        g = [t.cpu().numpy().astype(np.float64) for t in net.gw]
        m = [t[0].cpu().numpy().astype(np.float64) for t in net.m]
        v = [t[0].cpu().numpy().astype(np.float64) for t in net.v]
        net.adam(1e-3)
        torch.cuda.synchronize()
        for li in range(3):
            want, _, _ = CO.adam_step(p0[li], g[li], m[li], v[li], step, 1e-3)
            got = net.master[li].cpu().numpy().astype(np.float64)
            assert np.abs(got - want).max() <= 1e-6 * max(np.abs(want).max(), 1e-3)
            p0[li] = got


def test_box_filter_matches_the_oracle():
    import torch
    from paper_2504_15574_amd.closure import vlbm_box_filter
    rng = np.random.default_rng(4)
    Bt, Hf, Wf, f = 3, 24, 48, 4
    fields = [1 + 0.1 * rng.random((Bt, Hf, Wf)), rng.normal(size=(Bt, Hf, Wf)), rng.normal(size=(Bt, Hf, Wf))]
    dev = [torch.from_numpy(a).cuda() for a in fields]
    out = [torch.zeros(Bt * (Hf // f) * (Wf // f), dtype=torch.float64, device="cuda") for _ in range(3)]
    vlbm_box_filter(Hf, Wf, f, Bt, *dev, *out)
    torch.cuda.synchronize()
    for b in range(Bt):
        ref = CO.box_filter(fields[0][b], fields[1][b], fields[2][b], f)
        for o, r in zip(out, ref):
            got = o.cpu().numpy().reshape(Bt, Hf // f, Wf // f)[b]
            assert np.abs(got - r).max() <= 1e-13 * np.abs(r).max()


def test_moment_correction_keeps_the_non_equilibrium_part():
    import workloads as W
    from paper_2504_15574_amd import Solver
    nt, nph = 16, 32
    st = W.random_state(nt, nph, seed=5, du=0.05)
    s = Solver(nt, nph, 1e-3, 1e-3)
    s.init_fields(*st)
    s.step(3)
    f0 = s.populations()
    rng = np.random.default_rng(6)
    d = [1e-3 * rng.normal(size=(nt, nph)) for _ in range(3)]
    s.correct_moments(*d)
    f1 = s.populations()
    s.close()
    r, ut, up = oracle.moments(f0)[:3]
    want = f0 + oracle.init(r + d[0], ut + d[1], up + d[2]) - oracle.init(r, ut, up)
    assert np.abs(f1 - want).max() <= 1e-14 * np.abs(f0).max()
    r1, u1, v1 = oracle.moments(f1)[:3]
    assert np.abs(r1 - r - d[0]).max() < 1e-13 and np.abs(u1 - ut - d[1]).max() < 1e-12


def test_training_reduces_the_loss():
    # Fit a fixed smooth target (a 3x3-stencil function of the input with the
    # pole padding) from random inputs: 300 Adam steps cut the loss tenfold.
    import torch
    H, W, Bt = 16, 32, 8
    net, rng = _setup(H, W, Bt, 9)
    from paper_2504_15574_amd.closure import f64_to_bf16_bits
    nbr, cross = CO.neighbours(H, W)
    teacher = CO.init_params(np.random.default_rng(123), hidden=8, cin=CIN)
    x = np.zeros((Bt, H, W, 8))
    x[..., :CIN] = rng.normal(size=(Bt, H, W, CIN))
    net.x[: x.size].copy_(torch.from_numpy(f64_to_bf16_bits(x).reshape(-1)).cuda())
    tgt, _ = CO.net_forward(teacher, x[..., :CIN], nbr, cross)
    tgt = tgt / np.abs(tgt).max()
    tg = torch.from_numpy(tgt.astype(np.float32).reshape(-1)).cuda()
    losses = []
    for it in range(300):
        net.forward(Bt)
        losses.append(net.loss(Bt, tg))
        net.backward(Bt)
        net.adam(3e-3)
    print(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.1 * losses[0]
