"""Throughput of the learned-closure network kernels on one device.

Runs the training step of the 3-layer 3x3 CNN (forward through the three
convolutions, loss, data and weight gradients, Adam) on a batch of random
inputs and prints one JSON line with the mean device time per call of each
entry point (HIP events on the network's stream) and the matrix-core rate of
the convolutions: dense multiply-adds of the 3x3 taps over the padded
channels, 2 * P * 9 * CIN * COUT flop per forward call (P pixels), the same
for the data gradient and for the weight gradient.

    python -m paper_2504_15574_amd.closure_bench --grid 128x256 --batch 16 --iters 20
"""
from __future__ import annotations

import argparse
import json

import numpy as np

BF16_PEAK_TFLOPS = 2500.0     # MI355X dense BF16 matrix-core peak (published)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--grid", default="128x256", help="n_theta x n_phi (n_phi a multiple of 16)")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--iters", type=int, default=20)
    a = ap.parse_args(argv)
    H, W = (int(x) for x in a.grid.split("x"))
    import torch
    from .closure import LAYERS, VECTOR_MASK_IN, ClosureNet, _ck, _ptr, f64_to_bf16_bits, lib
    torch.cuda.set_device(0)
    Bt = a.batch
    P = Bt * H * W
    net = ClosureNet(H, W, Bt, seed=1)
    rng = np.random.default_rng(1)
    x = np.zeros((P, 8))
    x[:, :LAYERS[0][1][0]] = rng.normal(size=(P, LAYERS[0][1][0]))
    net.x.copy_(torch.from_numpy(f64_to_bf16_bits(x).reshape(-1)).cuda())
    tgt = torch.from_numpy((0.1 * rng.normal(size=P * 3)).astype(np.float32)).cuda()
    L = lib()
    stream = torch.cuda.current_stream()
    times = {}

    def timed(name, fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        times.setdefault(name, []).append(e0.elapsed_time(e1))

    for it in range(a.iters + 2):
        for li, ((ci, co), _) in enumerate(LAYERS):
            src = net.x if li == 0 else net.a[li - 1]
            timed(f"conv_forward_{ci}x{co}", lambda: _ck(L.vlbm_clo_conv_forward(
                net.ctx, ci, co, Bt, _ptr(src), _ptr(net.w[li]), _ptr(net.bias[li]),
                VECTOR_MASK_IN if li == 0 else 0, 1 if li < 2 else 0, _ptr(net.z[li]),
                _ptr(net.a[li])), "forward"))
        timed("loss", lambda: net.loss(Bt, tgt))
        for li in (2, 1, 0):
            (ci, co), _ = LAYERS[li]
            src = net.x if li == 0 else net.a[li - 1]
            timed(f"conv_backward_weight_{ci}x{co}", lambda: _ck(L.vlbm_clo_conv_backward_weight(
                net.ctx, ci, co, Bt, _ptr(src), _ptr(net.dz[li]), VECTOR_MASK_IN if li == 0 else 0,
                _ptr(net.gw[li]), _ptr(net.gb[li])), "backward_weight"))
            if li > 0:
                timed(f"conv_backward_data_{ci}x{co}", lambda: _ck(L.vlbm_clo_conv_backward_data(
                    net.ctx, ci, co, Bt, _ptr(net.dz[li]), _ptr(net.wt[li]), _ptr(net.z[li - 1]),
                    _ptr(net.dz[li - 1])), "backward_data"))
        timed("adam_and_pack", lambda: net.adam(1e-4))
    out = {"grid": f"{H}x{W}", "batch": Bt, "pixels": P, "iters": a.iters, "calls": {}}
    for name, v in times.items():
        ms = float(np.mean(v[2:]))            # the first two iterations warm up
        e = {"ms_per_call": round(ms, 4)}
        if name.startswith("conv_"):
            ci, co = (int(t) for t in name.rsplit("_", 1)[1].split("x"))
            flop = 2.0 * P * 9 * ci * co
            e["tflops"] = round(flop / (ms * 1e-3) / 1e12, 2)
            e["frac_of_bf16_peak"] = round(flop / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4)
        out["calls"][name] = e
    net.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
