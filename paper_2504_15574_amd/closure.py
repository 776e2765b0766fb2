"""Learned closure: ctypes binding of include/vlbm_closure.h and the network driver.

The network (three 3x3 convolutions, 3 -> 32 -> 32 -> 3 channels, ReLU) runs
entirely in the library's HIP kernels: BF16 MFMA convolutions, their data and
weight gradients, the loss and Adam.  PyTorch only provides device memory and
the stream.  Channel counts are padded for the matrix cores: the 3 input
channels to 8 and the 3 output channels to 16 (zero weights).
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np

from . import vlbm as B

_vp = ctypes.c_void_p
_i = ctypes.c_int
_f = ctypes.c_float
_d = ctypes.c_double

SIGNATURES = [
    ("vlbm_clo_workspace_bytes", ctypes.c_size_t, [_i, _i, _i]),
    ("vlbm_clo_create", _i, [_i, _i, _i, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    ("vlbm_clo_destroy", _i, [_vp]),
    ("vlbm_clo_conv_forward", _i, [_vp, _i, _i, _i, _vp, _vp, _vp, ctypes.c_uint32, _i, _vp, _vp]),
    ("vlbm_clo_conv_backward_data", _i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp]),
    ("vlbm_clo_conv_backward_weight", _i, [_vp, _i, _i, _i, _vp, _vp, ctypes.c_uint32, _vp, _vp]),
    ("vlbm_clo_loss", _i, [_vp, _i, _vp, _vp, _vp, _vp, ctypes.POINTER(_i)]),
    ("vlbm_clo_adam", _i, [_vp, _i, _vp, _vp, _vp, _vp, _i, _f, _f, _f, _f]),
    ("vlbm_clo_pack_weights", _i, [_vp, _i, _i, _vp, _vp, _vp]),
    ("vlbm_clo_pack_input", _i, [_vp, _i, _vp, _vp, _vp, _vp, _d, _d, _d, _vp]),
    ("vlbm_clo_unpack_output", _i, [_vp, _i, _vp, _d, _d, _vp, _vp, _vp]),
    ("vlbm_clo_pack_target", _i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _vp]),
    ("vlbm_box_filter", _i, [_i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
]

_bound = False


def lib():
    global _bound
    L = B.load()
    if not _bound:
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _ck(st, what):
    B._check(st, what)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _fld(t, n, dtype=None):
    """Device address of a caller's contiguous tensor holding at least n values
    of ``dtype`` (float64 unless given); the kernels touch n values there."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise B.VlbmError(f"expected a contiguous {dtype} device tensor")
    if t.numel() < n:
        raise B.VlbmError(f"expected at least {n} values, got a tensor of {t.numel()}")
    return t.data_ptr()


# layer shapes: (cin, cout) padded for MFMA, (cin, cout) of the network
LAYERS = [((8, 32), (4, 32)), ((32, 32), (32, 32)), ((32, 16), (32, 3))]
VECTOR_MASK_IN = 0b110      # input channels 1, 2 are u_theta, u_phi (0: rho - 1, 3: T - 1)


def kpad(cin):
    return (9 * cin + 31) // 32 * 32


def vlbm_box_filter(n_theta_f, n_phi_f, factor, batch, rho, ut, up, rc, uc, vc, stream=None):
    """Coarse-grain FP64 device fields (torch tensors) by factor x factor boxes."""
    import torch
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    nf = max(batch, 0) * max(n_theta_f, 0) * max(n_phi_f, 0)
    nc = nf // (factor * factor) if factor > 0 else 0
    _ck(lib().vlbm_box_filter(n_theta_f, n_phi_f, factor, batch, _fld(rho, nf), _fld(ut, nf), _fld(up, nf),
                              _fld(rc, nc), _fld(uc, nc), _fld(vc, nc), s), "vlbm_box_filter")


class ClosureNet:
    """The 3-layer CNN with its parameters, optimiser state and activations on
    the device, for batches of up to ``max_batch`` fields on one grid."""

    def __init__(self, n_theta, n_phi, max_batch, seed=0, stream=None):
        import torch
        lib()
        self.H, self.W, self.max_batch = int(n_theta), int(n_phi), int(max_batch)
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream().cuda_stream if stream is None else stream
        nb = lib().vlbm_clo_workspace_bytes(self.H, self.W, self.max_batch)
        if nb == 0:
            raise B.VlbmError(f"closure grid {n_theta}x{n_phi} (batch {max_batch}) not supported")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.dev)
        out = _vp()
        _ck(lib().vlbm_clo_create(self.H, self.W, self.max_batch, _vp(self.stream),
                                  _vp(self.ws.data_ptr()), nb, ctypes.byref(out)), "vlbm_clo_create")
        self.ctx = out.value
        P = self.H * self.W * self.max_batch
        f32, i16 = dict(dtype=torch.float32, device=self.dev), dict(dtype=torch.int16, device=self.dev)
        self.master, self.bias, self.w, self.wt = [], [], [], []
        self.m, self.v = [], []
        self.gw, self.gb = [], []
        for (ci, co), _ in LAYERS:
            self.master.append(torch.zeros(co * 9 * ci, **f32))
            self.bias.append(torch.zeros(co, **f32))
            self.w.append(torch.zeros(co * kpad(ci), **i16))
            self.wt.append(torch.zeros(9 * ci * co, **i16))
            self.gw.append(torch.zeros(co * 9 * ci, **f32))
            self.gb.append(torch.zeros(co, **f32))
            self.m.append([torch.zeros(co * 9 * ci, **f32), torch.zeros(co, **f32)])
            self.v.append([torch.zeros(co * 9 * ci, **f32), torch.zeros(co, **f32)])
        self.x = torch.zeros(P * 8, **i16)
        self.z = [torch.zeros(P * co, **f32) for (_, co), _ in LAYERS]
        self.a = [torch.zeros(P * co, **i16) for (_, co), _ in LAYERS]
        self.dz = [torch.zeros(P * co, **i16) for (_, co), _ in LAYERS]
        self.lpart = torch.zeros((P + 255) // 256, **f32)
        self.step_count = 0
        self.set_params(init_params(np.random.default_rng(seed)))

    # ---- parameters (oracle layout: w [Cout, 9, Cin], b [Cout]) -------------
    def set_params(self, params):
        import torch
        for li, ((ci, co), (rci, rco)) in enumerate(LAYERS):
            w = np.zeros((co, 9, ci), np.float32)
            w[:rco, :, :rci] = params[2 * li]
            b = np.zeros(co, np.float32)
            b[:rco] = params[2 * li + 1]
            self.master[li].copy_(torch.from_numpy(w.reshape(-1)))
            self.bias[li].copy_(torch.from_numpy(b))
        self._pack()

    def get_params(self):
        out = []
        for li, ((ci, co), (rci, rco)) in enumerate(LAYERS):
            w = self.master[li].cpu().numpy().reshape(co, 9, ci)[:rco, :, :rci].astype(np.float64)
            out += [w, self.bias[li].cpu().numpy()[:rco].astype(np.float64)]
        return out

    def bf16_params(self):
        """The parameters as the matrix cores see them (weights rounded to bf16)."""
        out = []
        for li, ((ci, co), (rci, rco)) in enumerate(LAYERS):
            w = bf16_to_f64(self.w[li]).reshape(co, kpad(ci))[:, :9 * ci].reshape(co, 9, ci)
            out += [w[:rco, :, :rci], self.bias[li].cpu().numpy()[:rco].astype(np.float64)]
        return out

    def _pack(self):
        for li, ((ci, co), _) in enumerate(LAYERS):
            _ck(lib().vlbm_clo_pack_weights(self.ctx, ci, co, _ptr(self.master[li]), _ptr(self.w[li]),
                                            _ptr(self.wt[li])), "vlbm_clo_pack_weights")

    # ---- forward / backward --------------------------------------------------
    def pack_input(self, batch, rho, ut, up, s_rho, s_u, T=None, s_T=0.0):
        """Input channels (rho - 1) s_rho, u s_u, (T - 1) s_T (0 without T)."""
        n = max(batch, 0) * self.H * self.W
        _ck(lib().vlbm_clo_pack_input(self.ctx, batch, _fld(rho, n), _fld(ut, n), _fld(up, n),
                                      _fld(T, n) if T is not None else None, float(s_rho), float(s_u),
                                      float(s_T), _ptr(self.x)), "vlbm_clo_pack_input")

    def forward(self, batch, x=None):
        """Run the three layers on self.x (or the given bf16 [P][8] tensor);
        returns the FP32 output tensor [P][16] (channels 0..2 used)."""
        xin = self.x if x is None else x
        L = lib()
        for li, ((ci, co), _) in enumerate(LAYERS):
            src = xin if li == 0 else self.a[li - 1]
            _ck(L.vlbm_clo_conv_forward(self.ctx, ci, co, batch, _ptr(src), _ptr(self.w[li]),
                                        _ptr(self.bias[li]), VECTOR_MASK_IN if li == 0 else 0,
                                        1 if li < 2 else 0, _ptr(self.z[li]), _ptr(self.a[li])),
                "vlbm_clo_conv_forward")
        return self.z[2]

    def loss(self, batch, target):
        """Weighted MSE of the last forward output against target (FP32 [P][3]);
        fills the output gradient.  Returns the loss (host float, synchronises)."""
        n = _i()
        _ck(lib().vlbm_clo_loss(self.ctx, batch, _ptr(self.z[2]), _ptr(target), _ptr(self.dz[2]),
                                _ptr(self.lpart), ctypes.byref(n)), "vlbm_clo_loss")
        return float(self.lpart[:n.value].double().sum().item())

    def backward(self, batch, x=None):
        """Gradients of the loss set by loss() into self.gw / self.gb."""
        xin = self.x if x is None else x
        L = lib()
        for li in (2, 1, 0):
            (ci, co), _ = LAYERS[li]
            src = xin if li == 0 else self.a[li - 1]
            _ck(L.vlbm_clo_conv_backward_weight(self.ctx, ci, co, batch, _ptr(src), _ptr(self.dz[li]),
                                                VECTOR_MASK_IN if li == 0 else 0, _ptr(self.gw[li]),
                                                _ptr(self.gb[li])), "vlbm_clo_conv_backward_weight")
            if li > 0:
                _ck(L.vlbm_clo_conv_backward_data(self.ctx, ci, co, batch, _ptr(self.dz[li]),
                                                  _ptr(self.wt[li]), _ptr(self.z[li - 1]),
                                                  _ptr(self.dz[li - 1])), "vlbm_clo_conv_backward_data")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        L = lib()
        for li in range(3):
            for p, g, m, v in ((self.master[li], self.gw[li], self.m[li][0], self.v[li][0]),
                               (self.bias[li], self.gb[li], self.m[li][1], self.v[li][1])):
                _ck(L.vlbm_clo_adam(self.ctx, p.numel(), _ptr(p), _ptr(g), _ptr(m), _ptr(v),
                                    self.step_count, lr, beta1, beta2, eps), "vlbm_clo_adam")
        self._pack()

    def pack_target(self, batch, a, b, o_rho, o_u, target):
        """target = (a - b) / (o_rho, o_u, o_u) from (rho, u_theta, u_phi) field triples."""
        import torch
        n = max(batch, 0) * self.H * self.W
        _ck(lib().vlbm_clo_pack_target(self.ctx, batch, *[_fld(t, n) for t in a], *[_fld(t, n) for t in b],
                                       float(o_rho), float(o_u), _fld(target, 3 * n, torch.float32)),
            "vlbm_clo_pack_target")

    def unpack_output(self, batch, o_rho, o_u, drho, dut, dup):
        n = max(batch, 0) * self.H * self.W
        _ck(lib().vlbm_clo_unpack_output(self.ctx, batch, _ptr(self.z[2]), float(o_rho), float(o_u),
                                         _fld(drho, n), _fld(dut, n), _fld(dup, n)), "vlbm_clo_unpack_output")

    def close(self):
        if getattr(self, "ctx", None):
            lib().vlbm_clo_destroy(_vp(self.ctx))
            self.ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():   # the HIP runtime may already be torn down
            return
        try:
            self.close()
        except Exception:
            pass


def init_params(rng, hidden=32, cin=4):
    """He-normal weights (the last layer scaled by 0.1), zero biases."""
    shapes = [(hidden, 9, cin), (hidden, 9, hidden), (3, 9, hidden)]
    ps = []
    for i, s in enumerate(shapes):
        std = np.sqrt(2.0 / (9 * s[2])) * (1.0 if i < 2 else 0.1)
        ps += [rng.normal(0.0, std, size=s), np.zeros(s[0])]
    return ps


def f64_to_bf16_bits(a):
    """Round-to-nearest-even bf16 bits (int16 array) of float values."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)
    return r.view(np.int16)


def bf16_to_f64(t):
    """Values of a bf16 tensor (torch int16, any device) as float64 numpy."""
    h = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return h.view(np.float32).astype(np.float64)
