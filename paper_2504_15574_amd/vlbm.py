"""Thin ctypes binding of ``libvlbm.so`` (the C ABI declared in include/vlbm.h).

The functions below carry the C names and only marshal arguments; every step
of the update runs in the library's HIP kernels.  ``Solver`` adds the one
convenience the ABI leaves to the caller: device memory for the workspace and
the stream, both taken from PyTorch (``torch.cuda``).  There is no CPU
fallback: without the built library or a HIP device the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvlbm.so")

ABI_VERSION = 1
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_UNSUPPORTED", 3: "ERR_ALLOC", 4: "ERR_DEVICE",
          5: "ERR_UNSTABLE"}
ADV_WENO5 = 0
ADVECTION = {"weno5": 0, "u1": 1, "u2": 2, "u3": 3}
ADV_KOMISSAROV = 0x100

# (name, restype, argtypes) of every symbol include/vlbm.h declares
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class vlbm_params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("n_theta", ctypes.c_int32),
        ("n_phi", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("radius", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("advection", ctypes.c_int32),
    ]


_P = ctypes.POINTER(vlbm_params)
SIGNATURES = [
    ("vlbm_workspace_bytes", ctypes.c_size_t, [_P]),
    ("vlbm_create", ctypes.c_int, [_P, _vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    ("vlbm_init_fields", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int]),
    ("vlbm_step", ctypes.c_int, [_vp, ctypes.c_int64]),
    ("vlbm_moments", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int]),
    ("vlbm_destroy", ctypes.c_int, [_vp]),
    ("vlbm_diagnostics", ctypes.c_int, [_vp, _dp]),
    ("vlbm_vorticity", ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    ("vlbm_get_populations", ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    ("vlbm_set_populations", ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    ("vlbm_suggest_dt", ctypes.c_double, [_P]),
    ("vlbm_stage_launches", ctypes.c_int64, [_vp]),
    ("vlbm_quadrature_f32", ctypes.c_int, [_vp, _vp, _dp]),
    ("vlbm_correct_moments", ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int]),
    ("vlbm_set_tile_shape", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    ("vlbm_step_batch", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int64]),
    ("vlbm_step_batch_persistent", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int64]),
    ("vlbm_set_barrier_spin_limit", ctypes.c_int, [ctypes.c_uint32]),
    ("vlbm_graph_create", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int64,
                                         ctypes.POINTER(_vp)]),
    ("vlbm_graph_create_persistent", ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int64,
                                                   ctypes.POINTER(_vp)]),
    ("vlbm_graph_launch", ctypes.c_int, [_vp]),
    ("vlbm_graph_check", ctypes.c_int, [_vp]),
    ("vlbm_graph_destroy", ctypes.c_int, [_vp]),
    ("vlbm_diagnostics_static", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_double, _vp, _vp, _vp]),
    ("vlbm_last_error", ctypes.c_char_p, []),
]

_lib = None


class VlbmError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise VlbmError(f"{path} is missing: build it with paper_2504_15574_amd/build.py")
        L = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int, what: str):
    if st != 0:
        msg = load().vlbm_last_error().decode(errors="replace")
        raise VlbmError(f"{what}: {STATUS.get(st, st)}: {msg}")


def make_params(n_theta, n_phi, tau, dt, storage="f64", radius=1.0, rho0=1.0, weno_eps=1e-6,
                q=4, scheme="weno5", komissarov=False) -> vlbm_params:
    adv = ADVECTION[scheme] | (ADV_KOMISSAROV if komissarov else 0)
    return vlbm_params(ABI_VERSION, int(n_theta), int(n_phi), int(q), float(radius), float(tau),
                       float(dt), float(rho0), float(weno_eps), STORAGE[storage], adv)


# ---- C-named wrappers (argument marshalling only) -------------------------------
def vlbm_workspace_bytes(p: vlbm_params) -> int:
    return int(load().vlbm_workspace_bytes(ctypes.byref(p)))


def vlbm_suggest_dt(p: vlbm_params) -> float:
    return float(load().vlbm_suggest_dt(ctypes.byref(p)))


def vlbm_quadrature_f32():
    """FP32 nodes (4), product weights (16) and the residuals of sum w = 1,
    sum w v_theta^2 = 1, sum w v_theta^4 = 3 and sum w v_theta^2 v_phi^2 = 1 on
    those FP32 values."""
    v = np.zeros(4, np.float32)
    w = np.zeros(16, np.float32)
    r = np.zeros(4)
    _check(load().vlbm_quadrature_f32(v.ctypes.data, w.ctypes.data, r.ctypes.data_as(_dp)),
           "vlbm_quadrature_f32")
    return v, w, r


def vlbm_create(p: vlbm_params, stream: int, workspace: int, nbytes: int) -> int:
    out = _vp()
    _check(load().vlbm_create(ctypes.byref(p), _vp(stream), _vp(workspace), nbytes,
                              ctypes.byref(out)), "vlbm_create")
    return out.value


def vlbm_init_fields(ctx, rho, ut, up, T, on_device: int):
    _check(load().vlbm_init_fields(_vp(ctx), _vp(rho), _vp(ut), _vp(up), _vp(T), on_device),
           "vlbm_init_fields")


def vlbm_step(ctx, n: int):
    _check(load().vlbm_step(_vp(ctx), int(n)), "vlbm_step")


def vlbm_moments(ctx, rho, ut, up, T, on_device: int):
    _check(load().vlbm_moments(_vp(ctx), _vp(rho), _vp(ut), _vp(up), _vp(T), on_device),
           "vlbm_moments")


def vlbm_correct_moments(ctx, drho, dut, dup, on_device: int):
    _check(load().vlbm_correct_moments(_vp(ctx), _vp(drho), _vp(dut), _vp(dup), on_device),
           "vlbm_correct_moments")


def vlbm_set_tile_shape(ctx, rows: int, cols: int):
    _check(load().vlbm_set_tile_shape(_vp(ctx), int(rows), int(cols)), "vlbm_set_tile_shape")


def vlbm_destroy(ctx):
    _check(load().vlbm_destroy(_vp(ctx)), "vlbm_destroy")


def vlbm_diagnostics(ctx, raise_unstable: bool = True) -> np.ndarray:
    out = np.zeros(8)
    st = load().vlbm_diagnostics(_vp(ctx), out.ctypes.data_as(_dp))
    if st == 5 and not raise_unstable:
        return out
    _check(st, "vlbm_diagnostics")
    return out


def vlbm_diagnostics_static(n_theta: int, n_phi: int, q: int, radius: float, f_dev: int,
                            out_dev: int, stream: int = 0):
    """vlbm_diagnostics_static: device pointers in, device pointer out, no
    allocation (asynchronous on `stream`)."""
    _check(load().vlbm_diagnostics_static(int(n_theta), int(n_phi), int(q), float(radius), _vp(f_dev),
                                          _vp(out_dev), _vp(stream)), "vlbm_diagnostics_static")


def vlbm_vorticity(ctx, om, on_device: int):
    _check(load().vlbm_vorticity(_vp(ctx), _vp(om), on_device), "vlbm_vorticity")


def vlbm_get_populations(ctx, f, on_device: int):
    _check(load().vlbm_get_populations(_vp(ctx), _vp(f), on_device), "vlbm_get_populations")


def vlbm_set_populations(ctx, f, on_device: int):
    _check(load().vlbm_set_populations(_vp(ctx), _vp(f), on_device), "vlbm_set_populations")


def vlbm_stage_launches(ctx) -> int:
    return int(load().vlbm_stage_launches(_vp(ctx)))


def _ctx_array(ctxs):
    return (_vp * len(ctxs))(*[_vp(c) for c in ctxs])


def vlbm_step_batch(ctxs, n: int):
    _check(load().vlbm_step_batch(_ctx_array(ctxs), len(ctxs), int(n)), "vlbm_step_batch")


def vlbm_step_batch_persistent(ctxs, n: int):
    _check(load().vlbm_step_batch_persistent(_ctx_array(ctxs), len(ctxs), int(n)),
           "vlbm_step_batch_persistent")


def vlbm_set_barrier_spin_limit(polls: int):
    _check(load().vlbm_set_barrier_spin_limit(int(polls)), "vlbm_set_barrier_spin_limit")


def vlbm_graph_create(ctxs, n: int) -> int:
    out = _vp()
    _check(load().vlbm_graph_create(_ctx_array(ctxs), len(ctxs), int(n), ctypes.byref(out)),
           "vlbm_graph_create")
    return out.value


def vlbm_graph_create_persistent(ctxs, n: int) -> int:
    out = _vp()
    _check(load().vlbm_graph_create_persistent(_ctx_array(ctxs), len(ctxs), int(n), ctypes.byref(out)),
           "vlbm_graph_create_persistent")
    return out.value


def vlbm_graph_check(graph):
    _check(load().vlbm_graph_check(_vp(graph)), "vlbm_graph_check")


def vlbm_graph_launch(graph):
    _check(load().vlbm_graph_launch(_vp(graph)), "vlbm_graph_launch")


def vlbm_graph_destroy(graph):
    _check(load().vlbm_graph_destroy(_vp(graph)), "vlbm_graph_destroy")


# ---- convenience object ---------------------------------------------------------
def _dptr(t, n):
    """Device address of a contiguous float64 device tensor of exactly n values
    (the kernels write n values there, so a shorter tensor is refused)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise VlbmError("expected a contiguous float64 device tensor")
    if t.numel() != n:
        raise VlbmError(f"expected {n} values, got a tensor of {t.numel()}")
    return t.data_ptr()


def _need_shape(a, shape, what):
    if a.shape != shape:
        raise VlbmError(f"{what}: expected shape {shape}, got {a.shape}")


def _host(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data


class Solver:
    """One vLBM run on the current HIP device.

    Workspace: a ``torch.uint8`` device tensor owned by this object; stream:
    ``torch.cuda.current_stream()`` at construction (or ``stream``)."""

    def __init__(self, n_theta, n_phi, tau, dt=None, storage="f64", radius=1.0, rho0=1.0,
                 weno_eps=1e-6, stream=None, scheme="weno5", komissarov=False, q=4):
        import torch
        if not torch.cuda.is_available():
            raise VlbmError("no HIP device visible to torch")
        load()
        self.n_theta, self.n_phi = int(n_theta), int(n_phi)
        p = make_params(n_theta, n_phi, tau, 1.0, storage, radius, rho0, weno_eps, q=q,
                        scheme=scheme, komissarov=komissarov)
        self.q = int(q)
        if dt is None:
            dt = vlbm_suggest_dt(p)
        p.dt = float(dt)
        self.params = p
        self.dt = float(dt)
        nbytes = vlbm_workspace_bytes(p)
        if nbytes == 0:
            raise VlbmError("invalid parameters: " + load().vlbm_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = vlbm_create(p, self.stream.cuda_stream, self.workspace.data_ptr(), nbytes)
        self.t = 0.0

    # fields: numpy (host) arrays [n_theta, n_phi]
    def init_fields(self, rho, ut, up, T=None):
        shape = (self.n_theta, self.n_phi)
        arrs = [_host(np.broadcast_to(a, shape)) for a in (rho, ut, up)]
        Ta = _host(np.broadcast_to(T, shape)) if T is not None else (None, None)
        vlbm_init_fields(self.ctx, arrs[0][1], arrs[1][1], arrs[2][1], Ta[1], 0)
        self.t = 0.0

    def step(self, n=1):
        vlbm_step(self.ctx, n)
        self.t += n * self.dt

    # fields already in device memory: contiguous FP64 torch tensors [n_theta, n_phi]
    def init_fields_device(self, rho, ut, up, T=None):
        n = self.n_theta * self.n_phi
        vlbm_init_fields(self.ctx, _dptr(rho, n), _dptr(ut, n), _dptr(up, n),
                         _dptr(T, n) if T is not None else None, 1)
        self.t = 0.0

    def moments_device(self, rho, ut, up, T=None):
        n = self.n_theta * self.n_phi
        vlbm_moments(self.ctx, _dptr(rho, n), _dptr(ut, n), _dptr(up, n),
                     _dptr(T, n) if T is not None else None, 1)

    def vorticity_device(self, omega):
        vlbm_vorticity(self.ctx, _dptr(omega, self.n_theta * self.n_phi), 1)

    def correct_moments_device(self, drho, dut, dup):
        n = self.n_theta * self.n_phi
        vlbm_correct_moments(self.ctx, _dptr(drho, n), _dptr(dut, n), _dptr(dup, n), 1)

    def moments(self, with_T=True):
        shape = (self.n_theta, self.n_phi)
        out = [np.empty(shape) for _ in range(4 if with_T else 3)]
        vlbm_moments(self.ctx, out[0].ctypes.data, out[1].ctypes.data, out[2].ctypes.data,
                     out[3].ctypes.data if with_T else None, 0)
        return tuple(out)

    def vorticity(self):
        om = np.empty((self.n_theta, self.n_phi))
        vlbm_vorticity(self.ctx, om.ctypes.data, 0)
        return om

    def populations(self):
        f = np.empty((self.q * self.q, self.n_theta, self.n_phi))
        vlbm_get_populations(self.ctx, f.ctypes.data, 0)
        return f

    def set_populations(self, f):
        f, ptr = _host(f)
        _need_shape(f, (self.q * self.q, self.n_theta, self.n_phi), "populations")
        vlbm_set_populations(self.ctx, ptr, 0)

    def correct_moments(self, drho, dut, dup):
        """Add (d_rho, d_u) to the moments through the equilibrium (host fields)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (drho, dut, dup)]
        for a in arrs:
            _need_shape(a, (self.n_theta, self.n_phi), "moment corrections")
        vlbm_correct_moments(self.ctx, arrs[0].ctypes.data, arrs[1].ctypes.data,
                             arrs[2].ctypes.data, 0)

    def diagnostics(self, raise_unstable=True):
        return vlbm_diagnostics(self.ctx, raise_unstable)

    def close(self):
        if getattr(self, "ctx", None):
            vlbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be gone: leave
        # the context to the process exit instead of calling into the library
        # (the check is bound at definition: module globals may be cleared then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Ensemble:
    """Independent runs advanced together (``vlbm_step_batch``).

    Runs may differ in grid, tau and dt; they share the storage format and the
    stream.  Two launch parameters never change a cell's arithmetic, so every
    choice gives the same bits: ``grouping`` splits the runs into launches
    (``"all"``: one launch per RK stage for everything, 64 runs per launch;
    ``"by_size"``: one launch per distinct grid; ``"single"``: one launch per
    run) and ``tile`` is the stage kernel's tile shape (15 x 16 or 7 x 32,
    rows x columns): one shape for every run, or, with ``"by_size"``, a dict
    {(n_theta, n_phi): shape} that lets each grid size use its own.
    ``autotune`` times the combinations and keeps the fastest.
    ``capture``/``replay`` record and replay a fixed number of steps as HIP
    graphs (one per launch group)."""

    GROUPINGS = ("all", "by_size", "single")
    TILES = ((15, 16), (7, 32))

    def __init__(self, solvers, grouping="all", tile=(15, 16)):
        self.solvers = list(solvers)
        self.graphs = []
        self.graph_steps = 0
        self.tile = None
        self.grouping = None
        self.configure(grouping, tile)

    @staticmethod
    def _size(s):
        return (s.n_theta, s.n_phi)

    def configure(self, grouping=None, tile=None):
        grouping = self.grouping if grouping is None else grouping
        tile = self.tile if tile is None else tile
        if grouping not in self.GROUPINGS:
            raise ValueError(grouping)
        if isinstance(tile, dict):
            if grouping != "by_size":
                raise ValueError("a tile shape per grid size needs grouping 'by_size'")
            tile = {tuple(k): tuple(v) for k, v in tile.items()}
            if set(tile) != {self._size(s) for s in self.solvers} or \
                    any(v not in self.TILES for v in tile.values()):
                raise ValueError(tile)
        else:
            tile = tuple(tile)
            if tile not in self.TILES:
                raise ValueError(tile)
        self.release()
        for s in self.solvers:
            vlbm_set_tile_shape(s.ctx, *(tile[self._size(s)] if isinstance(tile, dict) else tile))
        self.tile = tile
        self.grouping = grouping
        if grouping == "all":
            groups = [self.solvers]
        elif grouping == "single":
            groups = [[s] for s in self.solvers]
        else:
            by = {}
            for s in self.solvers:
                by.setdefault(self._size(s), []).append(s)
            groups = list(by.values())
        self.groups = [[s.ctx for s in g] for g in groups]
        self._group_sizes = [self._size(g[0]) for g in groups]

    def _step_size(self, ctxs, size, n):
        vlbm_step_batch(ctxs, n)
        for s in self.solvers:
            if self._size(s) == size:
                s.t += n * s.dt

    def tile_name(self):
        """The tile choice as text: "15x16", or "128x256:7x32,256x512:15x16"."""
        if isinstance(self.tile, dict):
            return ",".join(f"{k[0]}x{k[1]}:{v[0]}x{v[1]}" for k, v in sorted(self.tile.items()))
        return f"{self.tile[0]}x{self.tile[1]}"

    def set_grouping(self, grouping):
        self.configure(grouping=grouping)

    def _require_open(self):
        # the launch groups and graphs hold the runs' contexts: a closed run
        # would leave them pointing at freed state
        if any(getattr(s, "ctx", None) is None for s in self.solvers):
            raise VlbmError("a run of this ensemble has been closed")

    def step(self, n=1, persistent=False):
        """n steps of every run; ``persistent``: one cooperative launch per
        launch group carries all n steps (``vlbm_step_batch_persistent``;
        D2Q16, standard WENO-5 form; returns when done)."""
        self._require_open()
        for g in self.groups:
            if persistent:
                vlbm_step_batch_persistent(g, n)
            else:
                vlbm_step_batch(g, n)
        for s in self.solvers:
            s.t += n * s.dt

    def capture(self, steps, persistent=False):
        """Record ``steps`` steps as one HIP graph per launch group; with
        ``persistent`` each graph holds one persistent launch
        (``vlbm_graph_create_persistent``)."""
        self._require_open()
        self.release()
        make = vlbm_graph_create_persistent if persistent else vlbm_graph_create
        self.graphs = [make(g, steps) for g in self.groups]
        self.graph_steps = steps

    def check(self):
        """Wait for the last replay; raise if a persistent launch in it gave up
        at a grid barrier."""
        self._require_open()
        for g in self.graphs:
            vlbm_graph_check(g)

    def replay(self):
        self._require_open()
        for g in self.graphs:
            vlbm_graph_launch(g)
        for s in self.solvers:
            s.t += self.graph_steps * s.dt

    def release(self):
        for g in self.graphs:
            vlbm_graph_destroy(g)
        self.graphs = []

    def autotune(self, steps=10, groupings=GROUPINGS, tiles=TILES):
        """Time ``steps`` eager steps per (grouping, tile) combination (this
        advances the runs) and keep the fastest; with "by_size" and several
        grid sizes, also the combination of each size's fastest tile shape on
        its own launches.  Returns {"grouping/tile": ms per step}."""
        self._require_open()
        import torch

        def timed(fn):
            fn(1)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(self.solvers[0].stream)
            fn(steps)
            e1.record(self.solvers[0].stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        times = {}
        for t in tiles:
            for c in groupings:
                self.configure(c, t)
                times[(c, t)] = timed(self.step)
        sizes = {self._size(s) for s in self.solvers}
        if "by_size" in groupings and len(sizes) > 1 and len(tiles) > 1:
            per = {}
            for t in tiles:
                self.configure("by_size", t)
                for g, sz in zip(self.groups, self._group_sizes):
                    per[(sz, t)] = timed(lambda n, g=g, sz=sz: self._step_size(g, sz, n))
            mix = {sz: min(tiles, key=lambda t: per[(sz, t)]) for sz in sizes}
            if len(set(mix.values())) > 1:
                self.configure("by_size", mix)
                times[("by_size", tuple(sorted(mix.items())))] = timed(self.step)
        c, t = min(times, key=times.get)
        per_size = isinstance(t[0], tuple)
        self.configure(c, dict(t) if per_size else t)
        out = {}
        for (c, t), v in times.items():
            if isinstance(t[0], tuple):
                key = ",".join(f"{k[0]}x{k[1]}:{w[0]}x{w[1]}" for k, w in t)
            else:
                key = f"{t[0]}x{t[1]}"
            out[f"{c}/{key}"] = v
        return out

    def close(self):
        """Destroy the recorded graphs (the runs stay open; close them
        separately, after this)."""
        self.release()

    def __del__(self, _finalizing=sys.is_finalizing):
        # graph destruction calls the HIP runtime, which may already be torn
        # down at interpreter shutdown: skip it there (the process exit frees it)
        if _finalizing():
            return
        try:
            self.release()
        except Exception:
            pass
