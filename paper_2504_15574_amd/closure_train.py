"""Learned-closure experiment on the GPU: training data from filtered fine vLBM
runs, training with the library's network kernels, evaluation against fine runs.

Setting (all runs on one device, every step of every run in the library):
  fine     n_theta_c f x n_phi_c f cells, FP32 deviation store, dt_f = dt_c / fine_sub
           (the largest divisor of the coarse step within the fine grid's
           stability rule; near the poles it is set by the phi CFL limit)
  coarse   n_theta_c x n_phi_c cells, FP32 store, dt_c = tau (the BGK limit)
  flow     decaying turbulence: streamfunction with E(l) ~ l^-3, l <= lmax,
           rms |u| = urms, nu = tau (T0 = 1)
  filter   box averages of f x f fine cells (area and momentum weighted)

The closure acts once per interval of k coarse steps (k = 1: every step): the
coarse run advances k steps, the network maps its moments (rho - 1, u, T - 1)
to a correction (d_rho, d_u), and the correction enters the populations
through the equilibrium (vlbm_correct_moments).  Training pairs come from the
fine runs: the input is the coarse run's state one interval after it started
from the filtered fine state X_n (rho, u and the mass-weighted temperature),
the target the filtered fine state X_{n+1} minus that prediction.  A network
trained on such pairs alone only ever sees states one interval away from a
filtered fine state; in a rollout its own corrections move the state away from
that set, and with a correction every step the errors compound until the run
blows up.  So after the first fit the closure is rolled out on the training
seeds (rollout_rounds times), restarted from the filtered fine state every
rollout_steps coarse steps: the states it reaches, one interval after each
correction, become further inputs, with the filtered fine state at the same
time as target, and the network is trained on all pairs again.  A rollout
stops collecting once its targets leave the range the first fit was scaled
for (rms above rollout_cap output units), so a run that drifts far does not
swamp the loss.

Evaluation compares, on held-out seeds, the plain coarse run and the coarse run
with the closure against the filtered fine run: relative L2 of vorticity and of
velocity, and the vorticity spectrum (spherical-harmonic degree spectrum,
mean |log10| ratio over l = 1 .. n_theta_c / 2), with the cost of each per unit
of simulated time.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import asdict, dataclass, field, replace

import numpy as np


@dataclass
class Config:
    n_theta_c: int = 32
    n_phi_c: int = 64
    factor: int = 8
    tau: float = 2e-4
    k: int = 25                  # coarse steps per closure interval
    intervals: int = 40
    urms: float = 0.1
    lmax: int = 64
    batch: int = 16              # fine runs advanced by one launch per stage
    train_seeds: list = field(default_factory=lambda: list(range(1000, 1032)))
    eval_seeds: list = field(default_factory=lambda: list(range(2000, 2008)))
    iters: int = 1500
    rollout_rounds: int = 1      # refits on pairs collected from closure rollouts
    rollout_steps: int = 50      # coarse steps between restarts of those rollouts
    rollout_cap: float = 4.0     # largest rms target (output units) collected
    minibatch: int = 32
    lr: float = 2e-3
    seed: int = 0

    @property
    def dt_c(self):
        return self.tau

    @property
    def n_theta_f(self):
        return self.n_theta_c * self.factor

    @property
    def n_phi_f(self):
        return self.n_phi_c * self.factor


def fine_substeps(cfg):
    from .vlbm import make_params, vlbm_suggest_dt
    dmax = vlbm_suggest_dt(make_params(cfg.n_theta_f, cfg.n_phi_f, cfg.tau, 1.0))
    return max(1, math.ceil(cfg.dt_c / dmax * (1 + 1e-12)))


def _fields(n, H, W, c=3):
    import torch
    return [torch.zeros((n, H, W), dtype=torch.float64, device="cuda") for _ in range(c)]


class _Events:
    def __init__(self):
        import torch
        self.ms = 0.0
        self._t = torch

    def __enter__(self):
        self.e0 = self._t.cuda.Event(enable_timing=True)
        self.e1 = self._t.cuda.Event(enable_timing=True)
        self.e0.record()
        return self

    def __exit__(self, *a):
        self.e1.record()
        self.e1.synchronize()
        self.ms += self.e0.elapsed_time(self.e1)


def fine_filtered(cfg, seeds, storage="f32"):
    """Filtered fine states X[n] (n = 0..intervals) for the seeds: four FP64
    device tensors per interval (rho, u_theta, u_phi, T), each
    [len(seeds)][n_theta_c][n_phi_c]; T is the mass-weighted box average.  Also
    returns the fine cost in ms of device time per run per unit simulated time."""
    import workloads as W
    from .closure import vlbm_box_filter
    from .vlbm import Ensemble, Solver
    sub = fine_substeps(cfg)
    dt_f = cfg.dt_c / sub
    Hf, Wf, Hc, Wc = cfg.n_theta_f, cfg.n_phi_f, cfg.n_theta_c, cfg.n_phi_c
    N = len(seeds)
    X = [_fields(N, Hc, Wc, 4) for _ in range(cfg.intervals + 1)]
    clock = _Events()
    for i0 in range(0, N, cfg.batch):
        chunk = seeds[i0:i0 + cfg.batch]
        B = len(chunk)
        sols = [Solver(Hf, Wf, cfg.tau, dt_f, storage=storage) for _ in chunk]
        for s, sd in zip(sols, chunk):
            s.init_fields(*W.turbulence_state(Hf, Wf, seed=sd, lmax=cfg.lmax, urms=cfg.urms)[:3])
        ens = Ensemble(sols)
        mom = _fields(B, Hf, Wf, 4)
        spare = _fields(B, Hc, Wc, 1)[0]
        for n in range(cfg.intervals + 1):
            for b, s in enumerate(sols):
                s.moments_device(mom[0][b], mom[1][b], mom[2][b], mom[3][b])
            Xn = [x[i0:i0 + B] for x in X[n]]
            vlbm_box_filter(Hf, Wf, cfg.factor, B, *mom[:3], *Xn[:3])
            # (rho, T, T) through the same filter: the momentum-weighted channel
            # of T is its mass-weighted average
            vlbm_box_filter(Hf, Wf, cfg.factor, B, mom[0], mom[3], mom[3], spare, Xn[3], spare)
            if n < cfg.intervals:
                with clock:
                    ens.step(cfg.k * sub)
        for s in sols:
            s.close()
    t_sim = cfg.intervals * cfg.k * cfg.dt_c
    return X, clock.ms / (N * t_sim)


class CoarsePool:
    """B coarse runs advanced together (one launch per stage for all)."""

    def __init__(self, cfg, B):
        from .vlbm import Ensemble, Solver
        self.cfg, self.B = cfg, B
        self.sols = [Solver(cfg.n_theta_c, cfg.n_phi_c, cfg.tau, cfg.dt_c, storage="f32")
                     for _ in range(B)]
        self.ens = Ensemble(self.sols)
        self.mom = _fields(B, cfg.n_theta_c, cfg.n_phi_c, 4)
        self.corr = _fields(B, cfg.n_theta_c, cfg.n_phi_c)

    def load(self, X, idx=None):
        for b, s in enumerate(self.sols):
            j = b if idx is None else int(idx[b])
            s.init_fields_device(X[0][j], X[1][j], X[2][j], X[3][j])

    def moments(self, out=None):
        """rho, u_theta, u_phi and T of every run."""
        out = self.mom if out is None else out
        for b, s in enumerate(self.sols):
            s.moments_device(out[0][b], out[1][b], out[2][b], out[3][b])
        return out

    def interval(self, net=None, stats=None):
        """k coarse steps, then the closure correction (if a network is given)."""
        self.ens.step(self.cfg.k)
        if net is not None:
            self.correct(net, stats, self.moments())

    def correct(self, net, stats, m):
        """Apply the network's correction for the moments m of every run."""
        net.pack_input(self.B, *m[:3], stats["s_rho"], stats["s_u"], T=m[3], s_T=stats["s_T"])
        net.forward(self.B)
        net.unpack_output(self.B, stats["o_rho"], stats["o_u"], *self.corr)
        for b, s in enumerate(self.sols):
            s.correct_moments_device(self.corr[0][b], self.corr[1][b], self.corr[2][b])

    def close(self):
        for s in self.sols:
            s.close()


def build_dataset(cfg, X, net=None, stats=None):
    """Inputs Y_n and targets X_{n+1}.  Without a network Y_n is the coarse
    state one interval after a restart from X_n.  With one, the runs restart
    from X_n every rollout_steps coarse steps and Y_n is the state one interval
    after the previous correction of the closure rollout; a rollout stops
    collecting (until its next restart) at the first interval whose rms target
    exceeds rollout_cap in output units."""
    import torch
    N = X[0][0].shape[0]
    pool = CoarsePool(cfg, N)
    Y, T = [], []
    every = 1 if net is None else max(1, cfg.rollout_steps // cfg.k)
    live = True
    for n in range(cfg.intervals):
        if n % every == 0:
            pool.load(X[n])
            live = True
        if not live:
            continue
        pool.ens.step(cfg.k)
        m = pool.moments()
        if net is not None:
            d = [(X[n + 1][c] - m[c]) / (stats["o_rho"] if c == 0 else stats["o_u"]) for c in range(3)]
            rms = math.sqrt(sum(float((x * x).mean()) for x in d) / 3)
            if not rms <= cfg.rollout_cap:       # also false for a run that blew up
                live = False
                continue
        Y.append([t.clone() for t in m])
        T.append(X[n + 1][:3])
        if net is not None:
            pool.correct(net, stats, m)
    pool.close()
    cat = lambda L, c: torch.cat([x[c] for x in L], 0).contiguous()
    return [cat(Y, c) for c in range(4)], [cat(T, c) for c in range(3)]


def fit(cfg, Y, T, log=None, net=None, stats=None):
    """Train the network on (Y, T); returns (net, stats, loss history).  A
    network and its input/output scales passed in are trained further."""
    import torch
    from .closure import ClosureNet
    M = Y[0].shape[0]
    if stats is None:
        d = [T[c] - Y[c] for c in range(3)]
        sT = float((Y[3] - 1.0).std())
        stats = {"s_rho": 1.0 / float((Y[0] - 1.0).std()),
                 "s_u": 1.0 / float(torch.cat([Y[1], Y[2]]).std()),
                 "s_T": 1.0 / sT if sT > 0 else 0.0,
                 "o_rho": float(d[0].std()), "o_u": float(torch.cat([d[1], d[2]]).std())}
        del d
    mb = min(cfg.minibatch, M)
    if net is None:
        # capacity for a minibatch and for the rollouts of all training or held-out runs
        cap = max(mb, len(cfg.train_seeds), len(cfg.eval_seeds))
        net = ClosureNet(cfg.n_theta_c, cfg.n_phi_c, cap, seed=cfg.seed)
    target = torch.zeros(mb * cfg.n_theta_c * cfg.n_phi_c * 3, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(cfg.seed)
    bufY = _fields(mb, cfg.n_theta_c, cfg.n_phi_c, 4)
    bufT = _fields(mb, cfg.n_theta_c, cfg.n_phi_c)
    hist = []
    for it in range(cfg.iters):
        idx = torch.from_numpy(rng.choice(M, size=mb, replace=False)).cuda()
        for c in range(4):
            torch.index_select(Y[c], 0, idx, out=bufY[c])
        for c in range(3):
            torch.index_select(T[c], 0, idx, out=bufT[c])
        net.pack_input(mb, *bufY[:3], stats["s_rho"], stats["s_u"], T=bufY[3], s_T=stats["s_T"])
        net.pack_target(mb, bufT, bufY[:3], stats["o_rho"], stats["o_u"], target)
        net.forward(mb)
        lr = cfg.lr * (0.1 ** (it / max(cfg.iters - 1, 1)))      # exponential decay to lr / 10
        hist.append(net.loss(mb, target))
        net.backward(mb)
        net.adam(lr)
        if log and (it % 250 == 0 or it == cfg.iters - 1):
            log(f"  iter {it}: loss {hist[-1]:.4f}")
    return net, stats, hist


def vorticity_spectrum(omega, lmax):
    """Degree spectrum E(l) = sum_m |w_lm|^2 of a field on the grid (midpoint
    quadrature in theta, FFT in phi)."""
    from workloads.fields import _legendre_columns
    H, Wd = omega.shape
    th = (np.arange(H) + 0.5) * np.pi / H
    F = np.fft.rfft(omega, axis=1) * (2 * np.pi / Wd)
    wq = np.sin(th) * np.pi / H
    E = np.zeros(lmax + 1)
    for m in range(0, lmax + 1):
        P, _ = _legendre_columns(lmax, m, th)
        c = P @ (wq * F[:, m])
        E[m:] += (1.0 if m == 0 else 2.0) * np.abs(c) ** 2
    return E


def _rel(a, b, w):
    return float(np.sqrt((w * (a - b) ** 2).sum() / (w * b ** 2).sum()))


def evaluate(cfg, net, stats, X, fine_ms):
    """Roll out plain coarse and coarse + closure from X[0] for all intervals and
    compare with the filtered fine states."""
    import torch
    from .vlbm import Solver
    B = X[0][0].shape[0]
    H, Wd = cfg.n_theta_c, cfg.n_phi_c
    w = np.sin((np.arange(H) + 0.5) * np.pi / H)[:, None]
    diag = Solver(H, Wd, cfg.tau, cfg.dt_c, storage="f64")
    om = torch.zeros((H, Wd), dtype=torch.float64, device="cuda")

    def vort(fields, b):
        diag.init_fields_device(fields[0][b], fields[1][b], fields[2][b])
        diag.vorticity_device(om)
        return om.cpu().numpy().copy()

    out = {}
    L = H // 2
    for name, use in (("coarse", False), ("closure", True)):
        pool = CoarsePool(cfg, B)
        pool.load(X[0])
        clock = _Events()
        errs = {"vorticity": [], "u": [], "spectrum_dex": []}
        for n in range(1, cfg.intervals + 1):
            with clock:
                pool.interval(net if use else None, stats)
            if n in (cfg.intervals // 4, cfg.intervals // 2, cfg.intervals):
                m = [t.clone() for t in pool.moments()]
                ev, eu, es = [], [], []
                for b in range(B):
                    o_run, o_ref = vort(m, b), vort(X[n], b)
                    ev.append(_rel(o_run, o_ref, w))
                    ur = [t[b].cpu().numpy() for t in m]
                    uf = [t[b].cpu().numpy() for t in X[n]]
                    eu.append(math.sqrt((_rel(ur[1], uf[1], w) ** 2 * (w * uf[1] ** 2).sum() +
                                         _rel(ur[2], uf[2], w) ** 2 * (w * uf[2] ** 2).sum()) /
                                        (w * (uf[1] ** 2 + uf[2] ** 2)).sum()))
                    Er, Ef = vorticity_spectrum(o_run, L), vorticity_spectrum(o_ref, L)
                    es.append(float(np.mean(np.abs(np.log10(Er[1:] / Ef[1:])))))
                errs["vorticity"].append((n, float(np.mean(ev))))
                errs["u"].append((n, float(np.mean(eu))))
                errs["spectrum_dex"].append((n, float(np.mean(es))))
        pool.close()
        t_sim = cfg.intervals * cfg.k * cfg.dt_c
        out[name] = {"errors": errs, "ms_per_unit_time_per_run": clock.ms / (B * t_sim)}
    diag.close()
    out["fine_ms_per_unit_time_per_run"] = fine_ms
    for name in ("coarse", "closure"):
        out[name]["cost_ratio_fine_over_this"] = fine_ms / out[name]["ms_per_unit_time_per_run"]
    return out


def _filtered_difference(cfg, A, Bf):
    """Mean over runs of the relative L2 of the vorticity of coarse fields A
    against Bf (three FP64 device tensors each, [runs][n_theta_c][n_phi_c])."""
    import torch
    from .vlbm import Solver
    H, Wd = cfg.n_theta_c, cfg.n_phi_c
    w = np.sin((np.arange(H) + 0.5) * np.pi / H)[:, None]
    diag = Solver(H, Wd, cfg.tau, cfg.dt_c, storage="f64")
    om = torch.zeros((H, Wd), dtype=torch.float64, device="cuda")
    errs = []
    for b in range(A[0].shape[0]):
        o = []
        for F in (A, Bf):
            diag.init_fields_device(F[0][b].contiguous(), F[1][b].contiguous(), F[2][b].contiguous())
            diag.vorticity_device(om)
            o.append(om.cpu().numpy().copy())
        errs.append(_rel(o[0], o[1], w))
    diag.close()
    return float(np.mean(errs))


def run(cfg, log=print, ks=None):
    """Fine data, training and evaluation for every closure interval k in ks
    (default: cfg.k) over the same simulated time cfg.intervals * cfg.k coarse
    steps.  The fine runs are made once, filtered at the finest interval;
    returns {k: result} (or the result of cfg.k alone when ks is None)."""
    import torch
    single = ks is None
    ks = [cfg.k] if single else list(ks)
    steps = cfg.intervals * cfg.k
    assert all(steps % k == 0 for k in ks), "every interval must divide the run"
    kmin = math.gcd(*ks) if len(ks) > 1 else ks[0]
    t0 = time.time()
    log(f"fine substeps per coarse step: {fine_substeps(cfg)}")
    base = replace(cfg, k=kmin, intervals=steps // kmin)
    Xtr_all, fine_ms = fine_filtered(base, cfg.train_seeds)
    Xev_all, fine_ms_ev = fine_filtered(base, cfg.eval_seeds)
    log(f"fine data: {len(cfg.train_seeds)} + {len(cfg.eval_seeds)} runs, {time.time() - t0:.1f} s")
    # the training and reference data come from FP32-store fine runs: their
    # filtered end state against FP64-store runs of the first two held-out seeds
    seeds2 = cfg.eval_seeds[:2]
    X64, _ = fine_filtered(replace(cfg, intervals=1, k=steps), seeds2, storage="f64")
    fine_fp32_err = _filtered_difference(cfg, [x[:2] for x in Xev_all[-1]], X64[-1])
    log(f"fine runs, FP32 vs FP64 store, filtered end state: vorticity rel L2 {fine_fp32_err:.2e}")
    out = {}
    for k in ks:
        t1 = time.time()
        ck = replace(cfg, k=k, intervals=steps // k)
        sub = k // kmin
        Xtr, Xev = Xtr_all[::sub], Xev_all[::sub]
        Y, T = build_dataset(ck, Xtr)
        net, stats, hist = fit(ck, Y, T, log)
        for _ in range(cfg.rollout_rounds):
            Yr, Tr = build_dataset(ck, Xtr, net, stats)
            Y = [torch.cat([a, b], 0) for a, b in zip(Y, Yr)]
            T = [torch.cat([a, b], 0) for a, b in zip(T, Tr)]
            del Yr, Tr
            net, stats, h2 = fit(ck, Y, T, log, net, stats)
            hist += h2
        del Y, T
        log(f"k = {k}: trained in {time.time() - t1:.1f} s")
        res = evaluate(ck, net, stats, Xev, fine_ms_ev)
        res["config"] = {a: v for a, v in asdict(ck).items() if a not in ("train_seeds", "eval_seeds")}
        res["config"].update(n_train=len(cfg.train_seeds), n_eval=len(cfg.eval_seeds),
                             fine_substeps=fine_substeps(cfg))
        res["loss_first_last"] = [hist[0], hist[-1]]
        res["fine_fp32_vs_fp64_vorticity_rel_l2"] = fine_fp32_err
        res["stats"] = stats
        res["wall_s"] = time.time() - t1
        net.close()
        out[k] = res
    return out[ks[0]] if single else out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=32, help="training runs")
    ap.add_argument("--eval", type=int, default=8, help="held-out runs")
    ap.add_argument("--intervals", type=int, default=40)
    ap.add_argument("--iters", type=int, default=1500)
    a = ap.parse_args(argv)
    cfg = Config(intervals=a.intervals, iters=a.iters,
                 train_seeds=list(range(1000, 1000 + a.train)),
                 eval_seeds=list(range(2000, 2000 + a.eval)))
    import torch
    torch.cuda.set_device(0)
    res = run(cfg, log=lambda s: print(s, file=sys.stderr, flush=True))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
