"""Throughput benchmark of the vLBM step on one MI355X.

Workload: decaying 2-D turbulence on the sphere, 2048 x 4096 cells, D2Q16
(Q = 16 populations), nu = tau = 1e-5, dt from the stability rule (2.52e-7),
seeded streamfunction with E(l) ~ l^-3 over l = 1..256 normalised to an rms
|u| of 0.05 (synthetic data).  A step is one full SSP-RK3 update (three fused
stage kernels) of all 16 populations on every cell; MLUPS = cells * steps /
seconds / 1e6, with the populations resident in HBM.

The headline ``value`` is the FP32-deviation-store MLUPS; the FP64 and FP16
runs, their roofline fractions, the FP32/FP16 error against the FP64 run
(area-weighted relative L2 of rho, rho - 1, u and vorticity after 1000 steps
from the same initial state, whatever --steps is) and the CPU oracle's
throughput (one step of the same grid on the host cores, and the 32 x 64
sound-wave workload on one core) are reported alongside.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# VALU issue rate of FP32/FP64 arithmetic: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64
# instruction per 4 cycles (integer adds, compares and selects issue faster, so a
# mixed stream can exceed it)
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
N_THETA, N_PHI, TAU = 2048, 4096, 1e-5
STORE_BYTES = {"f64": 8, "f32": 4, "f16": 2}
KERNEL_NAME = {"f64": "stage_kernel<StF64>", "f32": "stage_kernel<StF32>", "f16": "stage_kernel<StF16>"}
# algorithmic population traffic per cell and RK step: stage 1 reads f_n and writes
# f1 (32 values), stages 2 and 3 read their input and f_n and write (48 each)
VALUES_PER_CELL_STEP = 128
# the precision comparison runs this many steps, independently of --steps
PRECISION_STEPS = 1000


def kernel_source_digest() -> str:
    """Digest of the kernel source with comments and white space removed, so
    that a counter summary stays valid across comment-only edits."""
    import re
    with open(os.path.join(ROOT, "paper_2504_15574_amd", "csrc", "vlbm.hip")) as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def measured_traffic(storage: str):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_c3_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_digest():
        return None
    e = d.get("per_storage", {}).get(storage)
    if not e:
        return None
    # each counter scaled by what it reads for a plain copy of known size
    return 1024.0 * (e["fetch_kib_per_dispatch"] * d["copy_scale_fetch"]
                     + e["write_kib_per_dispatch"] * d["copy_scale_write"])


def measured_valu(storage: str):
    """VALU wave-instructions per stage launch from the committed counter
    summary (SQ_INSTS_VALU), or None when missing or from another kernel source."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_c3_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_digest():
        return None
    return d.get("per_storage", {}).get(storage, {}).get("valu_wave_insts_per_dispatch")


def area_rel_l2(a, b, w):
    return float(np.sqrt((w * (a - b) ** 2).sum() / max((w * b ** 2).sum(), 1e-300)))


def run_gpu(storage, state, steps, warmup, precision_steps=0):
    """Time `steps` steps after `warmup` untimed ones.  With precision_steps,
    the run first advances that many steps from the initial state and keeps
    its moment and vorticity fields (device copies, taken without a host
    synchronisation), then continues into the warm-up and timed steps: the
    device does not idle between the two legs."""
    import torch
    from paper_2504_15574_amd import Solver, vlbm_stage_launches

    sol = Solver(N_THETA, N_PHI, TAU, storage=storage)
    sol.init_fields(*state)
    fields = None
    if precision_steps:
        sol.step(precision_steps)
        dev = [torch.empty((N_THETA, N_PHI), dtype=torch.float64, device="cuda") for _ in range(4)]
        sol.moments_device(*dev[:3])
        sol.vorticity_device(dev[3])
    sol.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    l0 = vlbm_stage_launches(sol.ctx)
    # the stage kernels run on sol.stream, the stream these events are recorded on
    ev0.record(sol.stream)
    sol.step(steps)
    ev1.record(sol.stream)
    torch.cuda.synchronize()
    launches = vlbm_stage_launches(sol.ctx) - l0
    ms = ev0.elapsed_time(ev1)
    diag = sol.diagnostics(raise_unstable=False)
    if precision_steps:
        fields = tuple(d.cpu().numpy() for d in dev)
        del dev
    dt = sol.dt
    sol.close()
    del sol
    torch.cuda.empty_cache()
    cells = N_THETA * N_PHI
    b = STORE_BYTES[storage]
    bytes_per_launch = VALUES_PER_CELL_STEP * b * cells / 3.0
    avg_launch_s = ms * 1e-3 / launches
    return {
        "ms_per_step": ms / steps,
        "mlups": cells * steps / (ms * 1e-3) / 1e6,
        "launches": launches,
        "avg_launch_us": avg_launch_s * 1e6,
        "achieved_gbs": bytes_per_launch / avg_launch_s / 1e9,
        "bytes_per_launch": bytes_per_launch,
        "dt": dt,
        "finite": bool(diag[4] == 0),
        "fields": fields,
    }


def precision_errors(fields, steps):
    """Area-weighted relative L2 of rho, rho - 1 (the density fluctuation), u
    (vector) and vorticity of every reduced format against the FP64 run."""
    th = (np.arange(N_THETA) + 0.5) * np.pi / N_THETA
    w = np.sin(th)[:, None] * np.ones((1, N_PHI))
    r64, a64, b64, o64 = fields["f64"]
    prec = {}
    for s, (r, a, b, o) in fields.items():
        if s == "f64":
            continue
        du = np.sqrt(((w * ((a - a64) ** 2 + (b - b64) ** 2)).sum())
                     / (w * (a64 ** 2 + b64 ** 2)).sum())
        e = {"rho": area_rel_l2(r, r64, w), "rho_minus_1": area_rel_l2(r - 1.0, r64 - 1.0, w),
             "u": float(du), "vorticity": area_rel_l2(o, o64, w)}
        e["f64_rms_rho_minus_1"] = float(np.sqrt((w * (r64 - 1.0) ** 2).sum() / w.sum()))
        e["rms_abs_rho_error"] = float(np.sqrt((w * (r - r64) ** 2).sum() / w.sum()))
        e["after_steps"] = steps
        e["rho_u_vorticity_within_1e-4"] = bool(max(e["rho"], e["u"], e["vorticity"]) <= 1e-4)
        prec[f"{s}_vs_f64"] = e
    return prec


def run_ensemble(steps):
    """The batched-ensemble workload: 32 runs at 128x256 and 32 at 256x512, FP32
    deviation store, tau = nu drawn uniformly in [1e-4, 1e-2] and an axisymmetric
    shock (rho = 1.5, T = 1.2 for theta < theta0, theta0 uniform in [pi/6, pi/3])
    per run, seed 0 (draws (nu, theta0) in run order); dt per run from the
    stability rule.  Times `steps` steps one run at a time, batched, batched
    from a HIP graph after the autotuner (launch grouping x tile shape), and
    in persistent launches (one per launch group of the tuned configuration,
    and one for all 64 runs with 15 x 16 tiles, also replayed from a HIP
    graph)."""
    import torch
    import workloads as W
    from paper_2504_15574_amd import Ensemble, Solver

    rng = np.random.default_rng(0)
    specs = []
    for i in range(64):
        nt, nph = (128, 256) if i < 32 else (256, 512)
        specs.append((nt, nph, float(rng.uniform(1e-4, 1e-2)), float(rng.uniform(np.pi / 6, np.pi / 3))))
    sols = [Solver(nt, nph, nu, storage="f32") for nt, nph, nu, _ in specs]
    states = [W.shock_state(nt, nph, th0, rho_in=1.5, T_in=1.2) for nt, nph, _, th0 in specs]

    def reset():
        for s, st in zip(sols, states):
            s.init_fields(*st)
        torch.cuda.synchronize()

    def timed(fn):
        reset()
        fn(1)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sols[0].stream)
        fn(steps)
        e1.record(sols[0].stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    cells = sum(nt * nph for nt, nph, _, _ in specs)
    ens = Ensemble(sols)
    reset()
    tune = ens.autotune(steps=10)
    one = timed(lambda n: [s.step(n) for s in sols])
    bat = timed(lambda n: ens.step(n))
    ens.capture(steps)
    reset()
    ens.replay()                      # warm replay
    torch.cuda.synchronize()
    reset()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sols[0].stream)
    ens.replay()
    e1.record(sols[0].stream)
    torch.cuda.synchronize()
    gr = e0.elapsed_time(e1)
    ens.release()
    # persistent: one cooperative launch per launch group carries all steps
    per_tuned = timed(lambda n: ens.step(n, persistent=True))
    tuned = (ens.grouping, ens.tile)
    ens.configure("all", (15, 16))
    per_all = timed(lambda n: ens.step(n, persistent=True))
    # the same single persistent launch recorded in a HIP graph
    ens.capture(steps, persistent=True)
    per_graph = timed(lambda n: (ens.replay(), ens.check()))
    ens.release()
    ens.configure(*tuned)
    finite = all(s.diagnostics(raise_unstable=False)[4] == 0 for s in sols)
    for s in sols:
        s.close()
    mlups = lambda ms: round(cells * steps / (ms * 1e-3) / 1e6, 1)
    return {"workload": "64 shock runs: 32 x 128x256 + 32 x 256x512, D2Q16, f32 deviation store",
            "steps": steps, "cells": cells, "grouping": ens.grouping,
            "tile": ens.tile_name(),
            "autotune_ms_per_step": {k: round(v, 4) for k, v in tune.items()},
            "mlups_one_run_per_launch": mlups(one), "mlups_batched": mlups(bat),
            "mlups_batched_graph": mlups(gr),
            "mlups_persistent": mlups(per_tuned), "mlups_persistent_one_launch": mlups(per_all),
            "mlups_persistent_graph": mlups(per_graph),
            "finite": finite}


def host_info():
    """The host the CPU baseline ran on: CPU model, logical CPUs, CPUs usable here."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(state, threads):
    import oracle
    import workloads as W

    f = oracle.init(*state)
    t0 = time.perf_counter()
    oracle.step(f, 1, tau=TAU, dt=oracle.suggest_dt(N_THETA, N_PHI, TAU), threads=threads)
    el = time.perf_counter() - t0
    out = {"value": round(N_THETA * N_PHI / el / 1e6, 4), "unit": "MLUPS", "cores": threads,
           "kind": "oracle",
           "sample": f"one SSP-RK3 step of the full {N_THETA}x{N_PHI} turbulence grid, "
                     f"FP64 plain-C oracle, OpenMP over theta rows, {el:.1f} s wall"}
    # the 32 x 64 sound-wave workload (rho = 1 + 1e-3 P2, nu = tau = dt = 1e-3,
    # 500 steps) on one core, as that workload is stated
    nt, nph, n = 32, 64, 500
    f1 = oracle.init(*W.sound_wave_p2(nt, nph))
    t0 = time.perf_counter()
    oracle.step(f1, n, tau=1e-3, dt=1e-3, threads=1)
    el1 = time.perf_counter() - t0
    out["sound_wave_32x64_one_core"] = {"wall_s": round(el1, 2), "steps": n, "cores": 1,
                                        "mlups": round(nt * nph * n / el1 / 1e6, 4)}
    return out


def _scheme_mlups(n_theta, n_phi, tau, state, steps, **kw):
    """MLUPS of one Solver configuration: `steps` timed steps after 2 warm-up
    steps, timed with HIP events on the run's stream; also whether it stayed
    finite."""
    import torch
    from paper_2504_15574_amd import Solver
    sol = Solver(n_theta, n_phi, tau, **kw)
    sol.init_fields(*state)
    sol.step(2)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sol.stream)
    sol.step(steps)
    e1.record(sol.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ok = sol.diagnostics(raise_unstable=False)[4] == 0
    sol.close()
    return {"mlups": round(n_theta * n_phi / (ms * 1e-3) / 1e6, 1), "finite": bool(ok)}


SCHEMES = [(sc, kom) for sc in ("u1", "u2", "u3", "weno5") for kom in (False, True)]


def _scheme_key(scheme, kom):
    return f"{scheme}{'+komissarov' if kom else ''}"


def run_schemes(state, steps):
    """Cost of the advection schemes on the benchmark grid: MLUPS of U1, U2, U3
    and WENO-5, each in the standard and the Komissarov form, FP32 and FP64
    deviation store, and of the D2Q9 model (Q = 3) with WENO-5; `steps` timed
    steps after 2 warm-up steps."""
    out = {}
    for storage in ("f32", "f64"):
        for scheme, kom in SCHEMES:
            out[f"{storage}/{_scheme_key(scheme, kom)}"] = _scheme_mlups(
                N_THETA, N_PHI, TAU, state, steps, storage=storage, scheme=scheme, komissarov=kom)
    for storage in ("f32", "f64"):
        out[f"{storage}/d2q9-weno5"] = _scheme_mlups(N_THETA, N_PHI, TAU, state, steps,
                                                     storage=storage, q=3)
    return out


def run_schemes_sound(steps, n=1024):
    """The scheme comparison of the paper's performance section (Sec. V): the
    sound wave u_theta = U0 theta (pi - theta), U0 = 1e-5, on a fully 2-D
    n x n grid, FP64, every advection scheme in the standard and the
    Komissarov form (FP32 deviation store alongside).  Besides the MLUPS the
    block gives the step-time ratios the paper states in words: WENO-5 over
    U1, U3 over U1 and each Komissarov form over its standard form."""
    import workloads as W
    state = W.sound_wave_parabolic(n, n, U0=1e-5)
    tau = 1e-3
    out = {"workload": f"sound wave u_theta = 1e-5 theta (pi - theta), {n}x{n} cells, "
                       f"D2Q16, tau = {tau}", "mlups": {}}
    for storage in ("f64", "f32"):
        for scheme, kom in SCHEMES:
            out["mlups"][f"{storage}/{_scheme_key(scheme, kom)}"] = _scheme_mlups(
                n, n, tau, state, steps, storage=storage, scheme=scheme, komissarov=kom)
    m = {k: v["mlups"] for k, v in out["mlups"].items()}
    ratios = {}
    for storage in ("f64", "f32"):
        ratios[f"{storage}/weno5_over_u1"] = round(m[f"{storage}/u1"] / m[f"{storage}/weno5"], 3)
        ratios[f"{storage}/u3_over_u1"] = round(m[f"{storage}/u1"] / m[f"{storage}/u3"], 3)
        for scheme, _ in SCHEMES[::2]:
            ratios[f"{storage}/{scheme}+komissarov_over_{scheme}"] = round(
                m[f"{storage}/{scheme}"] / m[f"{storage}/{scheme}+komissarov"], 3)
    out["step_time_ratios"] = ratios
    return out


def run_closure():
    """Learned closure (coarse 32x64 FP32 + 3x3 CNN vs fine 256x512 runs filtered
    8x): 32 training seeds, 8 held-out seeds, t = 0.2 (1000 coarse steps), the
    correction applied once per 25 coarse steps (the main block) and after
    every coarse step ("per_step").  Reports errors against the filtered fine
    run at the end and the cost of each run per unit simulated time."""
    from paper_2504_15574_amd.closure_train import Config, run
    cfg = Config()
    rs = run(cfg, log=lambda s: print("[bench]" + s, file=sys.stderr, flush=True), ks=(cfg.k, 1))

    def block(r, k):
        last = lambda name, key: round(r[name]["errors"][key][-1][1], 5)
        out = {"workload": "decaying turbulence, coarse 32x64 FP32 (+closure) vs fine 256x512 FP32 "
                           f"filtered 8x; 32 training / 8 held-out seeds, t = 0.2; inputs rho, u, T; "
                           f"correction every {k} coarse step{'s' if k > 1 else ''}; trained on "
                           f"restart pairs + {cfg.rollout_rounds} round of rollout pairs",
               "correction_interval_steps": k,
               "train_loss_first_last": [round(x, 4) for x in r["loss_first_last"]]}
        for name in ("coarse", "closure"):
            out[name] = {"vorticity_rel_l2": last(name, "vorticity"), "u_rel_l2": last(name, "u"),
                         "vorticity_spectrum_mean_abs_log10": last(name, "spectrum_dex"),
                         "ms_device_per_unit_time_per_run": round(r[name]["ms_per_unit_time_per_run"], 2),
                         "cost_ratio_fine_over_this": round(r[name]["cost_ratio_fine_over_this"], 1)}
        out["fine_ms_device_per_unit_time_per_run"] = round(r["fine_ms_per_unit_time_per_run"], 1)
        out["fine_fp32_vs_fp64_vorticity_rel_l2"] = float(f"{r['fine_fp32_vs_fp64_vorticity_rel_l2']:.3e}")
        out["wall_s"] = round(r["wall_s"], 1)
        return out

    out = block(rs[cfg.k], cfg.k)
    out["per_step"] = block(rs[1], 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--storages", default="f32,f64,f16",
                    help="comma list; the first is the headline value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 64-run batched-ensemble measurement")
    ap.add_argument("--ensemble-steps", type=int, default=400)
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip the advection-scheme cost comparison (U1/U2/U3/WENO-5, Komissarov)")
    ap.add_argument("--scheme-steps", type=int, default=100)
    ap.add_argument("--scheme-steps-sound", type=int, default=200)
    ap.add_argument("--no-closure", action="store_true",
                    help="skip the learned-closure experiment (training and evaluation, ~20 s)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (5 times); "
                         "calibrates the HBM byte counters against a known traffic")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one MI355X only: --gpus {args.gpus} (WORLD_SIZE {world}) "
              "is not supported; the multi-GPU layout (theta bands with halo exchange) is "
              "described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "copies": 5}))
        return
    storages = args.storages.split(",")
    t0 = time.time()
    state = W.turbulence_state(N_THETA, N_PHI, seed=0, lmax=256, urms=0.05)
    print(f"[bench] initial state built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    # each format's run first advances PRECISION_STEPS steps for the precision
    # comparison (whatever --steps is), then the warm-up and the timed steps
    psteps = 0 if args.no_precision or "f64" not in storages else PRECISION_STEPS
    res = {}
    for s in storages:
        torch.cuda.synchronize()
        res[s] = run_gpu(s, state, args.steps, args.warmup, psteps)
        print(f"[bench] {s}: {res[s]['mlups']:.0f} MLUPS, {res[s]['ms_per_step']:.3f} ms/step, "
              f"{res[s]['achieved_gbs']:.0f} GB/s algorithmic", file=sys.stderr, flush=True)

    head = storages[0]
    h = res[head]
    traffic = measured_traffic(head)
    out = {
        "metric": "MLUPS (2048x4096,Q=16) FP32-store vs FP64 at <=1e-4 rel err; % HBM peak",
        "value": round(h["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": "decaying turbulence on the sphere, 2048x4096 cells, D2Q16, "
                               f"{head} deviation store",
                   "n_theta": N_THETA, "n_phi": N_PHI, "q": 16, "tau": TAU,
                   "dt": h["dt"], "storage": head, "seed": 0},
        "roofline": {"bound": "hbm", "achieved": round(h["achieved_gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(h["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": round(traffic, 1) if traffic else None,
                     "kernel": KERNEL_NAME[head],
                     "avg_launch_us": round(h["avg_launch_us"], 2),
                     "algorithmic_bytes_per_launch": h["bytes_per_launch"]},
    }
    valu = measured_valu(head)
    if valu:
        # the stage kernel's VALU issue rate: what holds the float kernels (the
        # HBM fraction above is of the algorithmic population bytes)
        ach = valu / (h["avg_launch_us"] * 1e-6) / 1e9
        out["roofline"]["valu"] = {"wave_insts_per_launch": valu, "achieved": round(ach, 1),
                                   "peak": VALU_PEAK_GINST, "unit": "G wave-instructions/s",
                                   "frac": round(ach / VALU_PEAK_GINST, 4)}
    per = {}
    for s in storages:
        per[s] = {"mlups": round(res[s]["mlups"], 1), "ms_per_step": round(res[s]["ms_per_step"], 4),
                  "hbm_frac_algorithmic": round(res[s]["achieved_gbs"] / HBM_PEAK_GBS, 4),
                  "avg_launch_us": round(res[s]["avg_launch_us"], 2), "finite": res[s]["finite"]}
        vs = measured_valu(s)
        if vs:
            per[s]["valu_issue_frac"] = round(vs / (res[s]["avg_launch_us"] * 1e-6) / 1e9 / VALU_PEAK_GINST, 4)
    out["per_storage"] = per
    if "f64" in res and "f32" in res:
        out["f32_over_f64_mlups"] = round(res["f32"]["mlups"] / res["f64"]["mlups"], 3)

    if psteps:
        out["precision"] = precision_errors({s: res[s]["fields"] for s in storages}, psteps)

    if not args.no_ensemble:
        print("[bench] batched ensemble ...", file=sys.stderr, flush=True)
        out["ensemble"] = run_ensemble(args.ensemble_steps)
        print(f"[bench] ensemble: {out['ensemble']}", file=sys.stderr, flush=True)

    if not args.no_schemes:
        print("[bench] advection schemes ...", file=sys.stderr, flush=True)
        out["schemes"] = run_schemes(state, args.scheme_steps)
        print(f"[bench] schemes: {out['schemes']}", file=sys.stderr, flush=True)
        print("[bench] advection schemes, 1024x1024 sound wave ...", file=sys.stderr, flush=True)
        out["schemes_sound_1024"] = run_schemes_sound(args.scheme_steps_sound)
        print(f"[bench] schemes_sound_1024: {out['schemes_sound_1024']}", file=sys.stderr,
              flush=True)

    if not args.no_closure:
        print("[bench] learned closure: fine data, training, evaluation ...", file=sys.stderr,
              flush=True)
        out["closure"] = run_closure()
        print(f"[bench] closure: {out['closure']}", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        threads = min(16, len(os.sched_getaffinity(0)))
        print(f"[bench] CPU oracle baseline on {threads} threads ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(state, threads)
        out["host"] = host_info()
    print(json.dumps(out), flush=True)
    # release device memory while the runtime is fully up (every run object is
    # closed by now; nothing is left to the interpreter's shutdown)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
