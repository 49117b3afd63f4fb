#!/usr/bin/env python3
"""Throughput of the two-electron split-step propagator on one MI355X.

Workload (default): the 64x64-per-electron FP64 case -- 16.8M complex128 grid
points (268 MB), box 800 x 600 nm, GaAs (m* = 0.067, eps_r = 12.9), B = 5 T,
dt = 2 fs, 2000 Strang steps, softened Coulomb (d = 2 nm), saddle QPC with
the first (V0, sigma_x) of the seeded 9-run sweep.  Synthetic, seeded inputs.

A step is one Strang step S(dt) of the whole hot path (Sec. II.C Eq.
(evoloperat) of arXiv 1903.02581): the x1 pass, the fused pass over each
(x2, y2) plane (x2 transform and kinetic phase, potential factor, y2 transform
and kinetic phase), and the y1 pass with the potential factor, with the region
probabilities (Eq. (p_bunching)) sampled every 100 steps inside the timed
region.  value = grid-point-steps per second = (nx ny)^2 * steps / time.

Extra objects on the JSON line:
  roofline     -- the dominant pass kernel, its launches timed with HIP events
                  on the library's stream over a repeat of the timed region,
                  against the 8 TB/s HBM peak (and, for context, against a
                  measured 1 GiB device copy), plus the whole step's
                  algorithmic bytes per second (step_GBps);
  cpu_baseline -- the FP64 CPU oracle on a bounded sample of the same workload;
  mixed        -- the complex64-storage form on the same workload and its error
                  against the FP64 GPU run (|dP_b|, relative L2 of psi, norm).
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
AXES = {0: "x1", 1: "y1", 2: "x2+V", 3: "y2+V", 4: "plane(x2,V,y2)", 5: "y1+V"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mid.json")
# what decides the code and launch shape of the timed pass kernels: the kernel
# headers whole, and the launch-planning functions of the host and launch sources
KERNEL_SOURCES = ["paper_1903_02581_amd/csrc/axis_pass.hpp", "paper_1903_02581_amd/csrc/dft_regs.hpp",
                  "paper_1903_02581_amd/csrc/plane_pass.hpp", "paper_1903_02581_amd/csrc/hom4d_internal.hpp"]
KERNEL_FUNCTIONS = [("paper_1903_02581_amd/csrc/hom4d_host.cpp", "AxisPlan plan_axis("),
                    ("paper_1903_02581_amd/csrc/hom4d_kernels.hip", "hipError_t launch_axis("),
                    ("paper_1903_02581_amd/csrc/hom4d_kernels.hip", "hipError_t launch_plane(")]


def _function_text(path: str, head: str) -> bytes:
    with open(os.path.join(ROOT, path)) as f:
        text = f.read()
    i = text.index(head)
    j = text.index("\n}\n", i)
    return text[i:j + 3].encode()


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    for p, head in KERNEL_FUNCTIONS:
        h.update(_function_text(p, head))
    return h.hexdigest()[:16]


PLAN = 0
COULOMB_MODE = "table"


def make_prop(w, precision):
    from paper_1903_02581_amd import Propagator
    p = Propagator.from_workload(w, precision=precision, coulomb_mode=COULOMB_MODE)
    p.set_pass_plan(PLAN)
    return p


def timed_run(prop, w, steps, warmup, sample_every):
    import torch
    prop.step(warmup)
    torch.cuda.synchronize()
    samples = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(sample_every, steps - done) if sample_every else steps
        prop.step(k)
        done += k
        if sample_every:
            o = prop.observables(w.w_top)
            samples.append((o["step"], o["p_b"], o["norm"]))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, samples


def pass_timing(prop, w, steps, sample_every):
    """Average duration of each pass kernel over a timed region: the same number of steps
    with the same observable sampling as the measured run, continuing its trajectory, with
    the library bracketing every pass kernel by a HIP event pair on its own stream (kept
    out of the run that gives the step rate, since the event records add a little time)."""
    prop.pass_timing(True)
    done = 0
    while done < steps:
        k = min(sample_every, steps - done) if sample_every else steps
        prop.step(k)
        done += k
        if sample_every:
            prop.observables(w.w_top)
    times = prop.pass_times()
    prop.pass_timing(False)
    three = prop.passes_per_step == 3
    label = {"x1": "x1", "y1": "y1+V" if three else "y1", "x2": "x2 (closing half)" if three else "x2+V",
             "y2": "y2+V", "plane": "plane(x2,V,y2)"}
    return {label[k]: sec / n for k, (sec, n) in times.items()}, {label[k]: n for k, (sec, n) in times.items()}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second) of a buffer far
    larger than the caches: the achievable-HBM reference for the roofline."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        dst.copy_(src)
    end.record()
    end.synchronize()
    gbs = 2 * nbytes * reps / (start.elapsed_time(end) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def describe(w):
    return (f"{w.name}: {w.nx}x{w.ny} grid per electron ({w.points} points), {w.lx:g}x{w.ly:g} nm, "
            f"GaAs, B={w.b_tesla:g}T, dt={w.dt_fs:g}fs, "
            + (f"softened Coulomb d={w.soft_nm:g}nm" if w.coulomb_c else "no Coulomb term"))


def cpu_baseline(w, budget_s):
    """The FP64 oracle, as it stands, on the first steps of the same workload."""
    import oracle as O
    g = O.make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, soft_nm=w.soft_nm,
                    coulomb_c=w.coulomb_c, mstar_rel=w.mstar_rel, eps_r=w.eps_r)
    psi = O.init_state(w.psi_a, w.psi_b, w.sym)
    n = 0
    t0 = time.perf_counter()
    while True:
        psi = O.strang_step(psi, g, w.v_table, w.dt_fs)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return n, el


def config_throughput(name, precision, steps, plan=None, **overrides):
    """Short timed run of another named workload (same kernels, other sizes)."""
    import torch
    from workloads import preset
    w = preset(name, **overrides)
    p = make_prop(w, precision)
    if plan is not None:
        p.set_pass_plan(plan)
    p.step(3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.step(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out = {"workload": name + "".join(f",{k}={v}" for k, v in overrides.items()),
           "nx": w.nx, "ny": w.ny, "points": w.points, "precision": precision,
           "steps": steps, "passes_per_step": p.passes_per_step,
           "gp_steps_per_s": w.points * steps / sec, "ms_per_step": sec / steps * 1e3}
    sbytes = 16 if precision == "fp64" else 8
    out["effective_GBps"] = out["gp_steps_per_s"] * 2 * sbytes * p.passes_per_step / 1e9
    out["effective_frac_of_hbm_peak"] = out["effective_GBps"] / HBM_PEAK_GBS
    p.close()
    del p
    torch.cuda.empty_cache()
    return out


def adjoint_throughput(precision, name="diff", steps=None, ckpt=None):
    """Forward with checkpoints + reverse sweep: the 48x48, 1000-step gradient workload, or
    a short recording on another workload (the 256x128 one: 20 steps, checkpoint every 10)."""
    import torch
    from workloads import preset
    w = preset(name)
    steps = steps or w.steps
    ckpt = ckpt or w.ckpt_every
    p = make_prop(w, precision)
    p.set_norm_tol(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.grad_begin(ckpt, steps)
    p.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss, dldv, dldb = p.grad_backward(w.w_top)
    t2 = time.perf_counter()
    p.close()
    return {"workload": f"{name}: {w.nx}x{w.ny}, {steps} steps, checkpoint every {ckpt}",
            "precision": precision, "forward_s": t1 - t0, "backward_s": t2 - t1,
            "backward_gp_steps_per_s": w.points * steps / (t2 - t1),
            "loss_p_b": loss, "dL_dB": dldb, "sum_dL_dV": float(dldv.sum()),
            "sum_abs_dL_dV": float(np.abs(dldv).sum())}


def read_traffic(nbytes_alg):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads' throughput and the adjoint timing")
    ap.add_argument("--workload", default="mid",
                    help="named workload for the timed run (default: the 64x64 case, run 0 of its sweep)")
    ap.add_argument("--coulomb-mode", default="table", choices=["table", "direct"],
                    help="potential factor from difference tables (default) or per point")
    ap.add_argument("--plan", type=int, default=0, choices=[0, 1],
                    help="0: fused three-pass steps (default), 1: four per-axis passes")
    ap.add_argument("--profile-passes", type=int, default=0,
                    help="only launch each pass kernel this many times (for counter runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import preset
    global PLAN, COULOMB_MODE
    PLAN = args.plan
    COULOMB_MODE = args.coulomb_mode

    w = preset("mid", run=0) if args.workload == "mid" else preset(args.workload)
    P = w.points
    if args.profile_passes:
        prop = make_prop(w, args.precision)
        axes = (0, 4, 5) if prop.passes_per_step == 3 else (0, 1, 2, 3)
        for axis in axes:
            prop.run_pass(axis, args.profile_passes)
        torch.cuda.synchronize()
        # a plain copy of known size for calibrating the HBM byte counters
        src = torch.empty(P * 2, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_passes": args.profile_passes, "copy_bytes": src.numel() * 8}))
        return

    prop = make_prop(w, args.precision)
    sec, samples = timed_run(prop, w, args.steps, args.warmup, args.sample_every)
    value = P * args.steps / sec
    psi64_final = None
    obs64 = prop.observables(w.w_top)
    if args.precision == "fp64" and not args.no_mixed:
        psi64_final = prop.store_state()

    passes_per_step = prop.passes_per_step
    passes, launches = pass_timing(prop, w, args.steps, args.sample_every)
    dom = max(passes, key=passes.get)
    sbytes = 16 if args.precision == "fp64" else 8
    alg_bytes = 2 * sbytes * P                 # one read + one write of the state per launch
    achieved = alg_bytes / passes[dom] / 1e9
    traffic = read_traffic(alg_bytes)
    prop.close()
    copy_gbs = copy_bandwidth()

    mixed = None
    if args.precision == "fp64" and not args.no_mixed:
        pm = make_prop(w, "mixed")
        sec_m, samples_m = timed_run(pm, w, args.steps, args.warmup, args.sample_every)
        om = pm.observables(w.w_top)       # same trajectory as the FP64 run: warmup + steps
        psi_m = pm.store_state()
        passes_m, _ = pass_timing(pm, w, args.steps, args.sample_every)
        pm.close()
        dpb = [abs(a[1] - b[1]) for a, b in zip(samples, samples_m)]
        mixed = {
            "value": P * args.steps / sec_m, "unit": "gp-steps/s", "dtype": "c64 storage, f64 arithmetic",
            "speedup_vs_fp64": (P * args.steps / sec_m) / value,
            "err_vs_fp64_gpu": {
                "abs_dP_b_final": abs(om["p_b"] - obs64["p_b"]),
                "abs_dP_b_max_sampled": max(dpb) if dpb else None,
                "rel_l2_psi_final": float(np.linalg.norm(psi_m - psi64_final) / np.linalg.norm(psi64_final)),
                "abs_dnorm_final": abs(om["norm"] - obs64["norm"]),
            },
            "pass_seconds": passes_m,
        }

    extras = None
    if not args.no_extras:
        extras = {
            "configs": [
                config_throughput("mixed", "fp64", 100),
                config_throughput("mixed", "mixed", 200),
                config_throughput("fp64_128", "fp64", 50),
                config_throughput("full", "mixed", 50),
                config_throughput("diff", "fp64", 500),
                config_throughput("tiny", "fp64", 2000),
                config_throughput("qpc", "fp64", 300, coulomb_c=1.0),
                config_throughput("qpc", "mixed", 300, coulomb_c=1.0),
            ],
            "adjoint": [adjoint_throughput("fp64"), adjoint_throughput("mixed"),
                        adjoint_throughput("mixed", "full", 20, 10)],
        }

    cpu = None
    if not args.no_cpu:
        n_cpu, t_cpu = cpu_baseline(w, args.cpu_budget)
        cpu = {"value": P * n_cpu / t_cpu, "unit": "gp-steps/s", "cores": os.cpu_count(),
               "kind": "oracle",
               "sample": f"first {n_cpu} Strang steps of the same 64x64 workload, FP64 numpy/scipy "
                         f"(scipy.fft workers={os.cpu_count()}), {t_cpu:.1f} s"}

    line = {
        # value: the FP64 rate; the mixed form and its bunching error sit in "mixed",
        # the fraction of HBM peak in "roofline"
        "metric": "4D grid-point-steps/s FP64 vs mixed-FP32 at <=1e-4 bunching error; %HBM peak",
        "value": value,
        "unit": "gp-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "c64-storage/f64",
        "data": "synthetic",
        "config": {"workload": describe(w) + (", sweep run 0" if w.name == "mid" else ""),
                   "nx": w.nx, "ny": w.ny, "points": P, "precision": args.precision,
                   "observables_every": args.sample_every, "passes_per_step": passes_per_step,
                   "final_p_b": obs64["p_b"],
                   "final_norm": obs64["norm"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (traffic["bytes_per_launch"][dom] if traffic else None),
                     "kernel": f"pass kernel {dom}", "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_launch_s": passes[dom], "launches_timed": launches[dom],
                     "pass_seconds": passes,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     # the whole step: every pass's algorithmic bytes over the timed step
                     # time (observable sampling included); a state near the 256 MB
                     # Infinity Cache (64x64 FP64: 268 MB) partly hits it, so this can
                     # exceed what HBM alone delivers
                     "step_GBps": alg_bytes * passes_per_step / (sec / args.steps) / 1e9,
                     "step_frac": alg_bytes * passes_per_step / (sec / args.steps) / 1e9 / HBM_PEAK_GBS},
        "cpu_baseline": cpu,
        "mixed": mixed,
        "extras": extras,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
