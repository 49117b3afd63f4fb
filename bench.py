#!/usr/bin/env python3
"""Throughput of the two-electron split-step propagator on one MI355X.

Headline workload (default): the full-scale mixed-precision case -- 256x128
grid per electron (1.07e9 grid points), complex64 state (8.6 GB) with FP64
arithmetic, box 2000 x 1000 nm, GaAs (m* = 0.067, eps_r = 12.9), B = 5 T,
dt = 0.5 fs, softened Coulomb (d = 2 nm), saddle QPC, packets sigma_x = 10 nm.
Synthetic, seeded inputs; the state is resident in HBM before timing starts.

A step is one Strang step S(dt) of the whole hot path (Sec. II.C Eq.
(evoloperat) of arXiv 1903.02581): four state passes -- x1 transform and
kinetic phase; x2 transform and kinetic phase, then the potential factor; y1
transform and kinetic phase; y2 transform and kinetic phase, then the
potential factor -- with the region probabilities of Eq. (p_bunching) sampled
every 100 steps and at the end of the timed region.
value = grid-point-steps per second = (nx ny)^2 * steps / time.

Extra objects on the JSON line:
  roofline      -- the dominant pass kernel of the headline run, its launches
                   timed with HIP events on the library's stream over a repeat
                   of the timed region, against the 8 TB/s HBM peak (and, for
                   context, a measured 1 GiB device copy); traffic is the
                   counter-derived HBM bytes per launch of the same kernel
                   (profiles/traffic_<workload>_<precision>.json, reported only
                   while the kernel sources hash to the profiled version);
  cpu_baseline  -- the FP64 CPU oracle, as it stands, on whole Strang steps of
                   the 128x96 workload (the largest the oracle finishes within
                   the budget), with the host CPU model and thread count;
  fp64          -- the FP64 path on the 128x128-per-electron comparison
                   workload (same box spacing, field and time step as the
                   headline), its dominant pass kernel against the peak;
  error_budget  -- the 128x96 workload (B = 6 T, dt = 1 fs, d = 1 nm) run for
                   its 5000 steps in complex64 storage and in FP64: |dP_b| at
                   every 100th step and at the end, relative L2 of the final
                   state, |dnorm|, and the two throughputs (the mixed form's
                   speedup on the same workload);
  extras        -- the other workloads (64x64 FP64 three-pass, 48x48, 16x16,
                   the 128x64 beam splitter) and adjoint timings.

Other modes: --profile-passes N (launch each pass kernel N times, for counter
runs), --ingest-counters FETCH.csv WRITE.csv (turn two rocprofv3 counter runs
of that mode into the traffic file), --full-run coulomb|factorised (the
256x128 configuration at its full length, see full_run()).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "4D grid-point-steps/s FP64 vs mixed-FP32 at <=1e-4 bunching error; %HBM peak"
PASS_OF_AXIS = {0: "x1", 1: "y1", 2: "x2", 3: "y2"}
# what decides the code and launch shape of the timed pass kernels: the kernel
# headers whole, and the launch-planning functions of the host and launch sources
KERNEL_SOURCES = ["paper_1903_02581_amd/csrc/axis_pass.hpp", "paper_1903_02581_amd/csrc/axis3_pass.hpp",
                  "paper_1903_02581_amd/csrc/dft_regs.hpp", "paper_1903_02581_amd/csrc/plane_pass.hpp",
                  "paper_1903_02581_amd/csrc/hom4d_internal.hpp"]
KERNEL_FUNCTIONS = [("paper_1903_02581_amd/csrc/hom4d_host.cpp", "AxisPlan plan_axis("),
                    ("paper_1903_02581_amd/csrc/hom4d_kernels.hip", "hipError_t resident_blocks("),
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


def traffic_path(workload: str, precision: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")


COULOMB_MODE = "table"
PLAN = 0


def make_prop(w, precision):
    from paper_1903_02581_amd import Propagator
    p = Propagator.from_workload(w, precision=precision, coulomb_mode=COULOMB_MODE)
    p.set_pass_plan(PLAN)
    return p


def sbytes(precision: str) -> int:
    return 16 if precision == "fp64" else 8


def timed_run(prop, w, steps, warmup, sample_every):
    """Warm-up steps, then `steps` timed steps with the region probabilities sampled
    every `sample_every` steps and at the end (0: only at the end)."""
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
        o = prop.observables(w.w_top)
        samples.append((o["step"], o["p_b"], o["norm"]))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, samples


def pass_timing(prop, w, steps, sample_every):
    """Average duration of each pass kernel over a repeat of the timed region (same steps,
    same sampling, continuing the trajectory), with the library bracketing every pass kernel
    by a HIP event pair on its own stream (kept out of the run that gives the step rate,
    since the event records add a little time)."""
    prop.pass_timing(True)
    done = 0
    while done < steps:
        k = min(sample_every, steps - done) if sample_every else steps
        prop.step(k)
        done += k
        prop.observables(w.w_top)
    times = prop.pass_times()
    prop.pass_timing(False)
    three = prop.passes_per_step == 3
    label = {"x1": "x1", "y1": "y1+V" if three else "y1", "x2": "x2 (closing half)" if three else "x2+V",
             "y2": "y2+V", "plane": "plane(x2,V,y2)"}
    return {label[k]: sec / n for k, (sec, n) in times.items()}, {label[k]: n for k, (sec, n) in times.items()}


def roofline_of(passes, launches, points, precision):
    """The dominant pass kernel against the HBM peak: algorithmic bytes of one launch (one
    read and one write of every grid point) over its average launch duration."""
    dom = max(passes, key=passes.get)
    alg = 2 * sbytes(precision) * points
    achieved = alg / passes[dom] / 1e9
    return dom, {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": achieved / HBM_PEAK_GBS, "kernel": f"pass kernel {dom}",
                 "algorithmic_bytes_per_launch": alg, "avg_launch_s": passes[dom],
                 "launches_timed": launches[dom], "pass_seconds": passes}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second) of a buffer far larger
    than the caches: the achievable-HBM reference for the roofline."""
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


def describe(w, precision):
    store = "complex128 state" if precision == "fp64" else "complex64 state, FP64 arithmetic"
    return (f"{w.name}: {w.nx}x{w.ny} grid per electron ({w.points} points), {store}, "
            f"{w.lx:g}x{w.ly:g} nm, GaAs, B={w.b_tesla:g}T, dt={w.dt_fs:g}fs, "
            + (f"softened Coulomb d={w.soft_nm:g}nm" if w.coulomb_c else "no Coulomb term")
            + f", sigma_x={w.sigma_x:g}nm")


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(name, budget_s):
    """The FP64 oracle, as it stands, on whole Strang steps of a named workload until the
    budget is spent (at least one step)."""
    import oracle as O
    from workloads import preset
    w = preset(name)
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
    del psi
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or None
    from oracle import splitstep
    workers = getattr(splitstep, "_WORKERS", os.cpu_count())
    return {"value": w.points * n / el, "unit": "gp-steps/s", "cores": int(workers), "kind": "oracle",
            "sample": f"{n} whole Strang step(s) of the {w.nx}x{w.ny} workload ({w.points} points, "
                      f"softened Coulomb on), FP64 numpy/scipy, scipy.fft workers={workers}"
                      + (f", OMP_NUM_THREADS={threads}" if threads else "")
                      + f", {el:.1f} s; host CPU: {host_cpu()}"}


def config_run(name, precision, steps, warmup=3, plan=None, **overrides):
    """Timed run of a named workload (same kernels, other sizes), with per-pass timing."""
    import torch
    from workloads import preset
    w = preset(name, **overrides)
    p = make_prop(w, precision)
    if plan is not None:
        p.set_pass_plan(plan)
    p.set_norm_tol(1.0)
    sec, _ = timed_run(p, w, steps, warmup, 0)
    passes, launches = pass_timing(p, w, steps, 0)
    dom, rl = roofline_of(passes, launches, w.points, precision)
    out = {"workload": name + "".join(f",{k}={v}" for k, v in overrides.items()),
           "nx": w.nx, "ny": w.ny, "points": w.points, "precision": precision,
           "steps": steps, "passes_per_step": p.passes_per_step,
           "gp_steps_per_s": w.points * steps / sec, "ms_per_step": sec / steps * 1e3,
           "roofline": {k: rl[k] for k in ("achieved", "frac", "kernel", "avg_launch_s", "pass_seconds")}}
    out["effective_GBps"] = out["gp_steps_per_s"] * 2 * sbytes(precision) * p.passes_per_step / 1e9
    out["effective_frac_of_hbm_peak"] = out["effective_GBps"] / HBM_PEAK_GBS
    p.close()
    del p
    torch.cuda.empty_cache()
    return out


def error_budget(name, steps, sample_every):
    """The same workload in complex64 storage and in FP64 for `steps` steps: the bunching
    error of the mixed form at every sampled step and at the end, the final state's
    relative L2 error and norm difference, and both throughputs."""
    import torch
    from workloads import preset
    w = preset(name)
    res = {}
    for prec in ("fp64", "mixed"):
        p = make_prop(w, prec)
        p.set_norm_tol(1.0)
        sec, samples = timed_run(p, w, steps, 0, sample_every)
        psi = p.store_state()
        p.close()
        del p
        torch.cuda.empty_cache()
        res[prec] = (sec, samples, psi)
    (s64, o64, psi64), (s32, o32, psi32) = res["fp64"], res["mixed"]
    dpb = [abs(a[1] - b[1]) for a, b in zip(o64, o32)]
    rel = float(np.linalg.norm(psi32 - psi64) / np.linalg.norm(psi64))
    return {"workload": describe(w, "mixed").split(",")[0] + f" x {steps} steps",
            "steps": steps, "sample_every": sample_every,
            "fp64_gp_steps_per_s": w.points * steps / s64, "mixed_gp_steps_per_s": w.points * steps / s32,
            "speedup_mixed_vs_fp64": s64 / s32,
            "abs_dP_b_final": dpb[-1], "abs_dP_b_max_sampled": max(dpb),
            "rel_l2_psi_final": rel, "abs_dnorm_final": abs(o32[-1][2] - o64[-1][2]),
            "p_b_final_fp64": o64[-1][1], "norm_final_fp64": o64[-1][2],
            "within_1e-4": bool(max(dpb) <= 1e-4 and rel <= 1e-4)}


def adjoint_timing(precision, name="diff", steps=None, ckpt=None):
    """Forward with checkpoints + reverse sweep: the 48x48, 1000-step gradient workload, or
    a short recording on another workload."""
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
    del p
    torch.cuda.empty_cache()
    return {"workload": f"{name}: {w.nx}x{w.ny}, {steps} steps, checkpoint every {ckpt}",
            "precision": precision, "forward_s": t1 - t0, "backward_s": t2 - t1,
            "backward_gp_steps_per_s": w.points * steps / (t2 - t1),
            "loss_p_b": loss, "dL_dB": dldb, "sum_dL_dV": float(dldv.sum()),
            "sum_abs_dL_dV": float(np.abs(dldv).sum())}


def read_traffic(workload, precision, kernel):
    try:
        with open(traffic_path(workload, precision)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t["bytes_per_launch"].get(kernel)


# ----------------------------------------------------------------- counter runs

def profile_passes(w, precision, reps):
    """Launch each pass kernel of the step plan `reps` times, then a plain device copy of
    the state's size (the calibration of the HBM byte counters)."""
    import torch
    prop = make_prop(w, precision)
    axes = (0, 4, 5) if prop.passes_per_step == 3 else (0, 1, 2, 3)
    for axis in axes:
        prop.run_pass(axis, reps)
    torch.cuda.synchronize()
    n = w.points * sbytes(precision) // 8
    src = torch.empty(n, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_passes": reps, "copy_bytes": n * 8, "axes": list(axes)}))


def _pass_of_kernel(name: str, three_pass: bool):
    if "k_plane2" in name:
        return "plane(x2,V,y2)"
    m = re.search(r"k_axis3?<HIP_vector_type<(?:float|double), 2u>, (\d+), ", name)
    if not m:
        return None
    ax = PASS_OF_AXIS[int(m.group(1))]
    if three_pass:
        return {"x1": "x1", "y1": "y1+V", "x2": "x2 (closing half)", "y2": "y2+V"}[ax]
    return {"x1": "x1", "y1": "y1", "x2": "x2+V", "y2": "y2+V"}[ax]


def ingest_counters(fetch_csv, write_csv, workload, precision, source):
    """HBM bytes per launch of every pass kernel from two rocprofv3 counter runs of
    --profile-passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
    the same counter reads for the plain copy of known size at the end of that run."""
    from workloads import preset
    w = preset(workload, run=0) if workload == "mid" else preset(workload)
    copy_bytes = w.points * sbytes(precision)
    three = workload in ("mid", "diff", "tiny")

    def per_kernel(path, counter):
        vals, copies = {}, []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                v = float(r["Counter_Value"]) * 1024.0
                if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) > 4096:
                    copies.append(v)
                    continue
                k = _pass_of_kernel(r["Kernel_Name"], three)
                if k:
                    vals.setdefault(k, []).append(v)
        if not copies:
            raise RuntimeError(f"{path}: no calibration copy found")
        # the copy reads and writes copy_bytes once
        scale = copy_bytes / copies[-1]
        return {k: float(np.mean(v)) * scale for k, v in vals.items()}, scale

    rd, fs = per_kernel(fetch_csv, "FETCH_SIZE")
    wr, ws = per_kernel(write_csv, "WRITE_SIZE")
    out = {"kernel_hash": kernel_hash(), "workload": workload, "precision": precision,
           "bytes_per_launch": {k: rd[k] + wr.get(k, 0.0) for k in rd},
           "read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
           "fetch_scale": fs, "write_scale": ws,
           "algorithmic_bytes_per_launch": 2 * copy_bytes, "source": source}
    path = traffic_path(workload, precision)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


# ------------------------------------------------------------ full-length run

def full_run(kind, steps, adj_steps, ckpt, report_every):
    """The 256x128 complex64 configuration at its full length.

    coulomb:    `steps` Strang steps with the region probabilities every `report_every`
                steps; the last `adj_steps` of them recorded (a checkpoint every `ckpt`) and
                the adjoint of the final bunching probability taken over them; dL/dB
                checked against a central difference (B +- 1e-4 relative) of two forward
                runs of those steps from the recorded start.  Reports the step rate, the
                reverse-sweep time, the peak device memory, sum dL/dV (zero by gauge
                invariance) and the dL/dB check.
    factorised: the same run with V12 = 0 against the exact factorisation into two 2D
                one-electron propagations (the oracle in 2D), point by point on sampled
                pairs and through P_TT, at every report and at the end."""
    import torch
    from workloads import preset
    t_all = time.perf_counter()
    out = {"mode": f"full-run {kind}", "steps": steps}

    def say(msg):
        print(f"[full-run {time.perf_counter() - t_all:7.1f}s] {msg}", file=sys.stderr, flush=True)

    if kind == "coulomb":
        w = preset("full")
        p = make_prop(w, "mixed")
        p.set_norm_tol(1.0)
        torch.cuda.reset_peak_memory_stats()
        fwd = steps - adj_steps
        series = []
        t0 = time.perf_counter()
        done = 0
        while done < fwd:
            k = min(report_every, fwd - done)
            p.step(k)
            done += k
            o = p.observables(w.w_top)
            series.append((done, o["p_b"], o["norm"]))
            say(f"step {done}: P_b {o['p_b']:.10f} norm {o['norm']:.12f}")
        p.grad_begin(ckpt, adj_steps)
        while done < steps:
            k = min(report_every, steps - done)
            p.step(k)
            done += k
            o = p.observables(w.w_top)
            series.append((done, o["p_b"], o["norm"]))
            say(f"step {done} (recorded): P_b {o['p_b']:.10f} norm {o['norm']:.12f}")
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t1 = time.perf_counter()
        loss, dldv, dldb = p.grad_backward(w.w_top)
        t_bwd = time.perf_counter() - t1
        say(f"adjoint over the last {adj_steps} steps: L {loss:.10f} dL/dB {dldb:.6e} ({t_bwd:.1f} s)")
        start = p.psi.clone()   # the state at the start of the recording
        h = 1e-4 * w.b_tesla
        lf = []
        for sgn in (1.0, -1.0):
            p.set_field(w.b_tesla + sgn * h)
            p.psi.copy_(start)
            p.step(adj_steps)
            lf.append(p.observables(w.w_top)["p_b"])
            say(f"forward at B {'+' if sgn > 0 else '-'} h: P_b {lf[-1]:.12f}")
        p.set_field(w.b_tesla)
        fd = (lf[0] - lf[1]) / (2 * h)
        peak = torch.cuda.max_memory_allocated()
        out.update({
            "workload": describe(w, "mixed"), "adjoint_steps": adj_steps, "ckpt_every": ckpt,
            "forward_s": t_fwd, "ms_per_step_forward": t_fwd / steps * 1e3,
            "gp_steps_per_s_forward": w.points * steps / t_fwd,
            "backward_s": t_bwd, "ms_per_step_backward": t_bwd / adj_steps * 1e3,
            "peak_device_bytes": peak, "loss_p_b": loss, "dL_dB_adjoint": dldb, "dL_dB_central_difference": fd,
            "dL_dB_rel_diff": abs(fd - dldb) / max(abs(dldb), 1e-300),
            "sum_dL_dV": float(dldv.sum()), "sum_abs_dL_dV": float(np.abs(dldv).sum()),
            "series": series})
        p.close()
    elif kind == "factorised":
        import oracle as O
        w = preset("full", coulomb_c=0.0)
        p = make_prop(w, "mixed")
        p.set_norm_tol(1.0)
        g = O.make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, soft_nm=w.soft_nm, coulomb_c=0.0,
                        mstar_rel=w.mstar_rel, eps_r=w.eps_r)
        a, b = w.psi_a.copy(), w.psi_b.copy()
        ab = np.vdot(w.psi_a, w.psi_b)
        scale = np.sqrt(2.0 * (1.0 - abs(ab) ** 2))
        nxy = w.nx * w.ny
        rng = np.random.default_rng(0)
        r1, r2 = rng.integers(0, nxy, 4000), rng.integers(0, nxy, 4000)
        idx = torch.as_tensor(r1 * nxy + r2, device=p.psi.device)
        wt = w.w_top.ravel()
        rows = []
        done = 0
        t_gpu = 0.0
        while done < steps:
            k = min(report_every, steps - done)
            # the GPU steps run while the host advances the two orbitals
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            p.step(k)
            e1.record()
            a = O.propagate_2d(a, g, w.v_table, w.dt_fs, k)
            b = O.propagate_2d(b, g, w.v_table, w.dt_fs, k)
            o = p.observables(w.w_top)
            t_gpu += e0.elapsed_time(e1) * 1e-3
            done += k
            af, bf = a.ravel(), b.ravel()
            ref = (af[r1] * bf[r2] - bf[r1] * af[r2]) / scale
            got = p.psi[idx].cpu().numpy().astype(np.complex128)
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            ta, tb = np.vdot(af, wt * af).real, np.vdot(bf, wt * bf).real
            tab, ovl = np.vdot(af, wt * bf), np.vdot(af, bf)
            p_tt = float((ta * tb - abs(tab) ** 2) / (1 - abs(ovl) ** 2))
            rows.append({"step": done, "rel_l2_sampled": err, "p_tt_gpu": o["p_tt"], "p_tt_2d_oracle": p_tt,
                         "abs_dp_tt": abs(o["p_tt"] - p_tt), "norm_gpu": o["norm"]})
            say(f"step {done}: sampled rel L2 {err:.3e}, P_TT gpu {o['p_tt']:.10f} 2D oracle {p_tt:.10f}")
        out.update({"workload": describe(w, "mixed"), "gp_steps_per_s": w.points * steps / t_gpu,
                    "ms_per_step": t_gpu / steps * 1e3, "max_rel_l2_sampled": max(r["rel_l2_sampled"] for r in rows),
                    "max_abs_dp_tt": max(r["abs_dp_tt"] for r in rows), "rows": rows,
                    "within_1e-4": bool(max(r["rel_l2_sampled"] for r in rows) <= 1e-4
                                        and max(r["abs_dp_tt"] for r in rows) <= 1e-4)})
        p.close()
    else:
        raise ValueError(kind)
    out["wall_s"] = time.perf_counter() - t_all
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="full",
                    help="named workload for the timed run (default: the 256x128 full-scale case)")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--cpu-workload", default="mixed", help="workload of the oracle baseline (default 128x96)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--budget-steps", type=int, default=5000,
                    help="steps of the 128x96 FP64-vs-mixed error budget (the workload's own count)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 comparison workload and the error budget")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads' throughput and the adjoint timing")
    ap.add_argument("--coulomb-mode", default="table", choices=["table", "direct"],
                    help="potential factor from difference tables (default) or per point")
    ap.add_argument("--plan", type=int, default=0, choices=[0, 1],
                    help="0: fused three-pass steps where built (default), 1: four per-axis passes")
    ap.add_argument("--profile-passes", type=int, default=0,
                    help="only launch each pass kernel this many times (for counter runs)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic file of --workload/--precision from two counter runs")
    ap.add_argument("--source", default="", help="with --ingest-counters: the profile summary it comes from")
    ap.add_argument("--full-run", choices=["coulomb", "factorised"],
                    help="the 256x128 configuration at its full length (20000 steps)")
    ap.add_argument("--full-steps", type=int, default=20000)
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--ckpt-every", type=int, default=100)
    ap.add_argument("--report-every", type=int, default=1000)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design note only)", file=sys.stderr)
        sys.exit(2)

    if args.ingest_counters:
        ingest_counters(args.ingest_counters[0], args.ingest_counters[1], args.workload, args.precision,
                        args.source)
        return

    import torch
    from workloads import preset
    global PLAN, COULOMB_MODE
    PLAN = args.plan
    COULOMB_MODE = args.coulomb_mode

    if args.full_run:
        full_run(args.full_run, args.full_steps, args.adjoint_steps, args.ckpt_every, args.report_every)
        return

    w = preset("mid", run=0) if args.workload == "mid" else preset(args.workload)
    P = w.points
    if args.profile_passes:
        profile_passes(w, args.precision, args.profile_passes)
        return

    prop = make_prop(w, args.precision)
    prop.set_norm_tol(1.0)
    sec, samples = timed_run(prop, w, args.steps, args.warmup, args.sample_every)
    value = P * args.steps / sec
    final = samples[-1]
    passes_per_step = prop.passes_per_step
    passes, launches = pass_timing(prop, w, args.steps, args.sample_every)
    dom, roofline = roofline_of(passes, launches, P, args.precision)
    roofline["traffic"] = read_traffic(args.workload, args.precision, dom)
    prop.close()
    del prop
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth()
    alg = roofline["algorithmic_bytes_per_launch"]
    roofline.update({
        "copy_GBps": copy_gbs, "frac_of_copy": roofline["achieved"] / copy_gbs,
        # the whole step: every pass's algorithmic bytes over the timed step time
        # (observable sampling included)
        "step_GBps": alg * passes_per_step / (sec / args.steps) / 1e9,
        "step_frac": alg * passes_per_step / (sec / args.steps) / 1e9 / HBM_PEAK_GBS})

    fp64 = budget = None
    if not args.no_compare:
        fp64 = config_run("fp64_128", "fp64", args.steps, warmup=args.warmup)
        fp64["value_ratio_headline_over_fp64"] = value / fp64["gp_steps_per_s"]
        budget = error_budget("mixed", args.budget_steps, 100)

    extras = None
    if not args.no_extras:
        extras = {
            "configs": [
                config_run("mid", "fp64", 500, run=0),
                config_run("mid", "mixed", 500, run=0),
                config_run("diff", "fp64", 500),
                config_run("tiny", "fp64", 2000),
                config_run("qpc", "fp64", 300, coulomb_c=1.0),
                config_run("qpc", "mixed", 300, coulomb_c=1.0),
            ],
            "adjoint": [adjoint_timing("fp64"), adjoint_timing("mixed"),
                        adjoint_timing("mixed", "full", 20, 10)],
        }

    cpu = None if args.no_cpu else cpu_baseline(args.cpu_workload, args.cpu_budget)

    line = {
        # value: the rate of the named workload (by default the complex64 256x128 case);
        # the FP64 comparison sits in "fp64", the bunching error of the mixed form in
        # "error_budget", the fraction of HBM peak in "roofline"
        "metric": METRIC,
        "value": value,
        "unit": "gp-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": describe(w, args.precision) + (", sweep run 0" if w.name == "mid" else ""),
                   "nx": w.nx, "ny": w.ny, "points": P, "precision": args.precision,
                   "storage": "complex128" if args.precision == "fp64" else "complex64",
                   "observables_every": args.sample_every, "passes_per_step": passes_per_step,
                   "final_p_b": final[1], "final_norm": final[2]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": fp64,
        "error_budget": budget,
        "extras": extras,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
