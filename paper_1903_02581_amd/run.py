"""Propagate a named workload on the GPU and write its time series as JSON lines.

    python -m paper_1903_02581_amd.run --preset qpc --precision mixed --every 100 --out run.jsonl

The first line describes the run (preset, seed, sizes, precision, physical
parameters); every `--every` steps one line holds the step, the time in fs,
the norm, the region probabilities P_TT, P_TB, P_BT, P_BB, P_b, P_ab (Sec. III,
Eq. (p_bunching)) and the spatial entanglement of the slice through the two
packets' rows (Sec. III.C); the last line holds the totals: wall time,
grid-point-steps per second of the propagation alone and of the whole run.
Every number comes from the HIP library through the C ABI.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def packet_rows(w) -> tuple[int, int]:
    """Rows y1*, y2* of the two initial packets' maxima (the slice of the entanglement)."""
    return (int(np.argmax(np.abs(w.psi_a).max(axis=0))), int(np.argmax(np.abs(w.psi_b).max(axis=0))))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--preset", default="tiny")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--coulomb-mode", default="table", choices=["table", "direct"])
    ap.add_argument("--steps", type=int, default=None, help="default: the preset's step count")
    ap.add_argument("--every", type=int, default=100, help="sampling interval in steps")
    ap.add_argument("--no-entanglement", action="store_true")
    ap.add_argument("--out", default="-", help="JSON-lines file, '-' for stdout")
    args = ap.parse_args(argv)
    if args.every <= 0:
        ap.error("--every must be positive")

    import torch
    from workloads import preset
    from .hom4d import Propagator

    w = preset(args.preset, seed=args.seed)
    steps = w.steps if args.steps is None else args.steps
    out = sys.stdout if args.out == "-" else open(args.out, "w")
    emit = lambda rec: (out.write(json.dumps(rec) + "\n"), out.flush())  # noqa: E731

    p = Propagator.from_workload(w, precision=args.precision, coulomb_mode=args.coulomb_mode)
    p.set_norm_tol(1.0)  # report drift in the series instead of failing on it
    ix = np.arange(w.nx)
    j1, j2 = packet_rows(w)
    emit({"run": args.preset, "seed": args.seed, "nx": w.nx, "ny": w.ny, "lx_nm": w.lx,
          "ly_nm": w.ly, "points": w.points, "precision": args.precision,
          "coulomb_mode": args.coulomb_mode, "b_tesla": w.b_tesla, "dt_fs": w.dt_fs,
          "steps": steps, "every": args.every, "sym": w.sym, "soft_nm": w.soft_nm,
          "coulomb_c": w.coulomb_c, "passes_per_step": p.passes_per_step,
          "entanglement_rows": None if args.no_entanglement else [j1, j2]})

    def sample(step):
        o = p.observables(w.w_top)
        rec = {"step": step, "t_fs": step * w.dt_fs}
        rec.update({k: o[k] for k in ("norm", "p_tt", "p_tb", "p_bt", "p_bb", "p_b", "p_ab")})
        if not args.no_entanglement:
            rec["entropy"] = p.entanglement(ix, j1, ix, j2)
        emit(rec)

    torch.cuda.synchronize()
    t_all = time.perf_counter()
    t_prop = 0.0
    done = 0
    sample(0)
    while done < steps:
        n = min(args.every, steps - done)
        t0 = time.perf_counter()
        p.step(n)
        p.synchronize()
        t_prop += time.perf_counter() - t0
        done += n
        sample(done)
    wall = time.perf_counter() - t_all
    emit({"done": True, "steps": done, "wall_s": wall, "propagation_s": t_prop,
          "gp_steps_per_s": w.points * done / t_prop if t_prop > 0 else None,
          "gp_steps_per_s_with_sampling": w.points * done / wall if wall > 0 else None})
    p.close()
    if out is not sys.stdout:
        out.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
