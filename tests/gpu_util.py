"""Shared helpers for the GPU parity tests (test infrastructure)."""
import os
import sys

import numpy as np

import oracle as O


def announce(msg: str) -> None:
    """Name the case on the real stderr (flushed, so it survives a dying run) and, when
    HOM4D_TEST_LOG names a file, append it there too (pytest captures stderr)."""
    line = f"[gpu-test] {msg}\n"
    sys.__stderr__.write(line)
    sys.__stderr__.flush()
    path = os.environ.get("HOM4D_TEST_LOG")
    if path:
        with open(path, "a") as f:
            f.write(line)


def grid_of(w, **kw):
    args = dict(b_tesla=w.b_tesla, soft_nm=w.soft_nm, coulomb_c=w.coulomb_c,
                mstar_rel=w.mstar_rel, eps_r=w.eps_r)
    args.update(kw)
    return O.make_grid(w.nx, w.ny, w.lx, w.ly, **args)


def rel_l2(a, b) -> float:
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def oracle_run(w, steps, sym=None, **grid_kw):
    g = grid_of(w, **grid_kw)
    psi0 = O.init_state(w.psi_a, w.psi_b, w.sym if sym is None else sym)
    return O.propagate(psi0, g, w.v_table, w.dt_fs, steps), g


def gpu_run(w, steps, precision="fp64", coulomb_mode="table", sym=None, **kw):
    from paper_1903_02581_amd import Propagator
    p = Propagator.from_workload(w, precision=precision, coulomb_mode=coulomb_mode, **kw)
    if sym is not None:
        p.init_state(w.psi_a, w.psi_b, sym)
    p.step(steps)
    psi = p.store_state()
    obs = p.observables(w.w_top)
    p.close()
    return psi, obs
