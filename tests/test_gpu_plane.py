"""The fused three-pass step (x1 | plane of (x2, y2) with X2, V, Y2 | y1 with V)
against the four per-axis passes and against the FP64 oracle."""
import numpy as np
import pytest

from workloads.presets import build
from tests.gpu_util import announce, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

PLANE_SIZES = [(16, 16), (24, 24), (32, 32), (48, 48), (64, 64), (48, 16), (16, 48)]


def _w(nx, ny, steps):
    return build("pl", nx, ny, 12.5 * nx, 9.375 * ny, b_tesla=5.0, dt_fs=2.0, steps=steps,
                 sigma_x=20.0, seed=nx * 7 + ny)


@pytest.mark.parametrize("nx,ny", PLANE_SIZES)
def test_three_pass_equals_four_pass(nx, ny):
    from paper_1903_02581_amd import Propagator
    w = _w(nx, ny, 3)
    announce(f"plane vs per-axis {nx}x{ny} steps=3")
    out = {}
    for plan in (0, 1):
        p = Propagator.from_workload(w)
        p.set_pass_plan(plan)
        assert p.passes_per_step == (3 if plan == 0 else 4)
        p.step(w.steps)
        out[plan] = p.store_state()
        p.close()
    assert rel_l2(out[0], out[1]) <= 1e-13


@pytest.mark.parametrize("nx,ny,steps", [(64, 64, 2), (48, 48, 6), (48, 16, 20)])
def test_three_pass_vs_oracle(nx, ny, steps):
    from paper_1903_02581_amd import Propagator
    w = _w(nx, ny, steps)
    announce(f"plane vs oracle {nx}x{ny} steps={steps}")
    p = Propagator.from_workload(w)
    assert p.passes_per_step == 3
    p.step(steps)
    psi = p.store_state()
    p.close()
    ref, _ = oracle_run(w, steps)
    assert rel_l2(psi, ref) <= 1e-10


@pytest.mark.parametrize("mode", ["table", "direct"])
@pytest.mark.parametrize("nx,ny,steps", [(48, 48, 30), (64, 64, 6), (16, 48, 30)])
def test_three_pass_mixed_and_direct(mode, nx, ny, steps):
    from paper_1903_02581_amd import Propagator
    w = _w(nx, ny, steps)
    announce(f"plane mixed/{mode} {nx}x{ny} steps={steps}")
    res = {}
    for prec in ("fp64", "mixed"):
        p = Propagator.from_workload(w, precision=prec, coulomb_mode=mode)
        p.step(w.steps)
        res[prec] = p.store_state()
        p.close()
    q = Propagator.from_workload(w, coulomb_mode=mode)
    q.set_pass_plan(1)
    q.step(w.steps)
    ref4 = q.store_state()
    q.close()
    assert rel_l2(res["fp64"], ref4) <= 1e-13
    assert rel_l2(res["mixed"], ref4) <= 1e-4

