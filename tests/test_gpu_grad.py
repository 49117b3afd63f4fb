"""Adjoint gradient of the GPU path against the oracle's stored-state adjoint
and against central finite differences of the GPU forward run."""
import numpy as np
import pytest

import oracle as O
from workloads.presets import build
from tests.gpu_util import announce, grid_of

pytestmark = pytest.mark.gpu


def _case(nx=8, ny=8, steps=6, sym=-1, seed=1, lx=None, sx=30.0):
    w = build("g", nx, ny, 25.0 * nx if lx is None else lx, 25.0 * ny, b_tesla=5.0, dt_fs=5.0,
              steps=steps, sigma_x=20.0, seed=seed, sym=sym, sx=sx)
    return w


# The last four reach the three-stage line kernels of the reverse sweep (n = 96, 128, 256).
# Every box lets the packets feel the potential within the recorded steps, so that dL/dV is
# well above the rounding of its sums (largest |dL/dV| / L: 2e-4 at 128x8, 1.6e-3 at 256x6).
@pytest.mark.parametrize("nx,ny,steps,ck,sym,lx,sx", [(8, 8, 6, 2, -1, None, 30.0),
                                                      (16, 8, 7, 3, -1, None, 30.0),
                                                      (8, 12, 5, 10, 0, None, 30.0),
                                                      (12, 16, 9, 4, 1, None, 30.0),
                                                      (128, 8, 5, 2, -1, None, 30.0),
                                                      (4, 96, 5, 3, -1, None, 30.0),
                                                      (256, 6, 4, 2, 1, 1280.0, 60.0),
                                                      (8, 128, 3, 2, 0, None, 30.0)])
def test_grad_vs_oracle_stored_adjoint(nx, ny, steps, ck, sym, lx, sx):
    from paper_1903_02581_amd import Propagator
    w = _case(nx, ny, steps, sym, lx=lx, sx=sx)
    announce(f"grad fp64 {nx}x{ny} steps={steps} ckpt={ck} sym={sym}")
    g = grid_of(w)
    psi0 = O.init_state(w.psi_a, w.psi_b, sym)
    L, gv, gb = O.loss_and_grad_stored(psi0, g, w.v_table, w.dt_fs, steps, w.w_top)
    p = Propagator.from_workload(w)
    p.init_state(w.psi_a, w.psi_b, sym)
    p.grad_begin(ck, steps)
    p.step(steps)
    L2, gv2, gb2 = p.grad_backward(w.w_top)
    assert abs(L - L2) <= 1e-12
    assert np.max(np.abs(gv - gv2)) <= 1e-10 * np.max(np.abs(gv))
    assert abs(gb - gb2) <= 1e-10 * max(abs(gb), 1e-12)
    assert abs(gv2.sum()) <= 1e-10 * np.abs(gv2).sum()
    # the state is back at the start of the recording
    back = p.store_state()
    assert np.max(np.abs(back - psi0)) <= 1e-13
    p.close()


def test_recording_refuses_steps_past_the_pool():
    """A recorded step whose checkpoints would not fit the pool is refused before anything
    runs: state, step count and recording are unchanged, and the reverse sweep of the
    recording still matches the oracle.  A step that exceeds the pool after a refusal is
    refused again, and a closed recording gives ESTATE."""
    from paper_1903_02581_amd import Propagator
    from paper_1903_02581_amd.hom4d import Hom4dError
    w = _case(8, 8, 6, -1)
    announce("grad recording: ENOMEM before any step")
    g = grid_of(w)
    psi0 = O.init_state(w.psi_a, w.psi_b, -1)
    p = Propagator.from_workload(w)
    ck, steps = 2, 6
    p.grad_begin(ck, steps)               # pool sized for 6 steps: 4 slots
    p.step(4)
    before = p.store_state()
    step_before = p.observables(w.w_top)["step"]
    # 8 and 104 recorded steps would reach slots 4 and 52; 2^62 and 2^63 - 1 more steps would
    # overflow a byte count or the step count itself
    for n in (4, 100, 2 ** 62, 2 ** 63 - 1):
        with pytest.raises(Hom4dError) as e:
            p.step(n)
        assert e.value.status == -4
        assert p.observables(w.w_top)["step"] == step_before
        assert np.array_equal(p.store_state(), before)
    p.step(2)                             # still fits: 6 steps, slot 3
    L, gv, gb = O.loss_and_grad_stored(psi0, g, w.v_table, w.dt_fs, steps, w.w_top)
    L2, gv2, gb2 = p.grad_backward(w.w_top)
    assert abs(L - L2) <= 1e-12
    assert np.max(np.abs(gv - gv2)) <= 1e-10 * np.max(np.abs(gv))
    assert abs(gb - gb2) <= 1e-10 * abs(gb)
    with pytest.raises(Hom4dError) as e:
        p.grad_backward(w.w_top)
    assert e.value.status == -3
    p.close()


def test_grad_mixed_close_to_fp64():
    from paper_1903_02581_amd import Propagator
    w = _case(16, 16, 20)
    announce("grad mixed 16x16 steps=20")
    out = {}
    for prec in ("fp64", "mixed"):
        p = Propagator.from_workload(w, precision=prec)
        p.grad_begin(5, w.steps)
        p.step(w.steps)
        out[prec] = p.grad_backward(w.w_top)
        p.close()
    (l1, v1, b1), (l2, v2, b2) = out["fp64"], out["mixed"]
    assert abs(l1 - l2) <= 1e-5
    assert np.max(np.abs(v1 - v2)) <= 1e-4 * np.max(np.abs(v1))
    assert abs(b1 - b2) <= 1e-4 * abs(b1)


def test_bunching_loss_autograd_vs_finite_differences():
    import torch
    from paper_1903_02581_amd import Propagator
    from paper_1903_02581_amd.autograd import bunching_loss, saddle_potential
    w = _case(12, 12, 8)
    announce("autograd BunchingLoss 12x12 steps=8")
    x = torch.tensor(-0.5 * w.lx + np.arange(w.nx) * (w.lx / w.nx), dtype=torch.float64)
    y = torch.tensor(-0.5 * w.ly + np.arange(w.ny) * (w.ly / w.ny), dtype=torch.float64)
    p = Propagator.from_workload(w)

    def loss_of(th, b):
        v = saddle_potential(th, x, y, w.ly)
        return bunching_loss(v, b, p, w.psi_a, w.psi_b, steps=w.steps, w_top=w.w_top,
                             ckpt_every=3)

    th = torch.tensor([w.v0, w.v1, w.sx, w.sy], dtype=torch.float64, requires_grad=True)
    b = torch.tensor(w.b_tesla, dtype=torch.float64, requires_grad=True)
    L = loss_of(th, b)
    L.backward()
    grads = np.concatenate([th.grad.numpy(), [b.grad.item()]])
    base = np.array([w.v0, w.v1, w.sx, w.sy, w.b_tesla])
    fd = np.empty(5)
    for i in range(5):
        h = 1e-4 * abs(base[i])
        vals = []
        for s in (+1, -1):
            t = base.copy()
            t[i] += s * h
            with torch.no_grad():
                vals.append(float(loss_of(torch.tensor(t[:4]), torch.tensor(t[4]))))
        fd[i] = (vals[0] - vals[1]) / (2 * h)
    for a, f in zip(grads, fd):
        assert abs(a - f) <= 1e-6 * max(abs(f), 1e-9), (grads, fd)
    p.close()
