"""The reverse sweep without allocation (hom4d_grad_backward_noalloc) against the
allocating entry point (hom4d_grad_backward), through the C ABI: two calls in a
row on one GPU, the second on a smaller grid, so that the second call finds the
fixed device scratch holding the first call's partial sums."""
import numpy as np
import pytest

from workloads.presets import build
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _case(nx, ny, steps, sym, seed):
    return build("g", nx, ny, 25.0 * nx, 25.0 * ny, b_tesla=5.0, dt_fs=5.0, steps=steps,
                 sigma_x=20.0, seed=seed, sym=sym)


def _both(w, ck, precision, coeffs):
    """(allocating result, no-allocation result) of the same recorded run."""
    from paper_1903_02581_amd import Propagator
    out = []
    for noalloc in (False, True):
        p = Propagator.from_workload(w, precision=precision)
        p.grad_begin(ck, w.steps)
        p.step(w.steps)
        out.append(p.grad_backward(w.w_top, coeffs, noalloc=noalloc))
        # the state is back at the start of the recording and the recording closed
        assert p.observables(w.w_top)["step"] == 0
        p.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_allocating_entry_two_calls(precision):
    cases = [(_case(16, 16, 9, -1, 3), 4, (1.0, 0.0, 0.0, 1.0)),   # first call: 16x16
             (_case(8, 12, 5, 0, 4), 2, (0.0, 1.0, 0.5, 0.0))]     # second, smaller: 8x12
    for w, ck, cf in cases:
        announce(f"no-alloc reverse sweep {precision} {w.nx}x{w.ny} steps={w.steps} ckpt={ck}")
        (l1, v1, b1), (l2, v2, b2) = _both(w, ck, precision, cf)
        # the bar of the FP64 path (1e-10 relative); the two share every kernel and the
        # fixed-order reductions, so they agree bit for bit
        assert np.max(np.abs(v2 - v1)) <= 1e-10 * np.max(np.abs(v1))
        assert abs(b2 - b1) <= 1e-10 * abs(b1) and abs(l2 - l1) <= 1e-12
        assert np.array_equal(v1, v2) and b1 == b2 and l1 == l2


def test_noalloc_refusals():
    """A grid whose partial sums exceed the fixed scratch is refused with ENOMEM and the
    recording stays open (the allocating entry point then completes it); with pass timing
    on the call is refused with ESTATE."""
    from paper_1903_02581_amd import Propagator
    from paper_1903_02581_amd.hom4d import Hom4dError
    from workloads import preset
    w = preset("full")                       # 256x128: 13.6M partial sums > 8M
    announce("no-alloc refusals: 256x128 one recorded step")
    p = Propagator.from_workload(w, precision="mixed")
    p.set_norm_tol(1.0)
    p.grad_begin(1, 1)
    p.step(1)
    with pytest.raises(Hom4dError) as e:
        p.grad_backward(w.w_top, noalloc=True)
    assert e.value.status == -4
    loss, dldv, dldb = p.grad_backward(w.w_top)
    assert np.isfinite(loss) and np.all(np.isfinite(dldv)) and np.isfinite(dldb)
    p.close()
    del p
    import torch
    torch.cuda.empty_cache()
    w = _case(8, 8, 3, -1, 5)
    p = Propagator.from_workload(w)
    p.grad_begin(1, 3)
    p.step(3)
    p.pass_timing(True)
    with pytest.raises(Hom4dError) as e:
        p.grad_backward(w.w_top, noalloc=True)
    assert e.value.status == -3
    p.pass_timing(False)
    l2, v2, b2 = p.grad_backward(w.w_top, noalloc=True)
    assert np.isfinite(l2)
    p.close()
