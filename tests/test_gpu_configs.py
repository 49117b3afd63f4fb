"""The named workloads at their full sizes and step counts, in the launch
configuration the benchmark times (the default three-pass plan where it is
built).  Where the FP64 oracle cannot follow a full run, the checks are
(a) the oracle itself on a short run at the full size, (b) properties that
hold at any size -- norm, exchange antisymmetry on sampled pairs, P_TB = P_BT,
sum of region probabilities = norm -- and (c) the exact factorisation of the
4D propagation into 2D one-electron propagations when V12 = 0 (computed by the
oracle in 2D), compared point by point on samples and through the region
probabilities."""
import numpy as np
import pytest

import oracle as O
from workloads import preset
from workloads.presets import mid_sweep
from tests.gpu_util import announce, grid_of, oracle_run, rel_l2

pytestmark = pytest.mark.gpu


def _pairs(nx, ny, count, seed):
    rng = np.random.default_rng(seed)
    r1 = rng.integers(0, nx * ny, count)
    r2 = rng.integers(0, nx * ny, count)
    return r1, r2


def _factorised_reference(w, steps):
    """Oracle in 2D: antisymmetrised product of the two propagated orbitals (V12 = 0)."""
    g = grid_of(w, coulomb_c=0.0)
    a = O.propagate_2d(w.psi_a, g, w.v_table, w.dt_fs, steps)
    b = O.propagate_2d(w.psi_b, g, w.v_table, w.dt_fs, steps)
    ab = np.vdot(w.psi_a, w.psi_b)
    scale = np.sqrt(2.0 * (1.0 - abs(ab) ** 2))
    return a, b, scale


def _check_factorised(psi_flat_get, w, a, b, scale, tol, seed=0):
    nxy = w.nx * w.ny
    r1, r2 = _pairs(w.nx, w.ny, 4000, seed)
    af, bf = a.ravel(), b.ravel()
    ref = (af[r1] * bf[r2] - bf[r1] * af[r2]) / scale
    got = psi_flat_get(r1 * nxy + r2)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= tol, err
    wt = w.w_top.ravel()
    ta, tb = np.vdot(af, wt * af).real, np.vdot(bf, wt * bf).real
    tab, ovl = np.vdot(af, wt * bf), np.vdot(af, bf)
    p_tt = (ta * tb - abs(tab) ** 2) / (1 - abs(ovl) ** 2)
    return p_tt


def _props(psi, w, tol):
    nxy = w.nx * w.ny
    m = psi.reshape(nxy, nxy)
    r1, r2 = _pairs(w.nx, w.ny, 20000, 1)
    assert np.max(np.abs(m[r1, r2] + m[r2, r1])) <= tol * np.max(np.abs(m))


@pytest.mark.parametrize("run", list(range(9)))
def test_mid_sweep_full_length_properties(run):
    from paper_1903_02581_amd import Propagator
    w = preset("mid", run=run)
    v0, sig = mid_sweep()[run]
    announce(f"mid sweep run {run} (V0={v0:.3f}, sigma={sig}) 64x64 steps={w.steps}")
    p = Propagator.from_workload(w)
    assert p.passes_per_step == 3
    p.step(w.steps)
    o = p.observables(w.w_top)
    psi = p.store_state()
    p.close()
    assert abs(o["norm"] - 1.0) <= 1e-10
    assert abs(o["p_tb"] - o["p_bt"]) <= 1e-12
    assert abs(o["p_tt"] + o["p_tb"] + o["p_bt"] + o["p_bb"] - o["norm"]) <= 1e-12
    _props(psi, w, 1e-12)
    announce(f"mid run {run}: P_b={o['p_b']:.12f} norm-1={o['norm'] - 1:.2e}")


def test_mid_short_run_vs_oracle():
    from paper_1903_02581_amd import Propagator
    w = preset("mid", run=4)
    announce("mid 64x64 vs oracle, 3 steps")
    p = Propagator.from_workload(w)
    p.step(3)
    psi = p.store_state()
    p.close()
    ref, _ = oracle_run(w, 3)
    assert rel_l2(psi, ref) <= 1e-10


def test_mid_full_length_factorisation_without_coulomb():
    from paper_1903_02581_amd import Propagator
    w = preset("mid", run=0, coulomb_c=0.0)
    announce(f"mid 64x64 V12=0 steps={w.steps} vs 2D oracle")
    p = Propagator.from_workload(w)
    p.step(w.steps)
    o = p.observables(w.w_top)
    flat = p.psi  # device tensor, canonical order

    def get(idx):
        import torch
        return flat[torch.as_tensor(idx, device=flat.device)].cpu().numpy()

    a, b, scale = _factorised_reference(w, w.steps)
    p_tt = _check_factorised(get, w, a, b, scale, 1e-10)
    assert abs(o["p_tt"] - p_tt) <= 1e-10
    p.close()


def test_mixed_config_error_budget():
    """128x96 per electron, 5000 steps, complex64 storage against the FP64 GPU run."""
    from paper_1903_02581_amd import Propagator
    w = preset("mixed")
    announce(f"mixed config 128x96 steps={w.steps}: fp64 run")
    res = {}
    for prec in ("fp64", "mixed"):
        p = Propagator.from_workload(w, precision=prec)
        p.set_norm_tol(1.0)
        samples = []
        for _ in range(w.steps // 500):
            p.step(500)
            samples.append(p.observables(w.w_top)["p_b"])
        o = p.observables(w.w_top)
        res[prec] = (o, samples, p.store_state())
        p.close()
        announce(f"mixed config: {prec} done, P_b={o['p_b']:.10f} norm={o['norm']:.12f}")
    (o64, s64, psi64), (o32, s32, psi32) = res["fp64"], res["mixed"]
    d_pb = max(abs(x - y) for x, y in zip(s64, s32))
    err = rel_l2(psi32, psi64)
    announce(f"mixed config errors: max|dPb|={d_pb:.3e} relL2={err:.3e} "
             f"dnorm={abs(o32['norm'] - o64['norm']):.3e}")
    assert d_pb <= 1e-4
    assert err <= 1e-4
    assert abs(o32["norm"] - o64["norm"]) <= 1e-4
    assert abs(o64["norm"] - 1.0) <= 1e-10


@pytest.mark.parametrize("mode", ["table", "direct"])
def test_mixed_config_coulomb_vs_oracle(mode):
    """128x96 per electron with the softened Coulomb term on (d = 1 nm), two steps in the
    launch configuration the benchmark times (four passes, three-stage kernels at n = 96 and
    128, non-temporal state accesses past 1 GiB), both storages, against the FP64 oracle:
    relative L2 of the whole state and the region probabilities."""
    import torch
    from paper_1903_02581_amd import Propagator
    w = preset("mixed")
    steps = 2
    announce(f"mixed config 128x96 Coulomb on ({mode}) steps={steps} vs oracle, both storages")
    ref, _ = _mixed_oracle_two_steps(w, steps)
    ro = O.observables(ref, w.w_top)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        p = Propagator.from_workload(w, precision=prec, coulomb_mode=mode)
        assert p.passes_per_step == 4
        p.step(steps)
        o = p.observables(w.w_top)
        psi = p.store_state()
        p.close()
        del p
        torch.cuda.empty_cache()
        err = rel_l2(psi, ref)
        announce(f"128x96 Coulomb {mode} {prec}: rel L2 {err:.3e}, |dP_b| {abs(o['p_b'] - ro['p_b']):.3e}")
        assert err <= tol
        for k in ("p_tt", "p_tb", "p_bt", "p_bb", "norm"):
            assert abs(o[k] - ro[k]) <= (1e-12 if prec == "fp64" else 1e-5), k
        del psi


_ORACLE_CACHE = {}


def _mixed_oracle_two_steps(w, steps):
    key = (w.name, steps)
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE.clear()
        _ORACLE_CACHE[key] = oracle_run(w, steps)
    return _ORACLE_CACHE[key]


def test_mixed_config_factorisation_without_coulomb():
    from paper_1903_02581_amd import Propagator
    w = preset("mixed", coulomb_c=0.0)
    steps = 1000
    announce(f"mixed config 128x96 V12=0 steps={steps} vs 2D oracle, both precisions")
    a, b, scale = _factorised_reference(w, steps)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        p = Propagator.from_workload(w, precision=prec)
        p.step(steps)
        o = p.observables(w.w_top)
        flat = p.psi

        def get(idx):
            import torch
            return flat[torch.as_tensor(idx, device=flat.device)].cpu().numpy().astype(np.complex128)

        p_tt = _check_factorised(get, w, a, b, scale, tol)
        assert abs(o["p_tt"] - p_tt) <= tol
        p.close()


def test_full_scale_short_run():
    """256x128 per electron (1.07e9 points): mixed against FP64 and against the 2D oracle."""
    from paper_1903_02581_amd import Propagator
    w = preset("full", coulomb_c=0.0)
    steps = 40
    announce(f"full 256x128 V12=0 steps={steps} both precisions")
    a, b, scale = _factorised_reference(w, steps)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        p = Propagator.from_workload(w, precision=prec)
        p.step(steps)
        o = p.observables(w.w_top)
        flat = p.psi

        def get(idx):
            import torch
            return flat[torch.as_tensor(idx, device=flat.device)].cpu().numpy().astype(np.complex128)

        p_tt = _check_factorised(get, w, a, b, scale, tol)
        assert abs(o["p_tt"] - p_tt) <= tol
        assert abs(o["norm"] - 1.0) <= (1e-10 if prec == "fp64" else 1e-4)
        p.close()
        del p, flat
        import torch
        torch.cuda.empty_cache()


def test_large_state_short_y_axis():
    """256x64 per electron (2.7e8 points; FP64 state 4.3 GB, complex64 2.1 GB): past 1 GiB every
    pass takes non-temporal state accesses, including the two-stage kernel of the n = 64 y lines.
    Both precisions against the 2D oracle through the V12 = 0 factorisation, then a short
    adjoint (dual-state passes with the same cache policy): FP64 against complex64 and the gauge
    identity sum dL/dV = 0."""
    import torch
    from workloads.presets import build
    from paper_1903_02581_amd import Propagator
    w = build("wide", 256, 64, 2000.0, 500.0, b_tesla=5.0, dt_fs=0.5, steps=12, sigma_x=20.0,
              coulomb_c=0.0, seed=7)
    announce(f"256x64 ({w.points} points) V12=0 steps={w.steps} both precisions + adjoint")
    a, b, scale = _factorised_reference(w, w.steps)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        p = Propagator.from_workload(w, precision=prec)
        assert p.passes_per_step == 4
        p.step(w.steps)
        o = p.observables(w.w_top)
        flat = p.psi

        def get(idx):
            return flat[torch.as_tensor(idx, device=flat.device)].cpu().numpy().astype(np.complex128)

        p_tt = _check_factorised(get, w, a, b, scale, tol, seed=3)
        assert abs(o["p_tt"] - p_tt) <= tol
        p.close()
        del p, flat
        torch.cuda.empty_cache()
    res = {}
    for prec in ("fp64", "mixed"):
        p = Propagator.from_workload(w, precision=prec)
        p.set_norm_tol(1.0)
        p.grad_begin(4, 8)
        p.step(8)
        res[prec] = p.grad_backward(w.w_top)
        p.close()
        del p
        torch.cuda.empty_cache()
    (l64, v64, b64), (l32, v32, b32) = res["fp64"], res["mixed"]
    assert np.all(np.isfinite(v64)) and np.isfinite(b64)
    assert abs(v64.sum()) <= 1e-10 * np.abs(v64).sum()
    assert abs(l32 - l64) <= 1e-6 * max(abs(l64), 1e-12) + 1e-12
    assert np.max(np.abs(v32 - v64)) <= 1e-4 * np.max(np.abs(v64))
    assert abs(b32 - b64) <= 1e-4 * abs(b64) + 1e-12


def test_maximum_size_256x256():
    """The largest supported grid, 256x256 per electron: 4.3e9 points, past 32-bit point
    indices (a complex128 state of 68.7 GB, complex64 34.4 GB).  Both precisions against the
    2D oracle through the V12 = 0 factorisation, on sampled points and P_TT."""
    from workloads.presets import build
    from paper_1903_02581_amd import Propagator
    import torch
    w = build("max", 256, 256, 2000.0, 2000.0, b_tesla=5.0, dt_fs=0.5, steps=3, sigma_x=20.0,
              coulomb_c=0.0, seed=5)
    announce(f"maximum size 256x256 ({w.points} points) V12=0 steps={w.steps} both precisions")
    a, b, scale = _factorised_reference(w, w.steps)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-4)):
        p = Propagator.from_workload(w, precision=prec)
        assert p.passes_per_step == 4
        p.step(w.steps)
        o = p.observables(w.w_top)
        flat = p.psi
        assert flat.numel() == w.points

        def get(idx):
            return flat[torch.as_tensor(idx, device=flat.device)].cpu().numpy().astype(np.complex128)

        # samples reach the last r1 rows, beyond 2^32 elements
        p_tt = _check_factorised(get, w, a, b, scale, tol)
        r1 = np.arange(w.nx * w.ny - 64, w.nx * w.ny)
        r2 = np.arange(64)
        af, bf = a.ravel(), b.ravel()
        ref = (af[r1] * bf[r2] - bf[r1] * af[r2]) / scale
        got = get(r1 * (w.nx * w.ny) + r2)
        amp = np.max(np.abs(af)) * np.max(np.abs(bf)) / scale      # scale of |Psi| anywhere
        assert np.max(np.abs(got - ref)) <= tol * amp
        assert abs(o["p_tt"] - p_tt) <= tol
        assert abs(o["norm"] - 1.0) <= (1e-10 if prec == "fp64" else 1e-4)
        announce(f"maximum size {prec}: norm-1={o['norm'] - 1:.2e} P_TT={o['p_tt']:.10f} (2D oracle {p_tt:.10f})")
        p.close()
        del p, flat
        torch.cuda.empty_cache()


def test_diff_config_gradient_vs_finite_differences():
    """48x48 per electron, 1000 steps, checkpoint every 100: adjoint dP_b/d(V0, V1, sx, sy, B)
    against central differences (h = 1e-4 relative) of the FP64 GPU forward run, and the
    mixed-precision adjoint against the FP64 one."""
    import torch
    from paper_1903_02581_amd import Propagator
    from paper_1903_02581_amd.autograd import bunching_loss, saddle_potential
    w = preset("diff")
    announce(f"diff config 48x48 steps={w.steps} adjoint vs FD")
    x = torch.tensor(-0.5 * w.lx + np.arange(w.nx) * (w.lx / w.nx), dtype=torch.float64)
    y = torch.tensor(-0.5 * w.ly + np.arange(w.ny) * (w.ly / w.ny), dtype=torch.float64)
    base = np.array([w.v0, w.v1, w.sx, w.sy, w.b_tesla])
    grads = {}
    for prec in ("fp64", "mixed"):
        p = Propagator.from_workload(w, precision=prec)
        p.set_norm_tol(1.0)
        th = torch.tensor(base[:4], dtype=torch.float64, requires_grad=True)
        bb = torch.tensor(base[4], dtype=torch.float64, requires_grad=True)
        L = bunching_loss(saddle_potential(th, x, y, w.ly), bb, p, w.psi_a, w.psi_b,
                          steps=w.steps, w_top=w.w_top, ckpt_every=w.ckpt_every)
        L.backward()
        grads[prec] = np.concatenate([th.grad.numpy(), [bb.grad.item()]])
        if prec == "fp64":
            fd = np.empty(5)
            for i in range(5):
                h = 1e-4 * abs(base[i])
                vals = []
                for sgn in (+1, -1):
                    t = base.copy()
                    t[i] += sgn * h
                    with torch.no_grad():
                        vals.append(float(bunching_loss(
                            saddle_potential(torch.tensor(t[:4]), x, y, w.ly), torch.tensor(t[4]),
                            p, w.psi_a, w.psi_b, steps=w.steps, w_top=w.w_top,
                            ckpt_every=w.ckpt_every)))
                fd[i] = (vals[0] - vals[1]) / (2 * h)
        p.close()
    g64, g32 = grads["fp64"], grads["mixed"]
    announce(f"diff grads fp64={g64} fd={fd} mixed={g32}")
    scale = np.max(np.abs(g64))
    assert np.max(np.abs(g64 - fd)) <= 1e-5 * scale
    assert np.max(np.abs(g32 - g64)) <= 1e-4 * scale


def test_full_scale_adjoint():
    """256x128 per electron (1.07e9 points), the adjoint over 20 recorded steps (checkpoint
    every 10): FP64 against complex64, the gauge identity sum dL/dV = 0, and dL/dB against a
    central difference of two FP64 forward runs (B +- 1e-4 relative)."""
    import torch
    from paper_1903_02581_amd import Propagator
    w = preset("full")
    steps, ck = 20, 10
    announce(f"full 256x128 adjoint steps={steps} ckpt={ck} both precisions + FD in B")
    res = {}
    for prec in ("fp64", "mixed"):
        p = Propagator.from_workload(w, precision=prec)
        p.set_norm_tol(1.0)
        p.grad_begin(ck, steps)
        p.step(steps)
        res[prec] = p.grad_backward(w.w_top)
        p.close()
        del p
        torch.cuda.empty_cache()
    (l64, v64, b64), (l32, v32, b32) = res["fp64"], res["mixed"]
    assert np.all(np.isfinite(v64)) and np.isfinite(b64)
    assert abs(v64.sum()) <= 1e-10 * np.abs(v64).sum()
    assert abs(l32 - l64) <= 1e-6 * max(abs(l64), 1e-12) + 1e-12
    assert np.max(np.abs(v32 - v64)) <= 1e-4 * np.max(np.abs(v64))
    assert abs(b32 - b64) <= 1e-4 * abs(b64)
    h = 1e-4 * w.b_tesla
    lf = []
    for sgn in (1.0, -1.0):
        p = Propagator.from_workload(w)
        p.set_norm_tol(1.0)
        p.set_field(w.b_tesla + sgn * h)
        p.step(steps)
        o = p.observables(w.w_top)
        lf.append(o["p_b"])
        p.close()
        del p
        torch.cuda.empty_cache()
    fd = (lf[0] - lf[1]) / (2 * h)
    announce(f"full adjoint: L={l64:.6e} dL/dB adjoint {b64:.6e} (mixed {b32:.6e}) FD {fd:.6e}")
    assert abs(fd - b64) <= 1e-4 * abs(b64)
