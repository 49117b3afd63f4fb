"""GPU path (libhom4d.so through the C ABI) against the FP64 CPU oracle.

Bar: relative L2 error of the final state <= 1e-10 for the FP64 path and
<= 1e-4 for the mixed (complex64-storage) path; observables compared too.
"""
import numpy as np
import pytest

import oracle as O
from workloads import preset
from workloads.presets import build, replace
from tests.gpu_util import announce, gpu_run, grid_of, oracle_run, rel_l2

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


def test_tiny_fp64_full_run():
    w = preset("tiny")
    announce(f"tiny fp64 {w.nx}x{w.ny} steps={w.steps}")
    psi, obs = gpu_run(w, w.steps)
    ref, _ = oracle_run(w, w.steps)
    assert rel_l2(psi, ref) <= FP64_TOL
    ro = O.observables(ref, w.w_top)
    for k in ("norm", "p_tt", "p_tb", "p_bt", "p_bb", "p_b", "p_ab"):
        assert abs(obs[k] - ro[k]) <= 1e-12, (k, obs[k], ro[k])
    assert obs["step"] == w.steps


# every supported line length appears on the x axes and on the y axes; (n, m) pairs keep
# the 4D state near 1e6 points so the oracle stays fast
SIZES = [(4, 6), (6, 4), (8, 12), (12, 8), (16, 24), (24, 16), (32, 12), (12, 32),
         (48, 16), (16, 48), (64, 8), (8, 64), (96, 8), (8, 96), (128, 4), (4, 128),
         (256, 4), (4, 256)]


@pytest.mark.parametrize("nx,ny", SIZES)
def test_sizes_fp64(nx, ny):
    w = build("sz", nx, ny, 10.0 * nx, 12.0 * ny, b_tesla=5.0, dt_fs=2.0, steps=4,
              sigma_x=max(10.0, 2.0 * nx), seed=nx + ny)
    announce(f"sizes fp64 {nx}x{ny} steps={w.steps}")
    psi, obs = gpu_run(w, w.steps)
    ref, _ = oracle_run(w, w.steps)
    assert rel_l2(psi, ref) <= FP64_TOL


@pytest.mark.parametrize("nx,ny", [(16, 16), (48, 16), (16, 96), (256, 8), (8, 256), (128, 12)])
def test_sizes_mixed(nx, ny):
    w = build("szm", nx, ny, 10.0 * nx, 12.0 * ny, b_tesla=5.0, dt_fs=2.0, steps=20,
              sigma_x=20.0, seed=3)
    announce(f"sizes mixed {nx}x{ny} steps={w.steps}")
    psi, obs = gpu_run(w, w.steps, precision="mixed")
    ref, _ = oracle_run(w, w.steps)
    assert rel_l2(psi, ref) <= MIXED_TOL
    ro = O.observables(ref, w.w_top)
    assert abs(obs["p_b"] - ro["p_b"]) <= MIXED_TOL


def test_tiny_mixed_full_run():
    w = preset("tiny")
    announce(f"tiny mixed steps={w.steps}")
    psi, obs = gpu_run(w, w.steps, precision="mixed")
    ref, _ = oracle_run(w, w.steps)
    err = rel_l2(psi, ref)
    ro = O.observables(ref, w.w_top)
    announce(f"tiny mixed rel_l2={err:.3e} dPb={abs(obs['p_b'] - ro['p_b']):.3e} "
             f"dnorm={abs(obs['norm'] - ro['norm']):.3e}")
    assert err <= MIXED_TOL
    assert abs(obs["p_b"] - ro["p_b"]) <= MIXED_TOL
    assert abs(obs["norm"] - ro["norm"]) <= MIXED_TOL


def test_direct_coulomb_mode():
    w = preset("tiny")
    announce("tiny fp64 direct coulomb steps=50")
    psi, _ = gpu_run(w, 50, coulomb_mode="direct")
    ref, _ = oracle_run(w, 50)
    assert rel_l2(psi, ref) <= FP64_TOL


def test_screened_coulomb():
    w = preset("tiny")
    announce("tiny fp64 screened steps=50")
    for mode in ("table", "direct"):
        psi, _ = gpu_run(w, 50, coulomb_mode=mode, screen_nm=5.0)
        ref, _ = oracle_run(w, 50, screen_nm=5.0)
        assert rel_l2(psi, ref) <= FP64_TOL


def test_coulomb_off():
    w = preset("tiny", coulomb_c=0.0)
    announce("tiny fp64 coulomb off steps=50")
    psi, _ = gpu_run(w, 50)
    ref, _ = oracle_run(w, 50)
    assert rel_l2(psi, ref) <= FP64_TOL


@pytest.mark.parametrize("sym", [1, 0])
def test_symmetric_and_product_states(sym):
    w = preset("tiny")
    announce(f"tiny fp64 sym={sym} steps=50")
    psi, obs = gpu_run(w, 50, sym=sym)
    ref, _ = oracle_run(w, 50, sym=sym)
    assert rel_l2(psi, ref) <= FP64_TOL
    ro = O.observables(ref, w.w_top)
    assert abs(obs["p_b"] - ro["p_b"]) <= 1e-12


def test_zero_steps_is_identity_and_init_matches():
    w = preset("tiny")
    announce("init only")
    psi, obs = gpu_run(w, 0)
    ref = O.init_state(w.psi_a, w.psi_b, -1)
    assert rel_l2(psi, ref) <= 1e-14
    assert abs(obs["norm"] - 1.0) <= 1e-13


def test_entanglement_and_slice():
    from paper_1903_02581_amd import Propagator
    w = preset("tiny")
    announce("entanglement tiny")
    p = Propagator.from_workload(w)
    p.step(40)
    psi = p.store_state()
    y = -0.5 * w.ly + np.arange(w.ny) * (w.ly / w.ny)
    j1 = int(np.argmin(np.abs(y - 11.5)))
    j2 = int(np.argmin(np.abs(y + 11.5)))
    ix = np.arange(w.nx)
    s_gpu = p.entanglement(ix, j1, ix, j2)
    s_ref = O.entanglement(psi, ix, j1, ix, j2)
    assert abs(s_gpu - s_ref) <= 1e-10
    sl = p.gather_slice(ix[::2], j1, ix[1::3], j2)
    assert np.array_equal(sl, psi[ix[::2], j1][:, ix[1::3], j2])
    p.close()


def test_load_store_roundtrip_and_determinism():
    from paper_1903_02581_amd import Propagator
    w = preset("tiny")
    announce("load/store + determinism")
    rng = np.random.default_rng(0)
    n = (w.nx * w.ny) ** 2
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for prec in ("fp64", "mixed"):
        p = Propagator.from_workload(w, precision=prec)
        p.load_state(x)
        back = p.store_state().ravel()
        if prec == "fp64":
            assert np.array_equal(back, x)
        else:
            assert np.array_equal(back, x.astype(np.complex64).astype(np.complex128))
        p.close()
    a, _ = gpu_run(w, 30)
    b, _ = gpu_run(w, 30)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name,precision", [("tiny", "fp64"), ("mid", "fp64"), ("mid", "mixed")])
def test_resume_from_stored_state_is_bitwise(name, precision):
    # checkpoint/resume: store after step(k), destroy the propagator, build a new one, load
    # the stored state and continue; the trajectory must equal step(k), step(rest) on one
    # propagator bit for bit (the mixed path stores complex64 exactly in complex128, so its
    # round trip is exact too).  One call step(k + rest) merges the two half-step x kinetic
    # factors at the seam into one, so it agrees only to rounding.
    from paper_1903_02581_amd import Propagator
    w = preset(name)
    k, rest = 7, 5
    announce(f"resume {name} {w.nx}x{w.ny} {precision} k={k} rest={rest}")
    p = Propagator.from_workload(w, precision=precision)
    p.step(k)
    p.step(rest)
    straight = p.store_state()
    o_straight = p.observables(w.w_top)
    p.close()
    p = Propagator.from_workload(w, precision=precision)
    p.step(k + rest)
    merged = p.store_state()
    p.close()
    assert rel_l2(merged, straight) <= (1e-13 if precision == "fp64" else 1e-6)
    p = Propagator.from_workload(w, precision=precision)
    p.step(k)
    saved = p.store_state()
    p.close()
    del p
    q = Propagator.from_workload(w, precision=precision)
    q.load_state(saved)
    assert q.observables(w.w_top)["step"] == 0       # loading restarts the step counter
    q.step(rest)
    resumed = q.store_state()
    o_resumed = q.observables(w.w_top)
    q.close()
    assert np.array_equal(resumed, straight)
    for key in ("norm", "p_tt", "p_tb", "p_bt", "p_bb", "p_b", "p_ab"):
        assert o_resumed[key] == o_straight[key], key


def test_step_zero_is_identity():
    # step(0) applies nothing: not even the opening and closing half-step x factors
    from paper_1903_02581_amd import Propagator
    w = preset("tiny")
    announce("step(0) identity (tiny, both plans)")
    for plan in (0, 1):
        p = Propagator.from_workload(w)
        p.set_pass_plan(plan)
        p.step(2)
        before = p.store_state()
        p.step(0)
        assert np.array_equal(p.store_state(), before)
        assert p.observables(w.w_top)["step"] == 2
        p.close()


# Determinism as the race detector: no float atomics, fixed-order reductions, so any
# missing synchronisation between LDS writes and reads shows up as run-to-run differences.
# Every supported line length on both axes, the fused plane sizes, both storages, and the
# dual-state reverse kernels, each run twice in fresh propagators.
REPEAT_SIZES = SIZES + [(16, 16), (24, 24), (32, 32), (48, 48), (64, 64), (48, 16), (16, 48)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bitwise_repeatable_every_size(precision):
    from paper_1903_02581_amd import Propagator
    announce(f"bitwise repeatability, {len(REPEAT_SIZES)} shapes, {precision}")
    for nx, ny in REPEAT_SIZES:
        w = build("rep", nx, ny, 10.0 * nx, 12.0 * ny, b_tesla=5.0, dt_fs=2.0, steps=3,
                  sigma_x=max(10.0, 2.0 * nx), seed=nx * ny)
        runs = []
        for _ in range(2):
            p = Propagator.from_workload(w, precision=precision)
            p.step(3)
            runs.append(p.store_state())
            p.close()
        assert np.array_equal(runs[0], runs[1]), (nx, ny, precision)


@pytest.mark.parametrize("nx,ny", [(128, 4), (4, 96), (256, 4), (8, 128), (16, 16)])
def test_reverse_sweep_bitwise_repeatable(nx, ny):
    from paper_1903_02581_amd import Propagator
    w = build("rep", nx, ny, 25.0 * nx, 25.0 * ny, b_tesla=5.0, dt_fs=5.0, steps=4,
              sigma_x=20.0, seed=2)
    announce(f"reverse sweep repeatability {nx}x{ny}")
    out = []
    for _ in range(2):
        p = Propagator.from_workload(w)
        p.grad_begin(2, 4)
        p.step(4)
        out.append(p.grad_backward(w.w_top))
        p.close()
    (l1, v1, b1), (l2, v2, b2) = out
    assert l1 == l2 and b1 == b2 and np.array_equal(v1, v2)


def test_watchdog_and_errors():
    from paper_1903_02581_amd import Propagator, Hom4dError
    w = preset("tiny")
    announce("watchdog and error paths")
    p = Propagator.from_workload(w)
    n = (w.nx * w.ny) ** 2
    bad = np.zeros(n, complex)
    bad[5] = np.nan
    p.load_state(bad)
    o = p.observables(w.w_top)
    assert o["status"] == -6
    with pytest.raises(Hom4dError):
        p.step(-1)
    with pytest.raises(Hom4dError):
        p.observables(np.full((w.nx, w.ny), 2.0))
    with pytest.raises(Hom4dError):
        p.entanglement([0, 99], 0, [0], 0)
    with pytest.raises(Hom4dError):
        p.init_state(w.psi_a, w.psi_a, -1)      # antisymmetrised identical orbitals: zero norm
    with pytest.raises(Hom4dError):
        p.grad_backward(w.w_top)                 # no recording
    for change in (lambda: p.set_field(w.b_tesla + 0.1), lambda: p.set_potential(w.v_table)):
        p.init_state(w.psi_a, w.psi_b, -1)
        p.grad_begin(2, 2)
        p.step(2)
        change()                                 # the recording used the old factors
        with pytest.raises(Hom4dError):
            p.grad_backward(w.w_top)
    p.set_field(w.b_tesla)
    p.init_state(w.psi_a, w.psi_b, -1)
    p.step(3)
    p.set_norm_tol(1e-300)
    with pytest.raises(Hom4dError):
        p.observables(w.w_top, check=True)
    p.close()


def test_marginal_and_conditional_densities():
    from paper_1903_02581_amd import Propagator
    w = preset("tiny")
    announce("marginal / conditional densities tiny")
    for prec, tol in (("fp64", 1e-13), ("mixed", 1e-6)):
        p = Propagator.from_workload(w, precision=prec)
        p.step(40)
        psi = p.store_state()
        m = p.marginal()
        assert np.max(np.abs(m - O.marginal(psi))) <= tol * np.max(m)
        assert abs(m.sum() - 1.0) <= (1e-12 if prec == "fp64" else 1e-5)
        for (ix2, jy2) in [(3, 11), (12, 4)]:
            c = p.conditional(ix2, jy2)
            assert np.array_equal(c, O.conditional(psi, ix2, jy2)) or \
                np.max(np.abs(c - O.conditional(psi, ix2, jy2))) <= 1e-15
            # Pauli node at r1 = r2*: exact zero up to the storage rounding
            assert c[ix2, jy2] <= (1e-20 if prec == "fp64" else 1e-9) * c.max()
        p.close()


def test_zero_field_and_identical_orbitals():
    # B = 0: the x kinetic factor loses its y dependence (free motion along x)
    w = preset("tiny", b_tesla=0.0)
    announce("tiny fp64 B=0 steps=50")
    psi, _ = gpu_run(w, 50)
    ref, _ = oracle_run(w, 50)
    assert rel_l2(psi, ref) <= FP64_TOL
    # the symmetric state of two identical orbitals (a doubly occupied orbital)
    announce("tiny fp64 identical orbitals sym=+1 steps=50")
    w2 = replace(preset("tiny"), sym=1)
    w2.psi_b = w2.psi_a.copy()
    psi, obs = gpu_run(w2, 50)
    ref = O.propagate(O.init_state(w2.psi_a, w2.psi_a, 1), grid_of(w2), w2.v_table, w2.dt_fs, 50)
    assert rel_l2(psi, ref) <= FP64_TOL
    assert abs(obs["p_tb"] - obs["p_bt"]) <= 1e-12
