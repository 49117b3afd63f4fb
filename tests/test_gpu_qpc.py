"""The resolving beam-splitter workload on the GPU (128x64 per electron, Fermi-
block constriction of Sec. II.C Eq. (pot_xy), 2500 steps of 1 fs).

Without the two-body term the exact 4D propagation is the antisymmetrised
product of the two orbitals propagated in 2D, so the FP64 oracle gives the
region probabilities at full size from 2D runs (orbital_observables).  The
GPU path (four per-axis passes per step at this size) must match them, and the
sigma sweep reproduces the qualitative result of Sec. III.A: bunching of the
Slater determinant decreases with the packet length, while distinguishable
electrons bunch with probability 1/2 at a balanced splitter, and displacing one
packet along its edge brings the bunching back towards 1/2.  The 1D model of
Sec. III.A Eq. (bunching) at zero displacement, P_b = (1 - sigma^2/Sigma^2)/2
with Sigma^2 = sigma^2 + a^2/(8 gamma), gives one QPC length a per sigma."""
import numpy as np
import pytest

import oracle as O
from workloads import preset
from tests.gpu_util import announce, grid_of

pytestmark = pytest.mark.gpu

SIGMAS = [10.0, 12.5, 15.0, 17.5, 20.0]
GAMMA = 4.0 * np.log(2.0)


def _orbitals(w):
    g = grid_of(w, coulomb_c=0.0)
    a = O.propagate_2d(w.psi_a, g, w.v_table, w.dt_fs, w.steps)
    b = O.propagate_2d(w.psi_b, g, w.v_table, w.dt_fs, w.steps)
    return a, b


def _gpu_obs(w, precision="fp64", sym=None):
    from paper_1903_02581_amd import Propagator
    p = Propagator.from_workload(w, precision=precision)
    if sym is not None:
        p.init_state(w.psi_a, w.psi_b, sym)
    p.step(w.steps)
    o = p.observables(w.w_top)
    p.close()
    return o


def test_sigma_sweep_exchange_only():
    pb = []
    for sig in SIGMAS:
        w = preset("qpc", sigma_x=sig)
        announce(f"qpc 128x64 fp64 sigma={sig} steps={w.steps} V12=0 antisym")
        o = _gpu_obs(w)
        a, b = _orbitals(w)
        ref = O.orbital_observables(a, b, w.w_top, -1)
        for k in ("p_tt", "p_tb", "p_bt", "p_bb", "p_b"):
            assert abs(o[k] - ref[k]) <= 1e-10, (sig, k, o[k], ref[k])
        assert abs(o["norm"] - 1.0) <= 1e-11
        a_fit = np.sqrt(8.0 * GAMMA * sig ** 2 * 2.0 * o["p_b"] / (1.0 - 2.0 * o["p_b"]))
        announce(f"qpc sigma={sig}: P_b={o['p_b']:.10f} (oracle {ref['p_b']:.10f}) a={a_fit:.1f} nm")
        pb.append(o["p_b"])
    assert all(x > y for x, y in zip(pb, pb[1:]))        # decreasing with the packet length
    assert max(pb) < 0.5


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_distinguishable_electrons_bunch_half(precision, tol):
    w = preset("qpc")
    announce(f"qpc 128x64 {precision} product state steps={w.steps}")
    o = _gpu_obs(w, precision=precision, sym=0)
    a, b = _orbitals(w)
    ref = O.orbital_observables(a, b, w.w_top, 0)
    assert abs(o["p_b"] - ref["p_b"]) <= tol
    assert abs(o["p_b"] - 0.5) < 0.01


def test_coulomb_mixed_against_fp64():
    w = preset("qpc", coulomb_c=1.0)
    announce(f"qpc 128x64 Coulomb on (d={w.soft_nm} nm) fp64 vs mixed steps={w.steps}")
    o64 = _gpu_obs(w, "fp64")
    o32 = _gpu_obs(w, "mixed")
    assert abs(o64["norm"] - 1.0) <= 1e-11
    assert abs(o64["p_tb"] - o64["p_bt"]) <= 1e-12
    assert abs(o32["p_b"] - o64["p_b"]) <= 1e-4
    w0 = preset("qpc")
    a, b = _orbitals(w0)
    ref0 = O.orbital_observables(a, b, w0.w_top, -1)
    announce(f"qpc sigma=15: P_b Coulomb {o64['p_b']:.6f} (mixed {o32['p_b']:.6f}), "
             f"exchange only {ref0['p_b']:.6f}")


def test_displaced_packets_recover_half():
    # a displacement between the packets along their edges reduces their overlap at the
    # splitter, and with it the exchange antibunching (Sec. III.B, the displacement axis)
    pb = {}
    for shift in (0.0, 40.0):
        w = preset("qpc", shift_nm=shift, steps=3200)
        announce(f"qpc 128x64 fp64 shift={shift} nm steps={w.steps} V12=0 antisym")
        o = _gpu_obs(w)
        a, b = _orbitals(w)
        ref = O.orbital_observables(a, b, w.w_top, -1)
        assert abs(o["p_b"] - ref["p_b"]) <= 1e-10
        announce(f"qpc shift={shift}: P_b={o['p_b']:.10f} (oracle {ref['p_b']:.10f})")
        pb[shift] = o["p_b"]
    assert pb[40.0] > pb[0.0] + 0.03


def test_exchange_symmetry_orders_bunching():
    # symmetric orbital state bunches above 1/2, the Slater determinant below,
    # distinguishable electrons at 1/2 (Sec. III.A, the two symmetries of Fig. 4)
    w = preset("qpc")
    a, b = _orbitals(w)
    pb = {}
    for sym in (1, 0, -1):
        announce(f"qpc 128x64 fp64 sym={sym} steps={w.steps}")
        o = _gpu_obs(w, sym=sym)
        ref = O.orbital_observables(a, b, w.w_top, sym)
        assert abs(o["p_b"] - ref["p_b"]) <= 1e-10
        pb[sym] = o["p_b"]
    announce(f"qpc P_b symmetric {pb[1]:.6f} product {pb[0]:.6f} antisymmetric {pb[-1]:.6f}")
    assert pb[1] > pb[0] + 0.1 and pb[0] > pb[-1] + 0.1


def test_screened_coulomb_between_bare_and_none():
    # the screened repulsion of Sec. III.B Eq. (screenedCoulomb) (C = 1, sigma_c = 5 nm)
    # is much weaker than the bare one at the electrons' separations, so its bunching
    # stays closer to the exchange-only value than the bare Coulomb bunching does
    from paper_1903_02581_amd import Propagator
    pb = {}
    for label, kw in (("none", dict(coulomb_c=0.0)), ("screened", dict(coulomb_c=1.0)),
                      ("bare", dict(coulomb_c=1.0))):
        w = preset("qpc", **kw)
        announce(f"qpc 128x64 fp64 Coulomb {label} steps={w.steps}")
        extra = dict(screen_nm=5.0) if label == "screened" else {}
        p = Propagator.from_workload(w, **extra)
        p.step(w.steps)
        o = p.observables(w.w_top)
        p.close()
        assert abs(o["norm"] - 1.0) <= 1e-11
        pb[label] = o["p_b"]
    announce(f"qpc P_b bare {pb['bare']:.6f} screened {pb['screened']:.6f} none {pb['none']:.6f}")
    assert pb["bare"] < pb["none"]
    assert abs(pb["screened"] - pb["none"]) < 0.5 * abs(pb["bare"] - pb["none"])


def test_time_resolved_entanglement():
    # spatial entanglement of the slice phi(x1, x2) = Psi(x1, y1*, x2, y2*) (Sec. III.C)
    # with y1*, y2* on the two incoming edges: zero for the incoming product-like state,
    # created by the scattering (0 -> 0.16 here); without the two-body term the slice is
    # built exactly from the two propagated orbitals
    from paper_1903_02581_amd import Propagator
    w = preset("qpc")
    g = grid_of(w, coulomb_c=0.0)
    j1 = int(np.argmax(np.abs(w.psi_a).max(axis=0)))    # row of the top packet
    j2 = int(np.argmax(np.abs(w.psi_b).max(axis=0)))    # row of the bottom packet
    ix = np.arange(w.nx)
    p = Propagator.from_workload(w)
    a, b = w.psi_a.copy(), w.psi_b.copy()
    scale = np.sqrt(2.0 * (1.0 - abs(np.vdot(w.psi_a, w.psi_b)) ** 2))
    done = 0
    s_t = []
    for t in (0, 1000, 2000, 2500):
        if t > done:
            p.step(t - done)
            a = O.propagate_2d(a, g, w.v_table, w.dt_fs, t - done)
            b = O.propagate_2d(b, g, w.v_table, w.dt_fs, t - done)
            done = t
        announce(f"qpc entanglement at step {t}")
        s_gpu = p.entanglement(ix, j1, ix, j2)
        phi = (np.outer(a[:, j1], b[:, j2]) - np.outer(b[:, j1], a[:, j2])) / scale
        s_ref = O.entanglement(phi[:, None, :, None], ix, 0, ix, 0)
        announce(f"qpc S(step {t}) = {s_gpu:.10f} (oracle {s_ref:.10f})")
        assert abs(s_gpu - s_ref) <= 1e-9
        s_t.append(s_gpu)
    p.close()
    assert s_t[0] < 1e-6 and s_t[-1] > 0.1


def test_coulomb_softening_sweep_distinguishable():
    # distinguishable electrons with the softened repulsion (Sec. III.B): strong at a thin
    # 2DEG (d = 1 nm), pushing P_b away from 1/2; a thick one (d = 100 nm) barely couples
    # them and P_b returns towards 1/2
    pb = {}
    for d in (1.0, 100.0):
        w = preset("qpc", coulomb_c=1.0, soft_nm=d, sym=0)
        announce(f"qpc 128x64 fp64 product state d={d} nm steps={w.steps}")
        o = _gpu_obs(w)
        assert abs(o["norm"] - 1.0) <= 1e-11
        pb[d] = o["p_b"]
    announce(f"qpc product state P_b d=1: {pb[1.0]:.6f}, d=100: {pb[100.0]:.6f}")
    assert abs(pb[100.0] - 0.5) < abs(pb[1.0] - 0.5)
