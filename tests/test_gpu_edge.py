"""The edge-state packet generator on the GPU (hom4d_edge_packet: Sec. II.A Eq. (H_effective),
Sec. II.B Eq. (singlepwp)) against the oracle's plain numpy version, at the workloads' grids and
at the extremes of the supported transverse sizes.  Bar: 1e-10 per complex entry (the packets
are normalised, entries up to ~0.1), k0 the same grid wave number, its level to 1e-10 relative."""
import numpy as np
import pytest

import oracle as O
import oracle.edge_states as ES
from workloads import preset
from workloads.presets import build
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _prop(w, precision="fp64"):
    from paper_1903_02581_amd import Propagator
    return Propagator.from_workload(w, precision=precision)


def _grid(w):
    return O.make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, mstar_rel=w.mstar_rel)


def _e_above(w, g):
    # the generator's target level minus hbar omega_c / 2 (= kappa eB / hbar)
    return w.info["alpha"]["target"] - g.kappa * g.e_over_hbar * g.b_tesla


def _check_workload(w, precision="fp64"):
    g = _grid(w)
    ea = _e_above(w, g)
    p = _prop(w, precision)
    try:
        for psi_in, xc, top in ((w.psi_a, w.info["xa"], True), (w.psi_b, w.info["xb"], False)):
            col = int(np.argmin(np.abs(g.x - xc)))
            psi, info = p.edge_packet(w.v_table[col], w.sigma_x, xc, top, ea)
            ref, rinfo = ES.edge_packet(g, w.v_table[col], w.sigma_x, xc, top, ea)
            assert np.max(np.abs(psi - ref)) <= TOL, np.max(np.abs(psi - ref))
            assert np.max(np.abs(psi - psi_in)) <= TOL
            assert abs(info["k0"] - rinfo["k0"]) <= 1e-14 * abs(rinfo["k0"])
            assert abs(info["e1_k0"] - rinfo["e1_k0"]) <= 1e-10 * abs(rinfo["e1_k0"])
            assert abs(info["target"] - rinfo["target"]) <= 1e-12 * abs(rinfo["target"])
            assert abs(np.sum(np.abs(psi) ** 2) - 1.0) <= 1e-13
    finally:
        p.close()


@pytest.mark.parametrize("name", ["tiny", "mid", "qpc", "mixed"])
def test_packets_match_oracle_on_workload_grids(name):
    w = preset(name)
    announce(f"edge packets {name} {w.nx}x{w.ny}")
    _check_workload(w)


def test_packets_full_scale_grid_complex64_handle():
    w = preset("full")
    announce(f"edge packets full {w.nx}x{w.ny} (complex64 handle)")
    _check_workload(w, "mixed")


@pytest.mark.parametrize("nx,ny", [(16, 4), (8, 6), (16, 256), (32, 96)])
def test_packets_extreme_transverse_sizes(nx, ny):
    w = build("edge", nx, ny, 25.0 * nx, 4.0 * ny, b_tesla=5.0, dt_fs=1.0, steps=1,
              sigma_x=12.0, seed=3)
    announce(f"edge packets {nx}x{ny}")
    _check_workload(w)


def test_gpu_packets_drive_the_same_run():
    """A state initialised from the GPU-built packets propagates like the one from the inputs."""
    w = preset("tiny")
    g = _grid(w)
    ea = _e_above(w, g)
    p = _prop(w)
    try:
        pk = []
        for xc, top in ((w.info["xa"], True), (w.info["xb"], False)):
            col = int(np.argmin(np.abs(g.x - xc)))
            pk.append(p.edge_packet(w.v_table[col], w.sigma_x, xc, top, ea)[0])
        p.init_state(pk[0], pk[1], w.sym)
        p.step(20)
        o_gpu = p.observables(w.w_top)
        p.init_state(w.psi_a, w.psi_b, w.sym)
        p.step(20)
        o_in = p.observables(w.w_top)
        for k in ("norm", "p_tt", "p_tb", "p_bt", "p_bb", "p_b"):
            assert abs(o_gpu[k] - o_in[k]) <= 1e-10, k
    finally:
        p.close()


def test_bad_arguments_refused():
    from paper_1903_02581_amd.hom4d import Hom4dError
    w = preset("tiny")
    p = _prop(w)
    try:
        v = w.v_table[0]
        for args in ((v, 0.0, 0.0, True, 2.0), (v, -1.0, 0.0, True, 2.0), (v, float("nan"), 0.0, True, 2.0),
                     (np.full(w.ny, np.inf), 10.0, 0.0, True, 2.0)):
            with pytest.raises(Hom4dError):
                p.edge_packet(*args)
        with pytest.raises(ValueError):
            p.edge_packet(np.zeros(w.ny + 1), 10.0, 0.0, True, 2.0)
        # the handle still works afterwards
        psi, _ = p.edge_packet(v, 20.0, 0.0, True, 2.0)
        assert abs(np.sum(np.abs(psi) ** 2) - 1.0) <= 1e-13
    finally:
        p.close()
