"""The resolving beam-splitter workload (Fermi-block constriction, Sec. II.C
Eq. (pot_xy)): grid conditions, symmetry, and the single-electron splitting
ratio and two-electron bunching computed by the FP64 oracle in 2D (the
two-body term off, so the 4D propagation factorises exactly)."""
import numpy as np
import pytest

import oracle as O
from workloads import preset
from workloads.presets import QPC_GAP_NM, _E_OVER_HBAR


@pytest.fixture(scope="module")
def qpc_orbitals():
    w = preset("qpc")
    g = O.make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, soft_nm=w.soft_nm, coulomb_c=0.0)
    a = O.propagate_2d(w.psi_a, g, w.v_table, w.dt_fs, w.steps)
    b = O.propagate_2d(w.psi_b, g, w.v_table, w.dt_fs, w.steps)
    return w, a, b


def test_grid_resolves_the_landau_problem():
    w = preset("qpc")
    lb2 = 1.0 / (_E_OVER_HBAR * w.b_tesla)          # l_B^2 in nm^2
    flux = w.lx * w.ly / (2.0 * np.pi * lb2)
    assert w.nx >= flux                              # every guiding centre is a grid wave number
    assert w.ly / w.ny < 0.5 * np.sqrt(lb2)           # dy < l_B / 2
    assert w.coulomb_c == 0.0 and w.sym == -1
    assert w.info["qpc_gap_nm"] == QPC_GAP_NM


def test_constriction_is_point_symmetric():
    # V(-x, -y) = V(x, y): the two injectors see the same splitter
    w = preset("qpc")
    v = w.v_table
    i = (-np.arange(w.nx)) % w.nx
    j = (-np.arange(w.ny)) % w.ny
    vr = v[i][:, j]
    inner = np.ix_(np.arange(1, w.nx), np.arange(1, w.ny))   # the grid point -L/2 has no mirror
    assert np.max(np.abs(vr[inner] - v[inner])) < 1e-9 * np.max(v)


def test_half_transmission_and_bunching(qpc_orbitals):
    w, a, b = qpc_orbitals
    t_a = float(np.sum(np.abs(a) ** 2 * w.w_top))     # alpha starts on the top edge
    r_b = float(np.sum(np.abs(b) ** 2 * w.w_top))     # beta starts on the bottom edge
    assert 0.45 < t_a < 0.55
    assert abs(t_a + r_b - 1.0) < 0.02                # same splitting ratio for both injectors
    prod = O.orbital_observables(a, b, w.w_top, 0)
    anti = O.orbital_observables(a, b, w.w_top, -1)
    # distinguishable electrons at a balanced splitter: P_b = 2 T (1 - T) ~ 1/2
    assert abs(prod["p_b"] - 0.5) < 0.01
    # exchange lowers the bunching probability of the Slater determinant
    assert anti["p_b"] < prod["p_b"] - 0.1
    assert abs(anti["p_tb"] - anti["p_bt"]) < 1e-12
