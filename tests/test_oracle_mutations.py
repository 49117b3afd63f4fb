"""Plant plausible mistakes in the oracle (CPU only) and check that a pin fails.

Each mutation replaces one oracle function with a subtly wrong version; the
pin tests of tests/test_oracle_pins.py are then run against the mutated oracle
and at least one of the named pins must fail.  This shows the pins are not
vacuous: a dropped term, a wrong sign, a transposed operand or a wrong half
step in the oracle would not go unnoticed.
"""
import numpy as np
import pytest

import importlib

import oracle as O
import oracle.splitstep as SS
from tests import test_oracle_pins as pins

# the package re-exports functions named like its modules: take the modules themselves
AD = importlib.import_module("oracle.adjoint")
OB = importlib.import_module("oracle.observables")


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _tiny_run_fixture():
    # the module-scoped fixture's body, evaluated against the current (mutated) oracle
    from workloads import preset
    w = preset("tiny")
    g = O.make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, soft_nm=w.soft_nm,
                    coulomb_c=w.coulomb_c, mstar_rel=w.mstar_rel, eps_r=w.eps_r)
    psi0 = O.init_state(w.psi_a, w.psi_b, -1)
    psi = O.propagate(psi0, g, w.v_table, w.dt_fs, 40)
    return w, g, psi0, psi


def _wrong_gauge_sign(g, tau, b_tesla=None):
    b = g.b_tesla if b_tesla is None else b_tesla
    shift = g.y[None, :] * (g.e_over_hbar * b)
    return (tau / g.hbar) * g.kappa * (g.kx[:, None] + shift) ** 2


def _dropped_coulomb_softening(g):
    x, y = g.x, g.y
    dx = x[:, None, None, None] - x[None, None, :, None]
    dy = y[None, :, None, None] - y[None, None, None, :]
    r = np.sqrt(dx ** 2 + dy ** 2)
    return g.coulomb_c * g.k_coul / np.maximum(r, g.soft_nm)


def _coulomb_missing_x2(g):
    x, y = g.x, g.y
    dx = x[:, None, None, None] + 0.0 * x[None, None, :, None]   # x1 instead of x1 - x2
    dy = y[None, :, None, None] - y[None, None, None, :]
    return g.coulomb_c * g.k_coul / np.sqrt(dx ** 2 + dy ** 2 + g.soft_nm ** 2)


def _ky_shift_nyquist(g, tau):
    k = g.ky.copy()
    k[g.ny // 2] = -k[g.ny // 2] if g.ny % 2 == 0 else k[g.ny // 2]
    k = k + 0.05 * (2 * np.pi / g.ly)
    return (tau / g.hbar) * g.kappa * k ** 2


def _lie_step(psi, g, v_table, dt):
    psi = SS.apply_x(psi, g, dt)
    psi = SS.apply_v(psi, g, v_table, dt)
    return SS.apply_y(psi, g, dt)


def _x_full_twice(psi, g, v_table, dt):
    psi = SS.apply_x(psi, g, dt)
    psi = SS.apply_v(psi, g, v_table, 0.5 * dt)
    psi = SS.apply_y(psi, g, dt)
    psi = SS.apply_v(psi, g, v_table, 0.5 * dt)
    return SS.apply_x(psi, g, dt)


def _wrong_kappa_theta_y(g, tau):
    return (tau / g.hbar) * (1.0001 * g.kappa) * g.ky ** 2


def _obs_tb_bt_swapped(psi, w_top):
    o = dict(_ORIG["observables"](psi, w_top))
    o["p_tb"], o["p_bt"] = o["p_bt"], o["p_tb"]
    return o


def _init_always_symmetric(psi_a, psi_b, sym):
    return _ORIG["init_state"](psi_a, psi_b, 1 if sym == -1 else sym)


def _entropy_in_bits(psi, ix1, jy1, ix2, jy2):
    return _ORIG["entanglement"](psi, ix1, jy1, ix2, jy2) / np.log(2.0)


def _attractive_coulomb(g):
    return -_ORIG["coulomb"](g)


def _v_full_dt_twice(psi, g, v_table, dt):
    psi = SS.apply_x(psi, g, 0.5 * dt)
    psi = SS.apply_v(psi, g, v_table, dt)
    psi = SS.apply_y(psi, g, dt)
    psi = SS.apply_v(psi, g, v_table, dt)
    return SS.apply_x(psi, g, 0.5 * dt)


def _dtheta_db_sign(g, tau):
    return -_ORIG["dtheta_x_db"](g, tau)


def _loss_bb_term_transposed(w_top, coeffs=(1.0, 0.0, 0.0, 1.0)):
    # the (B, B) term weighted by (1 - w1) w2 instead of (1 - w1)(1 - w2)
    w = np.asarray(w_top, dtype=np.float64)
    w1, w2 = w[:, :, None, None], w[None, None, :, :]
    a_tt, a_tb, a_bt, a_bb = coeffs
    return (a_tt * w1 * w2 + a_tb * w1 * (1 - w2) + a_bt * (1 - w1) * w2
            + a_bb * (1 - w1) * w2)


def _loss_tb_bt_swapped(w_top, coeffs=(1.0, 0.0, 0.0, 1.0)):
    a_tt, a_tb, a_bt, a_bb = coeffs
    return _ORIG["loss_weights"](w_top, (a_tt, a_bt, a_tb, a_bb))


# unmutated functions, for the mutations that wrap them
_ORIG = {"observables": OB.observables, "init_state": SS.init_state,
         "entanglement": OB.entanglement, "coulomb": SS.coulomb, "dtheta_x_db": SS.dtheta_x_db,
         "loss_weights": AD.loss_weights}


MUTATIONS = {
    "gauge sign (k_x + eBy/hbar)": ("theta_x", _wrong_gauge_sign, ["p2"]),
    "softening dropped from V12": ("coulomb", _dropped_coulomb_softening, ["p4"]),
    "V12 with x2 dropped from the distance": ("coulomb", _coulomb_missing_x2, ["p4"]),
    "shifted k_y grid": ("theta_y", _ky_shift_nyquist, ["p1", "p4"]),
    "kappa off by 1e-4 in T_y": ("theta_y", _wrong_kappa_theta_y, ["p1", "p2"]),
    "first-order (Lie) product": ("strang_step", _lie_step, ["p4", "p6"]),
    "X halves at full dt": ("strang_step", _x_full_twice, ["p4"]),
    "V halves at full dt": ("strang_step", _v_full_dt_twice, ["p4"]),
    "attractive V12": ("coulomb", _attractive_coulomb, ["p4"]),
    "P_TB and P_BT weights swapped": ("observables", _obs_tb_bt_swapped, ["obs"]),
    "symmetric state for sym = -1": ("init_state", _init_always_symmetric, ["p3"]),
    "entropy in bits": ("entanglement", _entropy_in_bits, ["p8"]),
    "d theta_X / dB with the wrong sign": ("dtheta_x_db", _dtheta_db_sign, ["p7"]),
    "loss weight of (B, B) taken as (1 - w1) w2": ("loss_weights", _loss_bb_term_transposed, ["loss"]),
    "loss coefficients of TB and BT swapped": ("loss_weights", _loss_tb_bt_swapped, ["loss"]),
}


def _run_pin(name):
    if name == "p1":
        return _fails(pins.test_p1_free_gaussian_closed_form)
    if name == "p2":
        return _fails(pins.test_p2_landau_level_eigenphase)
    if name == "p4":
        return _fails(pins.test_p4_dense_expm_bruteforce, 0.0)
    if name == "p6":
        return _fails(pins.test_p6_time_reversal, _tiny_run_fixture())
    if name == "p3":
        return _fails(pins.test_p3_invariants_tiny, _tiny_run_fixture())
    if name == "p7":
        return _fails(pins.test_p7_adjoint_vs_finite_differences)
    if name == "p8":
        return _fails(pins.test_p8_entanglement_special_cases)
    if name == "obs":
        return _fails(pins.test_orbital_observables_brute_force, 0)
    if name == "loss":
        return _fails(pins.test_loss_weights_are_region_probabilities)
    raise KeyError(name)


@pytest.mark.parametrize("label", list(MUTATIONS))
def test_pins_catch_planted_mistake(label, monkeypatch):
    attr, fake, which = MUTATIONS[label]
    # the defining module, the package's re-export and the modules that imported the name
    for mod in (SS, OB, AD, O):
        if hasattr(mod, attr):
            monkeypatch.setattr(mod, attr, fake)
    caught = [p for p in which if _run_pin(p)]
    assert caught, f"no pin among {which} caught the mutation {label!r}"


def test_pins_pass_unmutated():
    for name in ("p2", "p4", "p3", "p8", "obs", "loss"):
        assert not _run_pin(name), name
