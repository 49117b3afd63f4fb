"""Plant plausible mistakes in the oracle (CPU only) and check that a pin fails.

Each mutation replaces one oracle function with a subtly wrong version; the
pin tests of tests/test_oracle_pins.py are then run against the mutated oracle
and at least one of the named pins must fail.  This shows the pins are not
vacuous: a dropped term, a wrong sign, a transposed operand or a wrong half
step in the oracle would not go unnoticed.
"""
import numpy as np
import pytest

import oracle as O
import oracle.splitstep as SS
from tests import test_oracle_pins as pins


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


MUTATIONS = {
    "gauge sign (k_x + eBy/hbar)": ("theta_x", _wrong_gauge_sign, ["p2"]),
    "softening dropped from V12": ("coulomb", _dropped_coulomb_softening, ["p4"]),
    "V12 with x2 dropped from the distance": ("coulomb", _coulomb_missing_x2, ["p4"]),
    "shifted k_y grid": ("theta_y", _ky_shift_nyquist, ["p1", "p4"]),
    "kappa off by 1e-4 in T_y": ("theta_y", _wrong_kappa_theta_y, ["p1", "p2"]),
    "first-order (Lie) product": ("strang_step", _lie_step, ["p4", "p6"]),
    "X halves at full dt": ("strang_step", _x_full_twice, ["p4"]),
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
    raise KeyError(name)


@pytest.mark.parametrize("label", list(MUTATIONS))
def test_pins_catch_planted_mistake(label, monkeypatch):
    attr, fake, which = MUTATIONS[label]
    monkeypatch.setattr(SS, attr, fake)
    # the package re-exports; patch those names and the modules that imported them too
    monkeypatch.setattr(O, attr, fake, raising=False)
    caught = [p for p in which if _run_pin(p)]
    assert caught, f"no pin among {which} caught the mutation {label!r}"


def test_pins_pass_unmutated():
    assert not _run_pin("p2") and not _run_pin("p4")
