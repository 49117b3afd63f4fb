"""Pins of the edge-state generator oracle (CPU only): Sec. II.A Eq. (H_effective) and
Sec. II.B Eq. (singlepwp), as restated in oracle/edge_states.py."""
import numpy as np
import pytest

import oracle.edge_states as ES
from oracle import make_grid


def _lll_grid():
    # dy = 4 nm < l_B / 2 at 5 T (l_B = 11.47 nm); guiding centres within +-96 nm of the
    # middle of a 384 nm box stay 8 l_B from the periodic boundary
    return make_grid(16, 96, 400.0, 384.0, b_tesla=5.0)


def test_lowest_landau_level_closed_form():
    """v = 0: E(k) = hbar omega_c / 2 and phi_k = Gaussian of width l_B at y0 = k l_B^2."""
    g = _lll_grid()
    e1, phi = ES.lowest_edge_states(g, np.zeros(g.ny))
    lb2 = 1.0 / (g.e_over_hbar * g.b_tesla)
    hw_c = 2.0 * g.kappa / lb2          # hbar omega_c = hbar e B / m* = 2 kappa / l_B^2
    checked = 0
    for m, k in enumerate(g.kx):
        y0 = k * lb2
        if abs(y0) > 96.0:
            continue
        gauss = np.exp(-(g.y - y0) ** 2 / (2.0 * lb2))
        gauss /= np.linalg.norm(gauss)
        assert abs(e1[m] - 0.5 * hw_c) <= 1e-11 * hw_c, (m, e1[m], 0.5 * hw_c)
        assert np.max(np.abs(phi[m] - gauss)) <= 1e-12, m
        checked += 1
    assert checked >= 12


def test_edge_states_orthonormal_and_signed():
    g = make_grid(8, 64, 400.0, 256.0, b_tesla=5.0)
    y = g.y
    v = 10000.0 * (1.0 / (1.0 + np.exp(-(y - 0.4 * g.ly) / 3.0)) + 1.0 / (1.0 + np.exp((y + 0.4 * g.ly) / 3.0)))
    e1, phi = ES.lowest_edge_states(g, v)
    for m in range(g.nx):
        assert abs(np.dot(phi[m], phi[m]) - 1.0) <= 1e-13
        assert phi[m][np.argmax(np.abs(phi[m]))] > 0
        h = ES.edge_hamiltonian(g, g.kx[m], v)
        assert np.linalg.norm(h @ phi[m] - e1[m] * phi[m]) <= 1e-9 * np.linalg.norm(h)


def _walls(g):
    y = g.y
    return 10000.0 * (1.0 / (1.0 + np.exp(-(y - 0.4 * g.ly) / 3.0)) + 1.0 / (1.0 + np.exp((y + 0.4 * g.ly) / 3.0)))


@pytest.mark.parametrize("top", [True, False])
def test_packet_weights_recovered_by_projection(top):
    """Projecting the packet on exp(i k (x - xc)) phi_k(y) returns exp(-sigma^2 (k - k0)^2)."""
    g = make_grid(64, 32, 800.0, 128.0, b_tesla=5.0)
    v = _walls(g)
    sigma, xc = 30.0, -150.0
    psi, info = ES.edge_packet(g, v, sigma, xc, top, 2.0)
    assert abs(np.sum(np.abs(psi) ** 2) - 1.0) <= 1e-13
    _, phi = ES.lowest_edge_states(g, v)
    c = np.array([np.sum(np.exp(-1j * k * (g.x - xc))[:, None] * phi[m][None, :] * psi)
                  for m, k in enumerate(g.kx)])
    want = np.exp(-sigma ** 2 * (g.kx - info["k0"]) ** 2)
    scale = c[np.argmax(want)] / want.max()
    assert np.max(np.abs(c - scale * want)) <= 1e-12 * abs(scale)
    assert abs(scale.imag) <= 1e-12 * abs(scale)


@pytest.mark.parametrize("top", [True, False])
def test_packet_k0_is_closest_level_on_its_side(top):
    g = make_grid(64, 32, 800.0, 128.0, b_tesla=5.0)
    v = _walls(g)
    e_above = 2.0
    _, info = ES.edge_packet(g, v, 30.0, 0.0, top, e_above)
    e1, _ = ES.lowest_edge_states(g, v)
    target = g.kappa * g.e_over_hbar * g.b_tesla + e_above
    best = None
    for m, k in enumerate(g.kx):       # brute force over the requested half of the k grid
        if (k > 0) != top or k == 0.0:
            continue
        if best is None or abs(e1[m] - target) < abs(e1[best] - target):
            best = m
    assert info["k0"] == g.kx[best]
    assert info["e1_k0"] == e1[best]
    assert abs(info["target"] - target) <= 1e-12 * target


def test_packets_match_the_input_generator():
    """The workload generator builds its kinetic matrix from FFTs; the oracle from DFT matrices."""
    from workloads import preset
    w = preset("qpc")
    g = make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, mstar_rel=w.mstar_rel)
    for psi_ref, xc, top in ((w.psi_a, w.info["xa"], True), (w.psi_b, w.info["xb"], False)):
        col = int(np.argmin(np.abs(g.x - xc)))
        psi, _ = ES.edge_packet(g, w.v_table[col], w.sigma_x, xc, top, 5.0)
        assert np.max(np.abs(psi - psi_ref)) <= 1e-12


# planted mistakes: each must fail one of the pins above
def _coupling_sign_flipped(g, k, v_col):
    d = g.kappa * (k + g.y * (g.e_over_hbar * g.b_tesla)) ** 2 + np.asarray(v_col, dtype=np.float64)
    return ES.kinetic_y(g) + np.diag(d)


def _kinetic_half(g):
    return 0.5 * _ORIG_KIN(g)


_ORIG_PACKET = ES.edge_packet
_ORIG_KIN = ES.kinetic_y


def _packet_phase_conjugated(g, v_col, sigma_x, xc, top, e_above_lll):
    psi, info = _ORIG_PACKET(g, v_col, sigma_x, xc, top, e_above_lll)
    return np.conj(psi), info


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("attr,fake,pin", [
    ("edge_hamiltonian", _coupling_sign_flipped,
     lambda: _fails(test_lowest_landau_level_closed_form)),
    ("kinetic_y", _kinetic_half, lambda: _fails(test_lowest_landau_level_closed_form)),
    ("edge_packet", _packet_phase_conjugated,
     lambda: _fails(test_packet_weights_recovered_by_projection, True)),
])
def test_pins_catch_planted_mistake(attr, fake, pin, monkeypatch):
    monkeypatch.setattr(ES, attr, fake)
    assert pin()
