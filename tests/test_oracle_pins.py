"""Pins of the FP64 oracle against what the physics and the mathematics fix.

Nothing here compares the oracle with itself: each test uses a route the
oracle does not take (an analytic Gaussian integral, a Strang eigen-solution of
the harmonic oscillator, dense matrix exponentials, a 2D propagation, finite
differences, published constants).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from oracle.adjoint import loss_weights
from workloads import preset
from workloads.presets import saddle_potential

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------------------- constants (golden)

def test_constants_against_codata():
    gold = json.load(open(os.path.join(GOLDEN, "constants.json")))
    g = O.make_grid(8, 8, 100.0, 100.0)
    got = {
        "hbar_eV_s": g.hbar * 1e-3 * 1e-15,
        "e2_over_4pi_eps0_eV_nm": g.k_coul * g.eps_r * 1e-3,
        "hbar2_over_2me_eV_nm2": g.kappa * g.mstar_rel * 1e-3,
        "hbar_over_e_T_nm2": 1.0 / g.e_over_hbar,
        "hw_c_per_tesla_gaas_meV": 2.0 * g.kappa * g.e_over_hbar,
    }
    for key, val in got.items():
        ref = gold[key]
        assert abs(val - ref["value"]) <= ref["rtol"] * abs(ref["value"]), (key, val, ref)


# --------------------------------------------------------- P1: free Gaussian, B = V = V12 = 0

def _gauss_t(x, x0, sig, k0, beta):
    """Closed-form free evolution of (2 pi sig^2)^(-1/4) exp(-(x-x0)^2/4sig^2 + i k0 (x-x0)),
    with beta = hbar t / 2m (Gaussian Fourier integral done by hand)."""
    s2 = sig ** 2 + 1j * beta
    amp = (2 * np.pi * sig ** 2) ** -0.25 * sig / np.sqrt(s2)
    return amp * np.exp((2 * sig ** 2 * k0 + 1j * (x - x0)) ** 2 / (4 * s2) - sig ** 2 * k0 ** 2)


def test_p1_free_gaussian_closed_form():
    sig = 15.0
    nx, ny = 48, 40
    lx, ly = 26 * sig, 24 * sig
    g = O.make_grid(nx, ny, lx, ly, b_tesla=0.0, coulomb_c=0.0)
    beta_per_fs = g.kappa / g.hbar          # hbar / 2m in nm^2/fs
    k0a, k0b = 0.5 / sig, -0.4 / sig
    xa, xb = -1.0 * sig, 1.0 * sig
    ya, yb = 0.5 * sig, -0.5 * sig

    def packet(t, x0, y0, k0):
        b = beta_per_fs * t
        return (_gauss_t(g.x, x0, sig, k0, b)[:, None] * _gauss_t(g.y, y0, sig, 0.0, b)[None, :]
                * np.sqrt((lx / nx) * (ly / ny)))

    v = np.zeros((nx, ny))
    dt, n = 25.0, 4
    for sym in (-1, 0):
        psi0 = O.init_state(packet(0.0, xa, ya, k0a), packet(0.0, xb, yb, k0b), sym)
        psi = O.propagate(psi0, g, v, dt, n)
        ref = O.init_state(packet(n * dt, xa, ya, k0a), packet(n * dt, xb, yb, k0b), sym)
        # init_state normalises the reference at time t: the norm is conserved exactly
        assert rel_l2(psi, ref) < 1e-10


# ----------------------------------------------- P2: Strang lowest-Landau-level eigenphase

def test_p2_landau_level_eigenphase():
    """With V = V12 = 0 and fixed k_x, X(dt/2) Y(dt) X(dt/2) is the symmetric splitting of a
    harmonic oscillator in y of frequency w_c = eB/m* centred at y0 = k_x l_B^2.  Its classical
    map has trace 2 - (w_c dt)^2, rotation angle th = 2 arcsin(w_c dt/2) and the invariant
    Gaussian of frequency W' = w_c sqrt(1 - (w_c dt/2)^2); that Gaussian is mapped to itself
    with phase exp(-i th/2).  A Slater determinant of two such one-electron states at two
    different k_x therefore gains exp(-i th) per step.  Fixes the sign and size of B, the
    gauge, kappa and the Strang order."""
    g = O.make_grid(4, 48, 400.0, 200.0, b_tesla=5.0, coulomb_c=0.0)
    eoh = g.e_over_hbar * g.b_tesla
    wc = 2.0 * g.kappa * eoh / g.hbar
    dt = 0.3 / wc
    a = wc * dt
    om = wc * np.sqrt(1.0 - a * a / 4.0)
    w2 = 2.0 * g.kappa / (g.hbar * om)            # hbar / (m* W')

    def orb(m):
        y0 = g.kx[m] / eoh
        p = np.exp(1j * g.kx[m] * g.x)[:, None] * np.exp(-(g.y - y0) ** 2 / (2 * w2))[None, :]
        return p / np.linalg.norm(p)

    psi0 = O.init_state(orb(0), orb(1), -1)
    n = 20
    psi = O.propagate(psi0, g, np.zeros((4, 48)), dt, n)
    ov = np.vdot(psi0, psi)
    th = 2.0 * np.arcsin(a / 2.0)
    assert abs(abs(ov) - 1.0) < 1e-12
    dphi = np.angle(ov * np.exp(1j * n * th))
    assert abs(dphi) < 1e-12 * n
    # the wrong field sign puts the minimum at -y0 and destroys the eigenstate
    gneg = O.make_grid(4, 48, 400.0, 200.0, b_tesla=-5.0, coulomb_c=0.0)
    bad = O.propagate(psi0, gneg, np.zeros((4, 48)), dt, n)
    assert abs(abs(np.vdot(psi0, bad)) - 1.0) > 1e-3


# ------------------------------------------------------------------------ P3: invariants

@pytest.fixture(scope="module")
def tiny_run():
    w = preset("tiny")
    g = O.make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, soft_nm=w.soft_nm,
                    coulomb_c=w.coulomb_c, mstar_rel=w.mstar_rel, eps_r=w.eps_r)
    psi0 = O.init_state(w.psi_a, w.psi_b, -1)
    psi = O.propagate(psi0, g, w.v_table, w.dt_fs, w.steps)
    return w, g, psi0, psi


def test_p3_invariants_tiny(tiny_run):
    w, g, psi0, psi = tiny_run
    obs = O.observables(psi, w.w_top)
    assert abs(obs["norm"] - 1.0) < 1e-12
    swapped = np.transpose(psi, (2, 3, 0, 1))
    assert np.linalg.norm(psi + swapped) / np.linalg.norm(psi) < 1e-12
    diag = psi.reshape(w.nx * w.ny, w.nx * w.ny).diagonal()
    assert np.max(np.abs(diag)) < 1e-12 * np.max(np.abs(psi))
    assert abs(obs["p_tb"] - obs["p_bt"]) < 1e-12
    tot = obs["p_tt"] + obs["p_tb"] + obs["p_bt"] + obs["p_bb"]
    assert abs(tot - obs["norm"]) < 1e-12
    # the state did move: the test is not vacuous
    assert rel_l2(psi, psi0) > 1e-2


# ------------------------------------------------------------ P4: dense brute force, 6x6

def _dense_ops(g, v_table):
    n_x, n_y = g.nx, g.ny

    def dft(n):
        j = np.arange(n)
        return np.exp(-2j * np.pi * np.outer(j, j) / n)

    def kvec(n, length):
        m = np.arange(n)
        return 2 * np.pi / length * np.where(m < n / 2, m, m - n)

    fx, fy = dft(n_x), dft(n_y)
    kx, ky = kvec(n_x, g.lx), kvec(n_y, g.ly)
    x = -g.lx / 2 + np.arange(n_x) * g.lx / n_x
    y = -g.ly / 2 + np.arange(n_y) * g.ly / n_y
    eoh = g.e_over_hbar * g.b_tesla
    ey, ex = np.eye(n_y), np.eye(n_x)
    ty = np.conj(fy).T @ np.diag(g.kappa * ky ** 2) @ fy / n_y
    d = n_x * n_y
    hx1 = np.zeros((n_x, n_y, n_x, n_y, n_x, n_y, n_x, n_y), complex)
    for jy in range(n_y):
        tx = np.conj(fx).T @ np.diag(g.kappa * (kx - y[jy] * eoh) ** 2) @ fx / n_x
        # acts on x1 at fixed y1 = jy, identity on (x2, y2)
        hx1[:, jy, :, :, :, jy, :, :] += np.einsum("ab,cd,ef->acebdf", tx, ex, ey)
    hx1 = hx1.reshape(d * d, d * d)
    swap = np.eye(d * d).reshape(n_x, n_y, n_x, n_y, n_x, n_y, n_x, n_y)
    swap = swap.transpose(2, 3, 0, 1, 4, 5, 6, 7).reshape(d * d, d * d)
    hx2 = swap @ hx1 @ swap
    hy1 = np.kron(np.kron(np.kron(ex, ty), ex), ey)
    hy2 = np.kron(np.kron(np.kron(ex, ey), ex), ty)
    vd = np.zeros((n_x, n_y, n_x, n_y))
    for i1 in range(n_x):
        for j1 in range(n_y):
            for i2 in range(n_x):
                for j2 in range(n_y):
                    r = np.hypot(x[i1] - x[i2], y[j1] - y[j2])
                    vc = g.coulomb_c * g.k_coul / np.sqrt(r * r + g.soft_nm ** 2)
                    if g.screen_nm > 0:
                        vc *= np.exp(-r / g.screen_nm)
                    vd[i1, j1, i2, j2] = v_table[i1, j1] + v_table[i2, j2] + vc
    hv = np.diag(vd.ravel()).astype(complex)
    return hx1 + hx2, hy1 + hy2, hv


@pytest.mark.parametrize("screen", [0.0, 5.0])
def test_p4_dense_expm_bruteforce(screen):
    rng = np.random.default_rng(3)
    g = O.make_grid(6, 6, 60.0, 48.0, b_tesla=5.0, soft_nm=2.0, coulomb_c=1.0,
                    screen_nm=screen)
    v = rng.uniform(-5, 5, (6, 6))
    hx, hy, hv = _dense_ops(g, v)
    for h in (hx, hy, hv):
        assert np.allclose(h, h.conj().T, atol=1e-9)
    psi0 = rng.standard_normal((6, 6, 6, 6)) + 1j * rng.standard_normal((6, 6, 6, 6))
    psi0 /= np.linalg.norm(psi0)
    dt = 4.0
    u = lambda h, tau: sla.expm(-1j * tau / g.hbar * h)   # noqa: E731
    s = u(hx, dt / 2) @ u(hv, dt / 2) @ u(hy, dt) @ u(hv, dt / 2) @ u(hx, dt / 2)
    ref = (s @ psi0.ravel()).reshape(psi0.shape)
    got = O.strang_step(psi0, g, v, dt)
    assert rel_l2(got, ref) < 1e-12
    # second order towards the exact propagator exp(-i H T / hbar)
    t_end = 16.0
    exact = (u(hx + hy + hv, t_end) @ psi0.ravel()).reshape(psi0.shape)
    errs = []
    for n in (8, 16, 32):
        errs.append(rel_l2(O.propagate(psi0, g, v, t_end / n, n), exact))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2.0) < 0.15), (errs, slopes)


# ---------------------------------------------------- P5: factorisation when V12 = 0

def test_p5_factorisation_without_coulomb():
    w = preset("tiny")
    g = O.make_grid(w.nx, w.ny, w.lx, w.ly, b_tesla=w.b_tesla, coulomb_c=0.0)
    n = 40
    psi = O.propagate(O.init_state(w.psi_a, w.psi_b, -1), g, w.v_table, w.dt_fs, n)
    a = O.propagate_2d(w.psi_a, g, w.v_table, w.dt_fs, n)
    b = O.propagate_2d(w.psi_b, g, w.v_table, w.dt_fs, n)
    ab = np.vdot(w.psi_a, w.psi_b)           # conserved by the unitary one-body step
    scale = np.sqrt(2.0 * (1.0 - abs(ab) ** 2))
    ref = (a[:, :, None, None] * b[None, None] - b[:, :, None, None] * a[None, None]) / scale
    assert rel_l2(psi, ref) < 1e-12
    # exact generalisation of the paper's Eq. (bunchingket) to overlapping packets
    wt = w.w_top
    t_a = np.vdot(a, wt * a).real
    t_b = np.vdot(b, wt * b).real
    t_ab = np.vdot(a, wt * b)
    ovl = np.vdot(a, b)
    p_tt = (t_a * t_b - abs(t_ab) ** 2) / (1 - abs(ovl) ** 2)
    wb = 1.0 - wt
    b_a, b_b, b_ab = np.vdot(a, wb * a).real, np.vdot(b, wb * b).real, np.vdot(a, wb * b)
    p_bb = (b_a * b_b - abs(b_ab) ** 2) / (1 - abs(ovl) ** 2)
    obs = O.observables(psi, wt)
    assert abs(obs["p_tt"] - p_tt) < 1e-12 and abs(obs["p_bb"] - p_bb) < 1e-12


# ---------------------------------------------------------------- P6: time reversal

def test_p6_time_reversal(tiny_run):
    w, g, psi0, psi = tiny_run
    back = O.propagate(psi, g, w.v_table, -w.dt_fs, w.steps)
    assert rel_l2(back, psi0) < 1e-12


# ------------------------------------------------------------------- P7: gradients

def _small_grad_case():
    nx, ny, lx, ly = 8, 8, 200.0, 200.0
    from workloads.presets import build
    w = build("g", nx, ny, lx, ly, b_tesla=5.0, dt_fs=5.0, steps=6, sigma_x=20.0, seed=1)
    g = O.make_grid(nx, ny, lx, ly, b_tesla=w.b_tesla, soft_nm=w.soft_nm, coulomb_c=1.0)
    return w, g


def test_p7_adjoint_vs_finite_differences():
    w, g = _small_grad_case()
    psi0 = O.init_state(w.psi_a, w.psi_b, -1)
    x, y = g.x, g.y
    theta = np.array([w.v0, w.v1, w.sx, w.sy, w.b_tesla])

    def vtab(t):
        return saddle_potential(x, y, t[0], t[1], t[2], t[3], w.ly)

    def loss_of(t):
        gg = O.make_grid(g.nx, g.ny, g.lx, g.ly, b_tesla=t[4], soft_nm=g.soft_nm,
                         coulomb_c=g.coulomb_c)
        p = O.propagate(psi0, gg, vtab(t), w.dt_fs, w.steps)
        return float(np.sum(loss_weights(w.w_top) * np.abs(p) ** 2))

    loss, g_v, g_b = O.loss_and_grad_stored(psi0, g, vtab(theta), w.dt_fs, w.steps, w.w_top)
    assert abs(loss - loss_of(theta)) < 1e-14
    # gauge invariance: a uniform shift of V is a global phase
    assert abs(g_v.sum()) < 1e-12 * np.abs(g_v).sum()
    # chain through V(theta) with exact partial derivatives of the saddle
    X, Y = x[:, None], y[None, :]
    dv = [np.exp(-X ** 2 / theta[2] ** 2) + 0 * Y,
          -np.exp(-Y ** 2 / theta[3] ** 2) + 0 * X,
          theta[0] * np.exp(-X ** 2 / theta[2] ** 2) * 2 * X ** 2 / theta[2] ** 3 + 0 * Y,
          -theta[1] * np.exp(-Y ** 2 / theta[3] ** 2) * 2 * Y ** 2 / theta[3] ** 3 + 0 * X]
    adj = np.array([np.sum(g_v * d) for d in dv] + [g_b])
    fd = O.grad_fd(loss_of, theta, h_rel=1e-4)
    for a_, f_ in zip(adj, fd):
        assert abs(a_ - f_) <= 1e-6 * max(abs(f_), 1e-6), (adj, fd)
    # single table entries, directly
    v0 = vtab(theta)
    big = np.argsort(np.abs(g_v).ravel())[-3:]
    for (i, j) in zip(*np.unravel_index(big, g_v.shape)):
        h = 1e-3

        def lv(s):
            vv = v0.copy()
            vv[i, j] += s
            return float(np.sum(loss_weights(w.w_top)
                                * np.abs(O.propagate(psi0, g, vv, w.dt_fs, w.steps)) ** 2))
        fd_ij = (lv(h) - lv(-h)) / (2 * h)
        assert abs(fd_ij - g_v[i, j]) <= 1e-6 * max(abs(fd_ij), 1e-8)


def _region_probabilities_by_loops(psi, top):
    """P_TT, P_TB, P_BT, P_BB of Eq. (p_bunching), Sec. III, for a hard partition of the
    one-electron plane: top[i, j] is True where (x_i, y_j) lies in T.  Each grid point of
    configuration space is visited once and its |Psi|^2 goes to the one region pair its
    two electrons occupy (pure-Python loops, no weight algebra)."""
    nx, ny = top.shape
    acc = {"TT": 0.0, "TB": 0.0, "BT": 0.0, "BB": 0.0}
    for i1 in range(nx):
        for j1 in range(ny):
            for i2 in range(nx):
                for j2 in range(ny):
                    key = ("T" if top[i1, j1] else "B") + ("T" if top[i2, j2] else "B")
                    z = psi[i1, j1, i2, j2]
                    acc[key] += z.real * z.real + z.imag * z.imag
    return acc


def test_loss_weights_are_region_probabilities():
    """The loss of the adjoint is the bunching probability of Eq. (p_bunching), Sec. III:
    with coefficients (1, 0, 0, 1) it is the probability that both electrons sit in the
    same region, and with a unit coefficient vector it is that region pair's probability.
    Checked for a hard T/B partition against sums by explicit loops over configuration
    space, on the initial state (zero steps) and after two Strang steps, where it must also
    equal the bunching probability of observables() of the propagated state."""
    from workloads.presets import build
    nx, ny = 4, 6
    w = build("g", nx, ny, 100.0, 150.0, b_tesla=5.0, dt_fs=5.0, steps=2, sigma_x=20.0, seed=4,
              sym=0)
    g = O.make_grid(nx, ny, w.lx, w.ly, b_tesla=w.b_tesla, soft_nm=w.soft_nm, coulomb_c=1.0)
    rng = np.random.default_rng(17)
    top = rng.uniform(size=(nx, ny)) < 0.5        # an irregular partition, both regions used
    top[0, 0], top[0, 1] = True, False
    w_top = top.astype(np.float64)
    psi0 = O.init_state(w.psi_a, w.psi_b, 0)      # product state: P_TB != P_BT
    units = {"TT": (1, 0, 0, 0), "TB": (0, 1, 0, 0), "BT": (0, 0, 1, 0), "BB": (0, 0, 0, 1)}
    for steps in (0, 2):
        psi = O.propagate(psi0, g, w.v_table, w.dt_fs, steps) if steps else psi0
        ref = _region_probabilities_by_loops(psi, top)
        assert abs(ref["TB"] - ref["BT"]) > 1e-6  # the pairs are distinguishable here
        for key, cf in units.items():
            loss, _, _ = O.loss_and_grad_stored(psi0, g, w.v_table, w.dt_fs, steps, w_top,
                                                coeffs=cf)
            assert abs(loss - ref[key]) < 1e-14, (steps, key, loss, ref[key])
        loss, _, _ = O.loss_and_grad_stored(psi0, g, w.v_table, w.dt_fs, steps, w_top)
        assert abs(loss - (ref["TT"] + ref["BB"])) < 1e-14
        assert abs(loss - O.observables(psi, w_top)["p_b"]) < 1e-14
    # soft weights (w in [0, 1]): the four region-pair losses partition the norm, and the
    # loss is linear in the coefficients
    w_soft = rng.uniform(size=(nx, ny))
    parts = [O.loss_and_grad_stored(psi0, g, w.v_table, w.dt_fs, 0, w_soft, coeffs=cf)[0]
             for cf in units.values()]
    norm = float(np.sum(np.abs(psi0) ** 2))
    assert abs(sum(parts) - norm) < 1e-14
    cf = (0.3, -1.2, 2.5, 0.7)
    mix = O.loss_and_grad_stored(psi0, g, w.v_table, w.dt_fs, 0, w_soft, coeffs=cf)[0]
    assert abs(mix - sum(c * q for c, q in zip(cf, parts))) < 1e-13


# --------------------------------------------------------------- P8: entanglement

def test_p8_entanglement_special_cases():
    rng = np.random.default_rng(0)
    nx, ny = 8, 4
    a = rng.standard_normal((nx, ny)) + 1j * rng.standard_normal((nx, ny))
    b = rng.standard_normal((nx, ny)) + 1j * rng.standard_normal((nx, ny))
    prod = a[:, :, None, None] * b[None, None]
    ix = np.arange(nx)
    assert abs(O.entanglement(prod, ix, 1, ix, 2)) < 1e-12
    # two-term Schmidt state with orthonormal factors on the slice rows
    q1, _ = np.linalg.qr(rng.standard_normal((nx, 2)) + 1j * rng.standard_normal((nx, 2)))
    q2, _ = np.linalg.qr(rng.standard_normal((nx, 2)) + 1j * rng.standard_normal((nx, 2)))
    psi = np.zeros((nx, ny, nx, ny), complex)
    psi[:, 1, :, 2] = (np.outer(q1[:, 0], q2[:, 0]) - np.outer(q1[:, 1], q2[:, 1])) / np.sqrt(2)
    assert abs(O.entanglement(psi, ix, 1, ix, 2) - np.log(2.0)) < 1e-12
    # SVD route against the eigenvalues of the reduced density matrix
    psi = rng.standard_normal((nx, ny, nx, ny)) + 1j * rng.standard_normal((nx, ny, nx, ny))
    phi = psi[:, 3, :, 0]
    phi = phi / np.linalg.norm(phi)
    lam = np.linalg.eigvalsh(phi @ phi.conj().T)
    lam = lam[lam > 1e-300]
    assert abs(O.entanglement(psi, ix, 3, ix, 0) + np.sum(lam * np.log(lam))) < 1e-12


# ----------------------------------------------------- marginal / conditional densities

def test_marginal_and_conditional_closed_forms():
    rng = np.random.default_rng(5)
    nx, ny = 6, 5
    a = rng.standard_normal((nx, ny)) + 1j * rng.standard_normal((nx, ny))
    b = rng.standard_normal((nx, ny)) + 1j * rng.standard_normal((nx, ny))
    a /= np.linalg.norm(a)
    b /= np.linalg.norm(b)
    prod = O.init_state(a, b, 0)
    assert np.allclose(O.marginal(prod), np.abs(a) ** 2, atol=1e-15)
    slater = O.init_state(a, b, -1)
    ab = np.vdot(a, b)                      # <a|b>
    ref = (np.abs(a) ** 2 + np.abs(b) ** 2 - 2 * np.real(np.conj(a) * b * np.conj(ab))) \
        / (2 * (1 - abs(ab) ** 2))
    assert np.allclose(O.marginal(slater), ref, atol=1e-14)
    assert abs(O.marginal(slater).sum() - 1.0) < 1e-14
    c = O.conditional(slater, 2, 3)
    assert c[2, 3] < 1e-30                  # Pauli node at r1 = r2*
    assert np.allclose(O.conditional(prod, 2, 3), np.abs(a) ** 2 * abs(b[2, 3]) ** 2, atol=1e-15)


# ---------------------------------------- region probabilities from two orbitals

@pytest.mark.parametrize("sym", [-1, 0, 1])
def test_orbital_observables_brute_force(sym):
    # the one-electron matrix-element form against the explicit 4D sum over
    # configuration space of the normalised state built by init_state
    rng = np.random.default_rng(11 + sym)
    nx, ny = 5, 4
    a = rng.standard_normal((nx, ny)) + 1j * rng.standard_normal((nx, ny))
    b = rng.standard_normal((nx, ny)) + 1j * rng.standard_normal((nx, ny))
    a /= np.linalg.norm(a)
    b /= np.linalg.norm(b)
    w = rng.uniform(0.0, 1.0, (nx, ny))
    psi = O.init_state(a, b, sym)
    d = np.abs(psi) ** 2
    w1, w2 = w[:, :, None, None], w[None, None, :, :]
    brute = dict(p_tt=np.sum(d * w1 * w2), p_tb=np.sum(d * w1 * (1 - w2)),
                 p_bt=np.sum(d * (1 - w1) * w2), p_bb=np.sum(d * (1 - w1) * (1 - w2)))
    got = O.orbital_observables(a, b, w, sym)
    for k, v in brute.items():
        assert abs(got[k] - v) < 1e-14, (k, got[k], v)
    assert abs(got["p_b"] - brute["p_tt"] - brute["p_bb"]) < 1e-14
    # and the 4D region sums of observables() itself (the product state, sym = 0, has
    # P_TB != P_BT, so a transposed weight cannot hide)
    full = O.observables(psi, w)
    for k, v in brute.items():
        assert abs(full[k] - v) < 1e-14, (k, full[k], v)
    assert abs(full["p_ab"] - brute["p_tb"] - brute["p_bt"]) < 1e-14
