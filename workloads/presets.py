"""Named, seeded workloads for the 4D two-electron split-step propagator.

Every number below is an *input* to the propagation: box and grid per
electron, GaAs material constants, field, time step, step count, the external
potential table, the two single-particle edge packets and the region weights.

Physics sources (arXiv 1903.02581):
  * edge states: Sec. II.A, Eq. (H_effective) -- the lowest transverse
    eigenstate of the Landau-gauge effective Hamiltonian for each wave vector;
  * wave packet: Sec. II.B, Eq. (singlepwp) -- a Gaussian superposition of
    edge states with spatial dispersion sigma along the propagation direction;
  * confining barrier: Sec. II.B, Eq. (pot_x) -- Fermi-function walls with
    height V_b = 10 eV and smoothness 3 nm (read as exp(x/tau));
  * material and field: Sec. III (GaAs m* = 0.067 m_e, B = 5 T).

Geometry used here (the paper leaves its QPC coordinates unstated): the gauge
is A = (-B y, 0), electrons propagate along x on the top (y > 0) and bottom
(y < 0) edges, x is periodic, Fermi walls sit at y = +-0.4 Ly and the beam
splitter is the saddle V0 exp(-x^2/sx^2) - V1 exp(-y^2/sy^2).  The top
packet starts at x = -Lx/4 moving +x, the bottom one at +Lx/4 moving -x; both
centres are jittered by a seeded uniform draw in [-dx/2, dx/2).

Units: nm, fs, meV, tesla.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# CODATA 2018 SI values, restated here so the generator depends on no other
# module of this repository.
_HBAR_SI = 1.054571817e-34      # J s
_QE_SI = 1.602176634e-19        # C
_ME_SI = 9.1093837015e-31       # kg

_HBAR = _HBAR_SI / _QE_SI * 1e18         # meV fs   (1 J = 1e3/e meV, 1 s = 1e15 fs)
_HB2_2ME = _HBAR_SI ** 2 / (2.0 * _ME_SI) / _QE_SI * 1e21   # meV nm^2 for m = m_e
_E_OVER_HBAR = _QE_SI / _HBAR_SI * 1e-18  # 1 / (T nm^2)

WALL_HEIGHT_MEV = 10000.0   # V_b = 10 eV
WALL_SMOOTH_NM = 3.0        # tau = 3 nm
WALL_POS_FRAC = 0.4         # walls at y = +-0.4 Ly


@dataclass
class Workload:
    """Everything one propagation run needs, as plain numpy arrays."""
    name: str
    nx: int
    ny: int
    lx: float            # nm, box along x (per electron)
    ly: float            # nm, box along y
    mstar_rel: float     # m*/m_e
    eps_r: float
    b_tesla: float
    dt_fs: float
    steps: int
    soft_nm: float       # Coulomb softening length (2DEG thickness d)
    coulomb_c: float     # prefactor C of the Coulomb term (1 = bare, 0 = off)
    sym: int             # -1 antisymmetric, +1 symmetric, 0 distinguishable product
    v0: float
    v1: float
    sx: float
    sy: float
    sigma_x: float
    seed: int
    v_table: np.ndarray = field(repr=False)    # [nx, ny] float64, meV
    psi_a: np.ndarray = field(repr=False)      # [nx, ny] complex128, sum |.|^2 = 1
    psi_b: np.ndarray = field(repr=False)
    w_top: np.ndarray = field(repr=False)      # [nx, ny] float64 in {0, 1/2, 1}
    ckpt_every: int = 100
    info: dict = field(default_factory=dict)

    @property
    def points(self) -> int:
        return (self.nx * self.ny) ** 2

    def cfg(self) -> dict:
        """Scalar settings in the order the C ABI configuration struct uses."""
        return dict(nx=self.nx, ny=self.ny, lx_nm=self.lx, ly_nm=self.ly,
                    mstar_rel=self.mstar_rel, eps_r=self.eps_r, b_tesla=self.b_tesla,
                    dt_fs=self.dt_fs, soft_nm=self.soft_nm, coulomb_c=self.coulomb_c)


def grid_x(n: int, length: float) -> np.ndarray:
    return -0.5 * length + np.arange(n) * (length / n)


def grid_k(n: int, length: float) -> np.ndarray:
    """Angular wave numbers in FFT order; the Nyquist index maps to -pi/dx."""
    m = np.arange(n)
    m = np.where(m < (n + 1) // 2, m, m - n)
    return 2.0 * np.pi * m / length


def saddle_potential(x: np.ndarray, y: np.ndarray, v0: float, v1: float,
                     sx: float, sy: float, ly: float) -> np.ndarray:
    """V(x, y) in meV on the outer grid: saddle + Fermi walls along y."""
    X = x[:, None]
    Y = y[None, :]
    yw = WALL_POS_FRAC * ly
    with np.errstate(over="ignore"):   # exp overflow -> inf -> the wall term is exactly 0
        walls = WALL_HEIGHT_MEV * (1.0 / (1.0 + np.exp((yw - Y) / WALL_SMOOTH_NM))
                                   + 1.0 / (1.0 + np.exp((yw + Y) / WALL_SMOOTH_NM)))
    return v0 * np.exp(-X ** 2 / sx ** 2) - v1 * np.exp(-Y ** 2 / sy ** 2) + walls


def fermi(u: np.ndarray) -> np.ndarray:
    """Fermi step 1 / (exp(u / tau) + 1) of the barrier smoothness tau = 3 nm: 1 for u << 0."""
    return 0.5 * (1.0 - np.tanh(0.5 * u / WALL_SMOOTH_NM))


def fermi_block_qpc(x: np.ndarray, y: np.ndarray, ly: float, gap: float,
                    half_len: float) -> np.ndarray:
    """V(x, y) in meV: Fermi walls along y plus a constriction made of two
    Fermi-function blocks of height V_b (Sec. II.C Eq. (pot_xy)).

    Each block is a product of Fermi steps, as in the paper, rotated to this
    geometry (propagation along x): one hangs from the top wall over
    |x| < half_len down to y = +gap/2, the other rises from the bottom wall to
    y = -gap/2, leaving an opening of width gap between them."""
    X = x[:, None]
    Y = y[None, :]
    yw = WALL_POS_FRAC * ly
    walls = WALL_HEIGHT_MEV * (fermi(yw - Y) + fermi(yw + Y))
    fx = fermi(-X - half_len) * fermi(X - half_len)
    blocks = WALL_HEIGHT_MEV * fx * (fermi(0.5 * gap - Y) + fermi(Y + 0.5 * gap))
    return walls + blocks


def top_weights(nx: int, ny: int, ly: float) -> np.ndarray:
    """Weight of each single-particle grid point in the top region T = {y > 0}."""
    y = grid_x(ny, ly)
    w = np.where(y > 0, 1.0, 0.0)
    w = np.where(y == 0.0, 0.5, w)
    return np.broadcast_to(w[None, :], (nx, ny)).copy()


def _edge_states(ny, ly, kx, b_tesla, mstar_rel, vy):
    """Lowest eigenpair of the transverse Landau-gauge Hamiltonian for each kx.

    H(k) = kappa [ -d^2/dy^2 + (k - y eB/hbar)^2 ] + v(y), spectral in y.
    """
    kappa = _HB2_2ME / mstar_rel
    y = grid_x(ny, ly)
    ky = grid_k(ny, ly)
    eye = np.eye(ny)
    dft = np.fft.fft(eye, axis=0)
    t_y = np.real(np.fft.ifft(ky[:, None] ** 2 * dft, axis=0)) * kappa
    t_y = 0.5 * (t_y + t_y.T)
    inv_lb2 = _E_OVER_HBAR * b_tesla
    e1 = np.empty(len(kx))
    phi = np.empty((len(kx), ny))
    for i, k in enumerate(kx):
        h = t_y + np.diag(kappa * (k - y * inv_lb2) ** 2 + vy)
        w, v = np.linalg.eigh(h)
        vec = v[:, 0]
        if vec[np.argmax(np.abs(vec))] < 0:
            vec = -vec
        e1[i] = w[0]
        phi[i] = vec
    return e1, phi


def _packet(nx, ny, lx, ly, b_tesla, mstar_rel, vy, sigma_x, xc, top: bool,
            e_above_lll: float):
    kx = grid_k(nx, lx)
    x = grid_x(nx, lx)
    e1, phi = _edge_states(ny, ly, kx, b_tesla, mstar_rel, vy)
    kappa = _HB2_2ME / mstar_rel
    hw_c = 2.0 * kappa * _E_OVER_HBAR * b_tesla
    target = 0.5 * hw_c + e_above_lll
    cand = np.where(kx > 0)[0] if top else np.where(kx < 0)[0]
    i0 = cand[np.argmin(np.abs(e1[cand] - target))]
    k0 = kx[i0]
    amp = np.exp(-sigma_x ** 2 * (kx - k0) ** 2)
    psi = np.einsum("n,nx,ny->xy", amp, np.exp(1j * kx[:, None] * (x[None, :] - xc)), phi)
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2))
    return psi, dict(k0=float(k0), e1_k0=float(e1[i0]), target=float(target),
                     offset=float(e1[i0] - 0.5 * hw_c))


def build(name: str, nx: int, ny: int, lx: float, ly: float, *, b_tesla: float,
          dt_fs: float, steps: int, soft_nm: float = 2.0, coulomb_c: float = 1.0,
          sym: int = -1, v0: float = 4.0, v1: float = 2.0, sx: float = 30.0,
          sy: float = 60.0, sigma_x: float = 20.0, seed: int = 0,
          mstar_rel: float = 0.067, eps_r: float = 12.9, ckpt_every: int = 100,
          e_above_lll: float = 2.0, qpc_gap_nm: float | None = None,
          qpc_half_nm: float = 15.0, shift_nm: float = 0.0) -> Workload:
    """qpc_gap_nm set: the beam splitter is the Fermi-block constriction
    (fermi_block_qpc) instead of the saddle, and v0, v1, sx, sy are unused.
    shift_nm moves the bottom packet's start away from the splitter along its
    edge (the displacement between the two packets of Sec. III.B)."""
    x = grid_x(nx, lx)
    y = grid_x(ny, ly)
    dx = lx / nx
    jit = np.random.default_rng(seed).uniform(-0.5 * dx, 0.5 * dx, 2)
    xa = -0.25 * lx + jit[0]
    xb = +0.25 * lx + shift_nm + jit[1]
    if qpc_gap_nm is None:
        v = saddle_potential(x, y, v0, v1, sx, sy, ly)
    else:
        v = fermi_block_qpc(x, y, ly, qpc_gap_nm, qpc_half_nm)
        v0 = v1 = 0.0
    # transverse potential seen by each packet: the column of V nearest its start
    ia = int(np.argmin(np.abs(x - xa)))
    ib = int(np.argmin(np.abs(x - xb)))
    psi_a, ia_info = _packet(nx, ny, lx, ly, b_tesla, mstar_rel, v[ia], sigma_x, xa, True,
                             e_above_lll)
    psi_b, ib_info = _packet(nx, ny, lx, ly, b_tesla, mstar_rel, v[ib], sigma_x, xb, False,
                             e_above_lll)
    return Workload(name=name, nx=nx, ny=ny, lx=lx, ly=ly, mstar_rel=mstar_rel, eps_r=eps_r,
                    b_tesla=b_tesla, dt_fs=dt_fs, steps=steps, soft_nm=soft_nm,
                    coulomb_c=coulomb_c, sym=sym, v0=v0, v1=v1, sx=sx, sy=sy,
                    sigma_x=sigma_x, seed=seed, v_table=v, psi_a=psi_a, psi_b=psi_b,
                    w_top=top_weights(nx, ny, ly), ckpt_every=ckpt_every,
                    info=dict(xa=xa, xb=xb, alpha=ia_info, beta=ib_info, qpc_gap_nm=qpc_gap_nm,
                              qpc_half_nm=qpc_half_nm, shift_nm=shift_nm))


def mid_sweep():
    """The 9 runs of the 64x64 sweep: 3 seeded V0 values x sigma_x in {10, 20, 40} nm."""
    v0s = np.random.default_rng(0).uniform(3.0, 5.0, 3)
    return [(float(v0s[r // 3]), (10.0, 20.0, 40.0)[r % 3]) for r in range(9)]


def _with(kw, **defaults):
    """Preset defaults, overridden by the caller's keywords."""
    out = dict(defaults)
    out.update(kw)
    return out


def _tiny(seed=0, **kw):
    return build("tiny", 16, 16, 400.0, 400.0, seed=seed,
                 **_with(kw, b_tesla=5.0, dt_fs=5.0, steps=200, soft_nm=2.0, sigma_x=20.0))


def _mid(seed=0, run=0, **kw):
    v0, sig = mid_sweep()[run]
    return build("mid", 64, 64, 800.0, 600.0, seed=seed if seed else run,
                 **_with(kw, v0=v0, sigma_x=sig, b_tesla=5.0, dt_fs=2.0, steps=2000, soft_nm=2.0))


def _mixed(seed=0, **kw):
    return build("mixed", 128, 96, 1600.0, 900.0, seed=seed,
                 **_with(kw, b_tesla=6.0, dt_fs=1.0, steps=5000, soft_nm=1.0, sigma_x=20.0))


def _diff(seed=0, **kw):
    return build("diff", 48, 48, 600.0, 450.0, seed=seed,
                 **_with(kw, b_tesla=5.0, dt_fs=2.0, steps=1000, soft_nm=2.0, sigma_x=20.0,
                         ckpt_every=100))


def _full(seed=0, **kw):
    return build("full", 256, 128, 2000.0, 1000.0, seed=seed,
                 **_with(kw, b_tesla=5.0, dt_fs=0.5, steps=20000, soft_nm=2.0, sigma_x=10.0))


def _fp64_128(seed=0, **kw):
    return build("fp64_128", 128, 128, 1000.0, 1000.0, seed=seed,
                 **_with(kw, b_tesla=5.0, dt_fs=0.5, steps=1000, soft_nm=2.0, sigma_x=10.0))


# Resolving beam-splitter workload.  At 5 T (l_B = 11.47 nm) the grid keeps
# nx >= flux count lx*ly / (2 pi l_B^2) = 124 (every Landau-gauge guiding centre
# y0 = k_x l_B^2 across the strip is a grid wave number) and dy = 4 nm < l_B / 2.
# The packets sit 5 meV above the lowest Landau level (group velocity ~80
# nm/ps here; at 2 meV the packets of this wall profile are slow and strongly
# dispersive), and the opening is set so that a sigma = 15 nm packet leaves
# the constriction half transmitted.  The run ends before the reflected parts
# wrap around the periodic x direction back into the constriction.
QPC_GAP_NM = 60.2


def _qpc(seed=0, **kw):
    return build("qpc", 128, 64, 400.0, 256.0, seed=seed,
                 **_with(kw, sigma_x=15.0, qpc_gap_nm=QPC_GAP_NM, e_above_lll=5.0, coulomb_c=0.0,
                         steps=2500, b_tesla=5.0, dt_fs=1.0, soft_nm=1.0))


PRESETS = {"tiny": _tiny, "mid": _mid, "mixed": _mixed, "diff": _diff, "full": _full,
           "fp64_128": _fp64_128, "qpc": _qpc}


def preset(name: str, seed: int = 0, **overrides) -> Workload:
    """Build a named workload; keyword overrides replace any build() argument."""
    if name not in PRESETS:
        raise KeyError(f"unknown preset {name!r}; choose from {sorted(PRESETS)}")
    return PRESETS[name](seed=seed, **overrides)


def small(nx: int, ny: int, lx: float, ly: float, **kw) -> Workload:
    """A custom-size workload with the tiny preset's physics (for parity sweeps)."""
    kw.setdefault("b_tesla", 5.0)
    kw.setdefault("dt_fs", 5.0)
    kw.setdefault("steps", 20)
    return build("custom", nx, ny, lx, ly, **kw)


def replace(w: Workload, **changes) -> Workload:
    return dataclasses.replace(w, **changes)
