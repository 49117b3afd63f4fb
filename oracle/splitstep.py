"""Split-step Fourier propagation of the two-electron state, FP64, on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What it computes (arXiv 1903.02581, Sec. II.C Eq. (evoloperat), Appendix A):
the two-particle Hamiltonian H = T_{x1,x2} + T_{y1,y2} + V1 + V2 + V12 is split
into three pieces, each diagonal in one mixed real/reciprocal representation,
and the state is advanced by products of their exponentials.  The two kinetic
pieces are applied with 2D discrete Fourier transforms over a pair of
coordinates, (x1, x2) or (y1, y2), exactly as the paper describes.

Readings taken where the paper is silent or garbled:
  * gauge A = (-B y, 0) for an electron of charge -e, so T_x = (hbar k_x - e B y)^2/2m*
    is diagonal in (k_x, y) and T_y = hbar^2 k_y^2/2m* in k_y (the paper uses the
    rotated gauge A = (0, B x, 0));
  * symmetric (Strang) order S(dt) = X(dt/2) V(dt/2) Y(dt) V(dt/2) X(dt/2); the
    paper prints the first-order product;
  * forward DFT with exp(-i k x), k from numpy's fftfreq, so the Nyquist index
    carries k = -pi/dx;
  * V12 = C e^2/(4 pi eps0 eps_r sqrt(|r1 - r2|^2 + d^2)), plain (non-periodic)
    coordinate differences, optionally times exp(-|r1 - r2|/sigma_c)
    (Eq. (coulomb), Eq. (screenedCoulomb));
  * the same external potential V(x, y) acts on both electrons.

Pins (tests/test_oracle_pins.py): free Gaussian closed form at B = 0 (P1),
Strang lowest-Landau-level eigenphase (P2), norm / exchange symmetry /
coincidence node (P3), dense matrix-exponential brute force on a 6x6 grid per
electron including the Coulomb term, plus the second-order convergence to
expm(-iHt) (P4), factorisation into 2D propagations when V12 = 0 (P5), time
reversal (P6).
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

# CODATA 2018 SI values.
HBAR_SI = 1.054571817e-34       # J s
QE_SI = 1.602176634e-19         # C
ME_SI = 9.1093837015e-31        # kg
EPS0_SI = 8.8541878128e-12      # F / m

_WORKERS = os.cpu_count() or 1


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    lx: float          # nm
    ly: float          # nm
    mstar_rel: float
    eps_r: float
    b_tesla: float
    soft_nm: float     # d
    coulomb_c: float   # C
    screen_nm: float   # sigma_c; 0 = unscreened

    # derived, in nm / fs / meV
    @property
    def hbar(self) -> float:
        """hbar in meV fs."""
        return HBAR_SI / QE_SI * 1e3 * 1e15

    @property
    def kappa(self) -> float:
        """hbar^2 / 2m* in meV nm^2."""
        return HBAR_SI ** 2 / (2.0 * self.mstar_rel * ME_SI) / QE_SI * 1e3 * 1e18

    @property
    def k_coul(self) -> float:
        """e^2 / (4 pi eps0 eps_r) in meV nm."""
        return QE_SI ** 2 / (4.0 * np.pi * EPS0_SI * self.eps_r) / QE_SI * 1e3 * 1e9

    @property
    def e_over_hbar(self) -> float:
        """e / hbar in 1 / (T nm^2); e B / hbar = 1 / l_B^2."""
        return QE_SI / HBAR_SI * 1e-18

    @property
    def x(self) -> np.ndarray:
        return -0.5 * self.lx + np.arange(self.nx) * (self.lx / self.nx)

    @property
    def y(self) -> np.ndarray:
        return -0.5 * self.ly + np.arange(self.ny) * (self.ly / self.ny)

    @property
    def kx(self) -> np.ndarray:
        return 2.0 * np.pi * np.fft.fftfreq(self.nx, d=self.lx / self.nx)

    @property
    def ky(self) -> np.ndarray:
        return 2.0 * np.pi * np.fft.fftfreq(self.ny, d=self.ly / self.ny)


def make_grid(nx, ny, lx, ly, *, mstar_rel=0.067, eps_r=12.9, b_tesla=5.0, soft_nm=2.0,
              coulomb_c=1.0, screen_nm=0.0) -> Grid:
    return Grid(int(nx), int(ny), float(lx), float(ly), float(mstar_rel), float(eps_r),
                float(b_tesla), float(soft_nm), float(coulomb_c), float(screen_nm))


# ----------------------------------------------------------------------------- angles

def theta_x(g: Grid, tau: float, b_tesla: float | None = None) -> np.ndarray:
    """Kinetic angle of one electron in the (k_x, y) representation, shape [nx, ny].

    theta = (tau/hbar) * (hbar k_x - e B y)^2 / 2m*  =  (tau/hbar) kappa (k_x - y eB/hbar)^2
    (Appendix A, Eq. (2PTB) rewritten in the gauge A = (-B y, 0)).
    """
    b = g.b_tesla if b_tesla is None else b_tesla
    shift = g.y[None, :] * (g.e_over_hbar * b)
    return (tau / g.hbar) * g.kappa * (g.kx[:, None] - shift) ** 2


def dtheta_x_db(g: Grid, tau: float) -> np.ndarray:
    """Derivative of theta_x with respect to B, shape [nx, ny] (per tesla)."""
    eoh = g.e_over_hbar
    q = g.kx[:, None] - g.y[None, :] * (eoh * g.b_tesla)
    return (tau / g.hbar) * g.kappa * 2.0 * q * (-g.y[None, :] * eoh)


def theta_y(g: Grid, tau: float) -> np.ndarray:
    """Kinetic angle along y, shape [ny]: (tau/hbar) hbar^2 k_y^2 / 2m*."""
    return (tau / g.hbar) * g.kappa * g.ky ** 2


def coulomb(g: Grid) -> np.ndarray:
    """Two-body potential V12(x1, y1, x2, y2) in meV, shape [nx, ny, nx, ny].

    Eq. (coulomb); with screen_nm > 0, Eq. (screenedCoulomb).
    """
    x, y = g.x, g.y
    dx = x[:, None, None, None] - x[None, None, :, None]
    dy = y[None, :, None, None] - y[None, None, None, :]
    r2 = dx ** 2 + dy ** 2
    v12 = g.coulomb_c * g.k_coul / np.sqrt(r2 + g.soft_nm ** 2)
    if g.screen_nm > 0.0:
        v12 = v12 * np.exp(-np.sqrt(r2) / g.screen_nm)
    return v12


def theta_v(g: Grid, v_table: np.ndarray, tau: float) -> np.ndarray:
    """Real-space angle (tau/hbar) [V(r1) + V(r2) + V12(r1, r2)], shape [nx, ny, nx, ny]."""
    v = np.asarray(v_table, dtype=np.float64)
    tot = v[:, :, None, None] + v[None, None, :, :]
    if g.coulomb_c != 0.0:
        tot = tot + coulomb(g)
    return (tau / g.hbar) * tot


# ---------------------------------------------------------------------------- factors

def apply_x(psi: np.ndarray, g: Grid, tau: float) -> np.ndarray:
    """exp(-i tau T_{x1,x2}/hbar): 2D transform over (x1, x2), phase, inverse."""
    th = theta_x(g, tau)
    phase = np.exp(-1j * (th[:, :, None, None] + th[None, None, :, :]))
    phi = sfft.fftn(psi, axes=(0, 2), workers=_WORKERS)
    return sfft.ifftn(phi * phase, axes=(0, 2), workers=_WORKERS)


def apply_y(psi: np.ndarray, g: Grid, tau: float) -> np.ndarray:
    """exp(-i tau T_{y1,y2}/hbar): 2D transform over (y1, y2), phase, inverse."""
    th = theta_y(g, tau)
    phase = np.exp(-1j * (th[None, :, None, None] + th[None, None, None, :]))
    phi = sfft.fftn(psi, axes=(1, 3), workers=_WORKERS)
    return sfft.ifftn(phi * phase, axes=(1, 3), workers=_WORKERS)


def apply_v(psi: np.ndarray, g: Grid, v_table: np.ndarray, tau: float) -> np.ndarray:
    """exp(-i tau (V1 + V2 + V12)/hbar), diagonal in 4D real space."""
    return psi * np.exp(-1j * theta_v(g, v_table, tau))


def strang_step(psi, g: Grid, v_table, dt: float):
    """One symmetric step S(dt) = X(dt/2) V(dt/2) Y(dt) V(dt/2) X(dt/2)."""
    psi = apply_x(psi, g, 0.5 * dt)
    psi = apply_v(psi, g, v_table, 0.5 * dt)
    psi = apply_y(psi, g, dt)
    psi = apply_v(psi, g, v_table, 0.5 * dt)
    psi = apply_x(psi, g, 0.5 * dt)
    return psi


def propagate(psi0, g: Grid, v_table, dt: float, n: int, every: int = 0, on_sample=None):
    """Apply S(dt) n times.  If every > 0, call on_sample(step, psi) after each
    multiple of `every` steps (observables are taken after whole steps only)."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for i in range(1, n + 1):
        psi = strang_step(psi, g, v_table, dt)
        if every and on_sample is not None and i % every == 0:
            on_sample(i, psi)
    return psi


def init_state(psi_a: np.ndarray, psi_b: np.ndarray, sym: int) -> np.ndarray:
    """Two-electron state of Sec. II.C Eq. (twopstate), normalised on the grid.

    sym = -1: psi_a(r1) psi_b(r2) - psi_a(r2) psi_b(r1)  (Slater determinant)
    sym = +1: the symmetric combination;  sym = 0: the product psi_a(r1) psi_b(r2).
    Normalisation: sum over the 4D grid of |Psi|^2 = 1.
    """
    a = np.asarray(psi_a, dtype=np.complex128)
    b = np.asarray(psi_b, dtype=np.complex128)
    psi = a[:, :, None, None] * b[None, None, :, :]
    if sym in (-1, 1):
        psi = psi + sym * (b[:, :, None, None] * a[None, None, :, :])
    elif sym != 0:
        raise ValueError("sym must be -1, 0 or +1")
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2))


# --------------------------------------------------- one electron (for the V12 = 0 pin)

def strang_step_2d(psi2, g: Grid, v_table, dt: float):
    """The same factors acting on a single-electron state psi(x, y)."""
    def ax(p, tau):
        th = theta_x(g, tau)
        return np.fft.ifft(np.fft.fft(p, axis=0) * np.exp(-1j * th), axis=0)

    def ay(p, tau):
        th = theta_y(g, tau)
        return np.fft.ifft(np.fft.fft(p, axis=1) * np.exp(-1j * th)[None, :], axis=1)

    def av(p, tau):
        return p * np.exp(-1j * (tau / g.hbar) * np.asarray(v_table))

    p = ax(psi2, 0.5 * dt)
    p = av(p, 0.5 * dt)
    p = ay(p, dt)
    p = av(p, 0.5 * dt)
    return ax(p, 0.5 * dt)


def propagate_2d(psi2, g: Grid, v_table, dt: float, n: int):
    p = np.array(psi2, dtype=np.complex128, copy=True)
    for _ in range(n):
        p = strang_step_2d(p, g, v_table, dt)
    return p
