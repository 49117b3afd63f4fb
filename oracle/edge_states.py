"""Edge states and Gaussian edge-state wave packets, FP64, on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Transverse eigenproblem (Sec. II.A, Eq. (H_effective)), written in the gauge
  A = (-B y, 0) used throughout, where the electrons propagate along x and the
  edge is transverse in y.  For each wave number k along x the one-electron
  Hamiltonian reduces to
      H(k) = kappa [ -d^2/dy^2 + (k - y eB/hbar)^2 ] + v(y),
  kappa = hbar^2 / 2m*; the quadratic term is m* omega_c^2 (y - y0)^2 / 2 with
  guiding centre y0 = k hbar / eB.  The second derivative is taken spectrally
  on the periodic y grid: the dense matrix F^-1 diag(kappa ky^2) F with the DFT
  matrix F written out.  Only the lowest eigenpair (the lowest Landau level's
  edge state) is kept; its sign is fixed by making the largest-magnitude
  component positive.
* Wave packet (Sec. II.B, Eq. (singlepwp)): a Gaussian superposition over the
  grid's wave numbers,
      psi(x, y) = sum_k exp(-sigma^2 (k - k0)^2) exp(i k (x - xc)) phi_k(y),
  normalised on the grid.  k0 is the wave number whose edge-state energy is
  closest to hbar omega_c / 2 + e_above (first such index), taken among k > 0
  for a packet on the top edge and k < 0 for the bottom edge.

Pins (tests/test_oracle_edge.py): with v = 0 and guiding centres well inside
the box the lowest eigenpair is the lowest Landau level, E = hbar omega_c / 2
and phi_k a Gaussian of width l_B centred at y0 = k l_B^2 (closed form); the
packet's projection on exp(i k x) phi_k(y) returns the Gaussian weights
exp(-sigma^2 (k - k0)^2) (the defining sum inverted, which fixes the sign of
the phase and xc); the chosen k0 is the brute-force closest level on the
requested side; the packet is normalised; and it agrees with the input
generator's packets (a separate implementation: FFT-built kinetic matrix).
"""
from __future__ import annotations

import numpy as np

from .splitstep import Grid


def kinetic_y(g: Grid) -> np.ndarray:
    """kappa (-d^2/dy^2) on the periodic y grid: F^-1 diag(kappa ky^2) F, dense, real."""
    n = g.ny
    j = np.arange(n)
    f = np.exp(-2j * np.pi * np.outer(j, j) / n)          # forward DFT matrix
    finv = np.conj(f) / n
    t = finv @ np.diag(g.kappa * g.ky ** 2) @ f
    return np.real(t)


def edge_hamiltonian(g: Grid, k: float, v_col: np.ndarray) -> np.ndarray:
    """H(k) of Eq. (H_effective) on the y grid (meV)."""
    d = g.kappa * (k - g.y * (g.e_over_hbar * g.b_tesla)) ** 2 + np.asarray(v_col, dtype=np.float64)
    return kinetic_y(g) + np.diag(d)


def lowest_edge_states(g: Grid, v_col: np.ndarray):
    """Lowest eigenpair of H(k) for every grid wave number k along x.

    Returns e1 [nx] (meV) and phi [nx, ny] (real, unit norm, largest-magnitude
    component positive)."""
    e1 = np.empty(g.nx)
    phi = np.empty((g.nx, g.ny))
    for m, k in enumerate(g.kx):
        w, v = np.linalg.eigh(edge_hamiltonian(g, k, v_col))
        vec = v[:, 0]
        if vec[np.argmax(np.abs(vec))] < 0:
            vec = -vec
        e1[m] = w[0]
        phi[m] = vec
    return e1, phi


def edge_packet(g: Grid, v_col: np.ndarray, sigma_x: float, xc: float, top: bool,
                e_above_lll: float):
    """Normalised packet psi [nx, ny] of Eq. (singlepwp) and its (k0, E(k0), target)."""
    e1, phi = lowest_edge_states(g, v_col)
    hw_c = 2.0 * g.kappa * g.e_over_hbar * g.b_tesla
    target = 0.5 * hw_c + e_above_lll
    kx = g.kx
    cand = np.where(kx > 0)[0] if top else np.where(kx < 0)[0]
    i0 = cand[np.argmin(np.abs(e1[cand] - target))]
    k0 = kx[i0]
    psi = np.zeros((g.nx, g.ny), dtype=np.complex128)
    for m, k in enumerate(kx):
        a = np.exp(-sigma_x ** 2 * (k - k0) ** 2)
        psi += a * np.exp(1j * k * (g.x - xc))[:, None] * phi[m][None, :]
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2))
    return psi, dict(k0=float(k0), e1_k0=float(e1[i0]), target=float(target))
