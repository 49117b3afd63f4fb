"""Observables of the two-electron state, FP64, on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Region-resolved probabilities (Sec. III, Eq. (p_bunching)): the single
  electron plane is split into a top region T and a bottom region B, given as a
  weight table w(x, y) in [0, 1] for T (1 - w for B).  Then
      P_ij = sum_{r1, r2} w_i(r1) w_j(r2) |Psi(r1, r2)|^2,   i, j in {T, B},
      P_b = P_TT + P_BB,  P_ab = P_TB + P_BT,  norm = sum |Psi|^2.
  The sums are the raw grid sums (not divided by the norm), so P_ab = 1 - P_b
  holds to the accuracy of the norm.
* Spatial entanglement (Sec. III.C, Eq. (reduced_density)): the slice
  phi(x1, x2) = Psi(x1, y1*, x2, y2*) is renormalised, the reduced density
  matrix rho_T = phi phi^dagger is formed and S = -Tr rho ln rho (natural log;
  the paper's formula drops the minus sign and has an index typo).  Computed
  from the singular values of phi: the eigenvalues of rho are their squares.

* Marginal and conditional one-electron densities (Fig. 3(b), Fig. 2 captions).

Pins: the marginal of a product state is |psi_a|^2 <b|b>; for the Slater
determinant the marginal has the closed form (|a|^2 + |b|^2 - 2 Re(conj(a) b
<b|a>)) / (2 (1 - |<a|b>|^2)) for normalised a, b; the conditional probability
vanishes at r1 = r2* (Pauli node of the Fig. 2 caption);
P_TT + P_TB + P_BT + P_BB = norm and P_TB = P_BT for exchange-symmetric
states (invariants); entanglement of a product state is 0 and of a two-term
Schmidt state with orthonormal factors is ln 2; the SVD route agrees with the
eigenvalues of rho computed by numpy.linalg.eigvalsh.
"""
from __future__ import annotations

import numpy as np


def region_weights_4d(w_top: np.ndarray):
    w = np.asarray(w_top, dtype=np.float64)
    w1 = w[:, :, None, None]
    w2 = w[None, None, :, :]
    return w1, w2


def observables(psi: np.ndarray, w_top: np.ndarray) -> dict:
    dens = np.abs(psi) ** 2
    w1, w2 = region_weights_4d(w_top)
    p_tt = float(np.sum(w1 * w2 * dens))
    p_tb = float(np.sum(w1 * (1.0 - w2) * dens))
    p_bt = float(np.sum((1.0 - w1) * w2 * dens))
    p_bb = float(np.sum((1.0 - w1) * (1.0 - w2) * dens))
    return dict(norm=float(np.sum(dens)), p_tt=p_tt, p_tb=p_tb, p_bt=p_bt, p_bb=p_bb,
                p_b=p_tt + p_bb, p_ab=p_tb + p_bt)


def marginal(psi: np.ndarray) -> np.ndarray:
    """Unconditional probability of electron 1 (Sec. III.A, Fig. 3(b) caption):
    P(x1, y1) = sum_{x2, y2} |Psi|^2."""
    return np.sum(np.abs(psi) ** 2, axis=(2, 3))


def conditional(psi: np.ndarray, ix2: int, jy2: int) -> np.ndarray:
    """Conditional probability of electron 1 with electron 2 at (x2*, y2*)
    (Sec. II.A, Fig. 2 caption): |Psi(x1, y1, x2*, y2*)|^2, not renormalised."""
    return np.abs(psi[:, :, ix2, jy2]) ** 2


def entanglement(psi: np.ndarray, ix1, jy1: int, ix2, jy2: int) -> float:
    ix1 = np.asarray(ix1, dtype=np.int64)
    ix2 = np.asarray(ix2, dtype=np.int64)
    phi = psi[ix1, jy1][:, ix2, jy2]
    nrm = np.sqrt(np.sum(np.abs(phi) ** 2))
    if nrm == 0.0:
        raise ValueError("slice has zero norm")
    phi = phi / nrm
    s = np.linalg.svd(phi, compute_uv=False)
    p = s ** 2
    p = p[p > 0.0]
    return float(-np.sum(p * np.log(p)))
