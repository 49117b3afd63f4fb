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
* Region probabilities of a two-electron state built from two orbitals
  (Sec. II.C Eq. (twopstate) with symmetry s): without the two-body term the
  4D propagation keeps this form with each orbital propagated in 2D, so the
  sums over configuration space reduce to one-electron matrix elements:
      sum w1 w2 |a1 b2 + s b1 a2|^2 = <a|w1|a><b|w2|b> + s^2 <b|w1|b><a|w2|a>
                                      + 2 s Re(<a|w1|b><b|w2|a>).

Pins: the orbital form of the region probabilities equals observables() of the
4D state init_state(a, b, s) for random orbitals and s = -1, 0, +1; the marginal of a product state is |psi_a|^2 <b|b>; for the Slater
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


def orbital_observables(a: np.ndarray, b: np.ndarray, w_top: np.ndarray, sym: int) -> dict:
    """Region probabilities of the normalised state a(r1) b(r2) + sym b(r1) a(r2)
    from one-electron matrix elements (no 4D array is formed)."""
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    wt = np.asarray(w_top, dtype=np.float64).ravel()
    wb = 1.0 - wt
    s = float(sym)

    def pair(w1, w2):
        return (np.vdot(a, w1 * a).real * np.vdot(b, w2 * b).real
                + s * s * np.vdot(b, w1 * b).real * np.vdot(a, w2 * a).real
                + 2.0 * s * np.real(np.vdot(a, w1 * b) * np.vdot(b, w2 * a)))

    one = np.ones_like(wt)
    norm = pair(one, one)
    p_tt, p_tb, p_bt, p_bb = (pair(wt, wt) / norm, pair(wt, wb) / norm, pair(wb, wt) / norm,
                              pair(wb, wb) / norm)
    return dict(norm=1.0, p_tt=p_tt, p_tb=p_tb, p_bt=p_bt, p_bb=p_bb, p_b=p_tt + p_bb,
                p_ab=p_tb + p_bt)


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
