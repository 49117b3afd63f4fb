"""Gradients of the bunching probability, FP64, on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

L = sum_{r1,r2} w_L(r1, r2) |Psi_N(r1, r2)|^2 with Psi_N = S(dt)^N Psi_0 and
w_L = a_TT w1 w2 + a_TB w1 (1-w2) + a_BT (1-w1) w2 + a_BB (1-w1)(1-w2); the
default (1, 0, 0, 1) is the bunching probability of Eq. (p_bunching).  The
initial state is held fixed; V(x, y) and B enter only through the factor
angles (B only through the x kinetic angle in the gauge A = (-B y, 0)).

Two independent routes:

* ``loss_and_grad_stored`` -- reverse mode with every intermediate state
  stored.  For a factor A = exp(-i diag(theta)) in some basis, applied to a
  state phi, with lambda = (later factors)^dagger w_L Psi_N:
      dL/dtheta_j = 2 Im( conj(lambda_j) (A phi)_j ),
  evaluated in the basis where A is diagonal; for the 2D transform over
  (x1, x2) the Parseval factor 1/nx^2 of the unnormalised DFT applies.  lambda
  is carried back through each factor by A^dagger = A(-tau).  Then
      dL/dV(x, y) = sum_V-factors (tau/hbar) [ sum_r2 g(x,y,r2) + sum_r1 g(r1,x,y) ],
      dL/dB       = sum_X-factors sum g_hat(k1,y1,k2,y2) dtheta_x/dB.
* ``grad_fd`` -- central finite differences of the plain forward propagation.

Pins: the two routes agree (tests), and sum_{x,y} dL/dV = 0 because a uniform
shift of V only multiplies the state by a global phase.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from .splitstep import Grid, apply_v, apply_x, apply_y, dtheta_x_db

_WORKERS = os.cpu_count() or 1


def loss_weights(w_top, coeffs=(1.0, 0.0, 0.0, 1.0)) -> np.ndarray:
    w = np.asarray(w_top, dtype=np.float64)
    w1 = w[:, :, None, None]
    w2 = w[None, None, :, :]
    a_tt, a_tb, a_bt, a_bb = coeffs
    return (a_tt * w1 * w2 + a_tb * w1 * (1 - w2) + a_bt * (1 - w1) * w2
            + a_bb * (1 - w1) * (1 - w2))


def _factors(dt):
    return [("x", 0.5 * dt), ("v", 0.5 * dt), ("y", dt), ("v", 0.5 * dt), ("x", 0.5 * dt)]


def _apply(kind, psi, g, v_table, tau):
    if kind == "x":
        return apply_x(psi, g, tau)
    if kind == "y":
        return apply_y(psi, g, tau)
    return apply_v(psi, g, v_table, tau)


def loss_and_grad_stored(psi0, g: Grid, v_table, dt: float, n: int, w_top,
                         coeffs=(1.0, 0.0, 0.0, 1.0)):
    """Returns (L, dL/dV [nx, ny], dL/dB)."""
    wl = loss_weights(w_top, coeffs)
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    after = []
    for _ in range(n):
        for kind, tau in _factors(dt):
            psi = _apply(kind, psi, g, v_table, tau)
            after.append((kind, tau, psi))
    loss = float(np.sum(wl * np.abs(psi) ** 2))
    lam = wl * psi
    g_v = np.zeros((g.nx, g.ny))
    g_b = 0.0
    for kind, tau, st in reversed(after):
        if kind == "v":
            c = 2.0 * np.imag(np.conj(lam) * st)
            g_v += (tau / g.hbar) * (c.sum(axis=(2, 3)) + c.sum(axis=(0, 1)))
        elif kind == "x":
            lh = sfft.fftn(lam, axes=(0, 2), workers=_WORKERS)
            sh = sfft.fftn(st, axes=(0, 2), workers=_WORKERS)
            c = 2.0 * np.imag(np.conj(lh) * sh) / (g.nx * g.nx)
            d = dtheta_x_db(g, tau)
            g_b += float(np.sum(c * (d[:, :, None, None] + d[None, None, :, :])))
        lam = _apply(kind, lam, g, v_table, -tau)
    return loss, g_v, g_b


def grad_fd(loss_of, theta, h_rel=1e-4):
    """Central differences of a scalar function of a parameter vector.

    Step h_i = h_rel * |theta_i| (h_rel if theta_i == 0)."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.empty_like(theta)
    for i in range(theta.size):
        h = h_rel * abs(theta[i]) if theta[i] != 0.0 else h_rel
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        out[i] = (loss_of(tp) - loss_of(tm)) / (tp[i] - tm[i])
    return out
