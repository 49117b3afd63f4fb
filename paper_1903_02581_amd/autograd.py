"""torch.autograd bridge for gradients of region probabilities.

BunchingLoss maps (V table, B) to L = sum_ij c_ij P_ij of the final state of a
recorded forward run (Eq. (p_bunching) of arXiv 1903.02581; c = (1, 0, 0, 1)
gives the bunching probability).  Its backward is the library's reverse sweep
(exact reverse propagation of state and adjoint with checkpoint restores).
The potential parameters (V0, V1, sx, sy) enter through saddle_potential,
written with torch ops so autograd chains dL/dV into dL/dtheta.
"""
from __future__ import annotations

import numpy as np
import torch

WALL_HEIGHT_MEV = 10000.0
WALL_SMOOTH_NM = 3.0
WALL_POS_FRAC = 0.4


def saddle_potential(theta: torch.Tensor, x: torch.Tensor, y: torch.Tensor, ly: float):
    """V(x, y) = V0 exp(-x^2/sx^2) - V1 exp(-y^2/sy^2) + Fermi walls at y = +-0.4 Ly
    (barrier shape of Eq. (pot_x): height 10 eV, smoothness 3 nm).  theta = (V0, V1, sx, sy)."""
    v0, v1, sx, sy = theta[0], theta[1], theta[2], theta[3]
    X = x[:, None]
    Y = y[None, :]
    yw = WALL_POS_FRAC * ly
    walls = WALL_HEIGHT_MEV * (torch.sigmoid((Y - yw) / WALL_SMOOTH_NM)
                               + torch.sigmoid(-(Y + yw) / WALL_SMOOTH_NM))
    return v0 * torch.exp(-X ** 2 / sx ** 2) - v1 * torch.exp(-Y ** 2 / sy ** 2) + walls


class BunchingLoss(torch.autograd.Function):
    """L(V, B) for a fixed initial state; see the module docstring.

    forward(v_table [nx, ny] float64, b (0-d float64), prop, psi_a, psi_b, sym, steps,
            w_top, ckpt_every, coeffs) -> L (0-d float64)
    """

    @staticmethod
    def forward(ctx, v_table, b, prop, psi_a, psi_b, sym, steps, w_top, ckpt_every, coeffs):
        prop.set_potential(v_table.detach().cpu().numpy())
        prop.set_field(float(b))
        prop.init_state(psi_a, psi_b, sym)
        prop.grad_begin(ckpt_every, steps)
        prop.step(steps)
        # the four region probabilities are the library's FP64 reduction of the final
        # state; the reverse sweep recomputes L with the same weights (checked in backward)
        o = prop.observables(w_top)
        c = np.asarray(coeffs, dtype=np.float64)
        loss = c[0] * o["p_tt"] + c[1] * o["p_tb"] + c[2] * o["p_bt"] + c[3] * o["p_bb"]
        ctx.loss = loss
        ctx.prop = prop
        ctx.w_top = w_top
        ctx.coeffs = c
        ctx.v_shape = v_table.shape
        ctx.v_dtype = v_table.dtype
        ctx.v_device = v_table.device
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        loss, dldv, dldb = ctx.prop.grad_backward(ctx.w_top, ctx.coeffs)
        if not abs(loss - ctx.loss) <= 1e-12 * max(1.0, abs(ctx.loss)):
            raise RuntimeError(f"reverse sweep's loss {loss!r} differs from the forward's {ctx.loss!r}")
        g = grad_out.detach().cpu().double()
        gv = torch.from_numpy(dldv).to(ctx.v_device, ctx.v_dtype) * g.to(ctx.v_device)
        gb = torch.tensor(dldb, dtype=torch.float64) * g
        return gv, gb, None, None, None, None, None, None, None, None


def bunching_loss(v_table, b, prop, psi_a, psi_b, *, sym=-1, steps, w_top, ckpt_every=100,
                  coeffs=(1.0, 0.0, 0.0, 1.0)):
    return BunchingLoss.apply(v_table, b, prop, psi_a, psi_b, sym, steps, w_top, ckpt_every,
                              coeffs)
