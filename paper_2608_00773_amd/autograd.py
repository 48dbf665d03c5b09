"""torch.autograd wrappers around q4c_integrate_H and its adjoint.

The forward is q4c_integrate_H (the five real parts of the atom-pair store
as a [5, store_len] tensor).  The backward is density_on_grid with the
upstream gradient as coefficients and weight_mode 1: dL/dv_g = w_g n_g,
the exact transpose of the forward on the stored elements (paper Eq. 39
with the density matrix replaced by dL/dH).  Both run in the HIP library.
"""
from __future__ import annotations

import torch

from . import (PREC_F64, TERM_ALL, Plan, density_on_grid, new_store, q4c_coef_from_spinor, q4c_integrate_H)


class Q4CIntegrate(torch.autograd.Function):
    """store = H(v); d store / d v is linear in v, so backward needs no saved tensors."""

    @staticmethod
    def forward(ctx, v: torch.Tensor, plan: Plan, precision: int = PREC_F64):
        v = v.contiguous()
        store = new_store(plan, v.device)
        q4c_integrate_H(plan, v, precision, 0, store)
        ctx.plan = plan
        ctx.n = v.numel()
        return store

    @staticmethod
    def backward(ctx, gstore: torch.Tensor):
        grad = None
        if ctx.needs_input_grad[0]:
            grad = torch.empty(ctx.n, dtype=torch.float64, device=gstore.device)
            density_on_grid(ctx.plan, gstore.contiguous(), TERM_ALL, 1, grad)
        return grad, None, None


def integrate(v: torch.Tensor, plan: Plan, precision: int = PREC_F64) -> torch.Tensor:
    """Differentiable H integration: [5, store_len] store from v [n_points]."""
    return Q4CIntegrate.apply(v, plan, precision)


def spinor_coefficients(plan: Plan, spin_d: torch.Tensor) -> torch.Tensor:
    """Store-layout coefficients whose contraction with the store gives
    Re Tr(D H) for a Hermitian spinor density matrix D (spinor block layout)."""
    out = new_store(plan, spin_d.device)
    q4c_coef_from_spinor(plan, spin_d.contiguous(), out)
    return out


def re_tr_dh(store: torch.Tensor, coef: torch.Tensor) -> torch.Tensor:
    """L = Re Tr(D H) = sum over stored elements of coef * store."""
    return torch.sum(coef * store)
