"""Differentiable effective stiffness: C_eff(E) for a per-voxel Young's modulus
field with a uniform Poisson ratio, as a torch.autograd.Function.

Forward: one batched solve of the nv unit load cases (``Homogenizer.solve``)
and the energy form of C_eff.  Backward: for the incoming gradient G = dJ/dC_eff
the library returns dJ/dE_v per voxel (``feh_energy_sensitivity_E`` with the
weights E^-1 G E^-T from ``feh_effective_stiffness_weights``; no second solve,
the problem being self-adjoint).  This module only marshals arguments.
"""
from __future__ import annotations

import torch

from . import feh_effective_stiffness_weights, unit_loads


class EffectiveStiffness(torch.autograd.Function):
    """C = EffectiveStiffness.apply(E, nu, homogenizer, tol, max_iter).

    E: device tensor of the grid shape in the homogenizer's precision;
    homogenizer: a Homogenizer with n_load = nv (3 in 2D, 6 in 3D).  Returns
    the nv x nv FP64 C_eff as a CPU tensor; its gradient with respect to E
    comes back on E's device in E's dtype."""

    @staticmethod
    def forward(ctx, E, nu, hz, tol, max_iter):
        nv = 3 if hz.dim == 2 else 6
        if hz.n_per != nv or hz.n_batch != 1:
            raise ValueError("the homogenizer must hold one microstructure and its nv unit load cases")
        hz.set_material(E=E.detach(), nu=float(nu))
        out = hz.solve(unit_loads(hz.dim), tol=tol, max_iter=max_iter)
        ctx.hz = hz
        ctx.E_device, ctx.E_dtype = E.device, E.dtype
        return torch.as_tensor(out["C_eff"], dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_C):
        hz = ctx.hz
        W = feh_effective_stiffness_weights(hz.dim, hz._last_Ebar, grad_C.detach().cpu().numpy())
        gE = hz.energy_sensitivity_E(W)
        return gE.to(device=ctx.E_device, dtype=ctx.E_dtype), None, None, None, None
