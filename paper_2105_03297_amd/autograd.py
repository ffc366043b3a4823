"""Differentiable effective stiffness: C_eff(E) for a per-voxel Young's modulus
field with a uniform Poisson ratio, as a torch.autograd.Function.

Forward: one batched solve of the nv unit load cases (``Homogenizer.solve``)
and the energy form of C_eff.  Backward: for the incoming gradient G = dJ/dC_eff
the library returns dJ/dlambda_v and dJ/dmu_v per voxel (``feh_energy_sensitivity``
with the weights E^-1 G E^-T; no second solve, the problem being
self-adjoint), and lambda, mu are linear in E at fixed nu.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Homogenizer, feh_effective_stiffness_weights

UNIT_STRAIN = 0.01


def unit_loads(dim):
    """Unit Voigt loads: tensor strain 0.01 per normal component, 0.01 per
    shear pair (engineering shear 0.02)."""
    pairs = [(0, 0), (1, 1), (0, 1)] if dim == 2 else [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    Eb = np.zeros((len(pairs), dim, dim))
    for k, (a, b) in enumerate(pairs):
        Eb[k, a, b] = Eb[k, b, a] = UNIT_STRAIN
    return Eb


def lame_derivatives(nu):
    """(dlambda/dE, dmu/dE) of plane strain / 3D isotropic elasticity."""
    return nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), 1.0 / (2.0 * (1.0 + nu))


class EffectiveStiffness(torch.autograd.Function):
    """C = EffectiveStiffness.apply(E, nu, homogenizer, tol, max_iter).

    E: device tensor of the grid shape in the homogenizer's precision;
    homogenizer: a Homogenizer with n_load = nv (3 in 2D, 6 in 3D).  Returns
    the nv x nv FP64 C_eff on the host device of E's choice (CPU tensor)."""

    @staticmethod
    def forward(ctx, E, nu, hz, tol, max_iter):
        nv = 3 if hz.dim == 2 else 6
        if hz.n_per != nv or hz.n_batch != 1:
            raise ValueError("the homogenizer must hold one microstructure and its nv unit load cases")
        hz.set_material(E=E.detach(), nu=float(nu))
        out = hz.solve(unit_loads(hz.dim), tol=tol, max_iter=max_iter)
        ctx.hz = hz
        ctx.nu = float(nu)
        ctx.E_device, ctx.E_dtype = E.device, E.dtype
        return torch.as_tensor(out["C_eff"], dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_C):
        hz = ctx.hz
        W = feh_effective_stiffness_weights(hz.dim, hz._last_Ebar, grad_C.detach().cpu().numpy())
        g_lam, g_mu = hz.energy_sensitivity(W)
        a, b = lame_derivatives(ctx.nu)
        gE = (a * g_lam.double() + b * g_mu.double()).to(device=ctx.E_device, dtype=ctx.E_dtype)
        return gE, None, None, None, None
