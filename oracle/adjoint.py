"""Sensitivities of the effective stiffness to the per-voxel material, FP64, CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Energy matrix.  For load cases l, m with equilibrium strains e_l, e_m (element
fields, Sec. "Compatibility projection": the weak form is the stationarity of
the strain energy over compatible fluctuations),
    W_lm = < e_l : C : e_m >,          C_eff = E^-T W E^-1,
with E the matrix whose columns are the engineering Voigt strains of the load
cases (the energy form of the effective stiffness).

Derivative.  W_ll is the minimum over compatible fluctuations of the energy
< (Ebar_l + B u) : C : (Ebar_l + B u) >, so a first-order change of C at fixed
strain gives the whole first-order change of W_ll (the fluctuation is
stationary).  W is a quadratic form in Ebar, so the off-diagonal entries
follow by polarisation:
    dW_lm / dlambda_v = < tr e_l  tr e_m >_v,
    dW_lm / dmu_v     = < 2 e_l : e_m >_v,
where < . >_v sums the element terms of voxel v only, with the weights of the
full-cell average (|e| / |Omega|).  No second (adjoint) solve is needed: the
problem is self-adjoint and the adjoint field of W_lm is the forward field of
load case m.

For an objective J = sum_IJ G_IJ C_eff_IJ the chain rule gives
    dJ / dW_lm = (E^-1 G E^-T)_lm.
With a uniform Poisson ratio, lambda and mu are linear in E, so
    dJ / dE_v = dJ/dlambda_v * nu / ((1 + nu)(1 - 2 nu)) + dJ/dmu_v / (2 (1 + nu))
(plane strain / 3D; the same Lame maps as fe.lame).

Arrays: strain fields e_l are (N, n_e, D, D) as returned by fe.fields; the
voxel index is the C-order flat index of the grid.
"""
from __future__ import annotations

import numpy as np

from . import fe


def _weights(dim, ne, N, h=None):
    """|e| / |Omega| for the elements of one voxel (all voxels alike)."""
    w = fe.element_volumes(dim, h)
    return w / (w.sum() * N)


def energy_sensitivity(eps_list, h=None, n_voxels=None):
    """dW/dlambda and dW/dmu per voxel: arrays (L, L, N) each.  With n_voxels,
    eps_list holds the strains of a subset of the voxels of a grid of
    n_voxels (fe.element_strains_at) and the result covers that subset."""
    L = len(eps_list)
    N, ne, dim, _ = eps_list[0].shape
    w = _weights(dim, ne, N if n_voxels is None else n_voxels, h)
    tr = [np.trace(e, axis1=2, axis2=3) for e in eps_list]  # (N, ne)
    dl = np.zeros((L, L, N))
    dm = np.zeros((L, L, N))
    for l in range(L):
        for m in range(L):
            dl[l, m] = (tr[l] * tr[m]) @ w
            dm[l, m] = (2.0 * np.einsum("neij,neij->ne", eps_list[l], eps_list[m])) @ w
    return dl, dm


def objective_weights(Ebars, G):
    """dJ/dW for J = sum G_IJ C_eff_IJ: the matrix E^-1 G E^-T."""
    Ev = np.stack([fe.voigt_strain(E) for E in Ebars], axis=1)
    Einv = np.linalg.inv(Ev)
    return Einv @ np.asarray(G, float) @ Einv.T


def objective_gradient(eps_list, Ebars, G, h=None, n_voxels=None):
    """dJ/dlambda_v and dJ/dmu_v (each (N,)) for J = sum G_IJ C_eff_IJ
    (n_voxels: as in energy_sensitivity)."""
    Wt = objective_weights(Ebars, G)
    dl, dm = energy_sensitivity(eps_list, h, n_voxels)
    return np.einsum("lm,lmn->n", Wt, dl), np.einsum("lm,lmn->n", Wt, dm)


def lame_derivatives(nu):
    """(dlambda/dE, dmu/dE) at a given Poisson ratio (plane strain / 3D)."""
    return nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), 1.0 / (2.0 * (1.0 + nu))


def e_gradient(g_lam, g_mu, nu):
    """dJ/dE_v for a uniform Poisson ratio."""
    a, b = lame_derivatives(nu)
    return a * np.asarray(g_lam) + b * np.asarray(g_mu)
