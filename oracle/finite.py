"""Finite-strain homogenization with the compatibility projection, FP64, CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (Sec. "Compatibility projection"): static equilibrium div_0 P(F) = 0 of
the periodic cell, with the deformation gradient F = grad_0 chi as the unknown
and its mean Fbar as the macroscopic boundary condition.  The weak form with
compatible test gradients is G * P(F) = 0, where G projects a second-order
tensor field onto compatible ones; per wavevector G_{i a b j} = delta_ij g_ab
(Eq. original-G for the Fourier derivative, Eq. discrete_projection_op for a
discrete symbol: g_ab = D_a conj(D_b) / sum_c |D_c|^2 over the n_e * D
derivative indices a = (T, alpha) of a voxel; g = 0 where the symbol vanishes).

Solver (the paper cites gradient-based optimizers that keep F compatible; the
reading used here is the Newton-Krylov scheme of its ref. deGeus2017): Newton on
G P(F) = 0 with F = Fbar + F~, F~ compatible with zero mean.  Each Newton step
solves the linearised problem G (K(F) : dF) = -G P(F) for a compatible dF by
plain CG from dF = 0 (Euclidean inner product over all tensor components, equal
point weights, stop at ||r|| <= cg_tol ||r_0|| or at a breakdown p.q <= 0) and
sets F += dF.  Newton stops when the equilibrium residual is at
||G P(F)|| <= equil_tol ||P(F)|| before a step, or after a step with
||dF|| <= newton_tol ||F|| (Frobenius norms over the whole field); the first
test keeps CG from iterating on a right-hand side that is only rounding.
The right-hand side is projected twice (G is idempotent): a single application
leaves a rounding residue of order eps ||P|| outside the compatible subspace,
which stalls CG when ||G P|| is many orders below ||P||.  Load
steps move Fbar linearly from I in n_steps equal increments; each step first
adds the uniform increment of Fbar to F.

Material: the isotropic finite-strain linear elastic law (Saint
Venant-Kirchhoff) with per-voxel Lame constants: Green-Lagrange strain
E = 1/2 (F^T F - I), second Piola-Kirchhoff S = lambda tr(E) I + 2 mu E,
first Piola-Kirchhoff P = F S.  Its tangent applied to an increment X:
dP = X S + F (lambda tr(dE) I + 2 mu dE), dE = 1/2 (X^T F + F^T X).  lambda = mu
= 0 (vacuum) is allowed.

The plain definition the FE kind reaches: the canonical nonlinear FE problem on
the same mesh (2 triangles / 6 Kuhn tetrahedra per voxel), nodal residual
R(u) = sum_e |e| B_e^T P(Fbar + grad_e u) = 0, solved by Newton with the
assembled tangent sum_e |e| B_e^T K_e B_e and a sparse direct solve.

Array conventions: fields F[grid..., n_e, D, D] with F[..., i, a] =
d chi_i / d r_a; element order of fe.elements.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe, projection


# ---------------------------------------------------------------------------
# material
# ---------------------------------------------------------------------------
def _bc(lam, mu, F):
    """Broadcast per-voxel constants over the trailing (n_e, D, D) axes."""
    extra = F.ndim - np.ndim(lam)
    shape = np.shape(lam) + (1,) * extra
    return np.reshape(lam, shape), np.reshape(mu, shape)


def green_lagrange(F):
    D = F.shape[-1]
    return 0.5 * (np.swapaxes(F, -1, -2) @ F - np.eye(D))


def pk2(lam, mu, F):
    E = green_lagrange(F)
    D = F.shape[-1]
    lam_, mu_ = _bc(lam, mu, F)
    tr = np.trace(E, axis1=-2, axis2=-1)[..., None, None]
    return lam_ * tr * np.eye(D) + 2.0 * mu_ * E


def pk1(lam, mu, F):
    """First Piola-Kirchhoff stress P = F S."""
    return F @ pk2(lam, mu, F)


def energy(lam, mu, F):
    """Strain energy density W = 1/2 lambda tr(E)^2 + mu E:E (P = dW/dF)."""
    E = green_lagrange(F)
    lam_, mu_ = _bc(lam, mu, F)
    tr = np.trace(E, axis1=-2, axis2=-1)
    return 0.5 * lam_[..., 0, 0] * tr ** 2 + mu_[..., 0, 0] * np.sum(E * E, axis=(-2, -1))


def tangent_apply(lam, mu, F, X):
    """dP = K(F) : X."""
    D = F.shape[-1]
    lam_, mu_ = _bc(lam, mu, F)
    S = pk2(lam, mu, F)
    FtX = np.swapaxes(F, -1, -2) @ X
    dE = 0.5 * (FtX + np.swapaxes(FtX, -1, -2))
    tr = np.trace(dE, axis1=-2, axis2=-1)[..., None, None]
    dS = lam_ * tr * np.eye(D) + 2.0 * mu_ * dE
    return X @ S + F @ dS


def tangent_matrix(lam, mu, F):
    """K_iJkL = d P_iJ / d F_kL = delta_ik S_JL + lambda F_iJ F_kL
    + mu (F_iL F_kJ + (F F^T)_ik delta_JL), array [..., D, D, D, D]."""
    D = F.shape[-1]
    S = pk2(lam, mu, F)
    lam_, mu_ = _bc(lam, mu, F)
    lam_ = lam_[..., None, None]
    mu_ = mu_[..., None, None]
    I = np.eye(D)
    FFt = F @ np.swapaxes(F, -1, -2)
    K = (np.einsum("ik,...JL->...iJkL", I, S)
         + lam_ * np.einsum("...iJ,...kL->...iJkL", F, F)
         + mu_ * (np.einsum("...iL,...kJ->...iJkL", F, F) + np.einsum("...ik,JL->...iJkL", FFt, I)))
    return K


# ---------------------------------------------------------------------------
# gradient projection
# ---------------------------------------------------------------------------
def projector(kind, shape, h=None):
    """g_ab(k) over the n_e * D derivative indices: array (d, d, *grid)."""
    return projection.gradient_projection(projection.symbols(kind, shape, h))


def apply_gradient_projection(g, X):
    """(G X)_{T i a} = sum_{L b} g_{(T a)(L b)} X_{L i b} per wavevector, on a
    real field X[grid..., n_e, D, D]; FFT pair of the transform appendix, real
    part of the inverse."""
    grid = g.shape[2:]
    nd = len(grid)
    ne, D = X.shape[nd], X.shape[nd + 1]
    Xh = np.fft.fftn(X, axes=tuple(range(nd)))
    # (grid, T, i, a) -> (i, (T a), grid)
    Xr = np.moveaxis(Xh, nd + 1, 0)                       # (i, grid, T, a)
    Xr = Xr.reshape((D,) + grid + (ne * D,))
    Xr = np.moveaxis(Xr, -1, 1)                           # (i, (T a), grid)
    Y = np.einsum("ab...,ib...->ia...", g, Xr)
    Y = np.moveaxis(Y, 1, -1).reshape((D,) + grid + (ne, D))
    Y = np.moveaxis(Y, 0, nd + 1)                         # (grid, T, i, a)
    return np.fft.ifftn(Y, axes=tuple(range(nd))).real


# ---------------------------------------------------------------------------
# Newton + projected CG
# ---------------------------------------------------------------------------
def _cg(A, b, tol, maxit, floor=0.0):
    """CG on A x = b from x = 0, stopped at ||r|| <= tol ||b|| or at
    ||r|| <= floor, the rounding level of the stress b is projected from:
    below it the residual is noise, and iterating on it lets the zero-energy
    modes of a vacuum drift without bound."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.sum(r * r)
    rr0 = rr
    it = 0
    if rr0 == 0.0 or rr0 <= floor * floor:
        return x, 0
    while it < maxit:
        q = A(p)
        pq = np.sum(p * q)
        if not pq > 0.0:
            break  # breakdown at the rounding floor: keep the current iterate
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rr_new = np.sum(r * r)
        if np.sqrt(rr_new / rr0) <= tol or rr_new <= floor * floor:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it


def solve(lam, mu, Fbar, kind="fe", h=None, n_steps=1, newton_tol=1e-10, equil_tol=1e-11, cg_tol=1e-10,
          max_newton=50, maxit=5000, history=None):
    """Returns (F[grid..., n_e, D, D], newton iterations, total CG iterations).

    The Fourier derivatives ('fourier', 'fourier2') need odd grid sizes: the
    paper's Sec. "Even vs. odd number of grid points" shows that their
    projection is exact only there (the derivative is ambiguous at the Nyquist
    wavevector of an even axis), and Newton on the inexact one need not
    converge."""
    lam = np.asarray(lam, float)
    mu = np.asarray(mu, float)
    shape = lam.shape
    dim = len(shape)
    if kind in ("fourier", "fourier2") and any(n % 2 == 0 for n in shape):
        raise ValueError("finite strain with a Fourier derivative needs odd grid sizes")
    g = projector(kind, shape, h)
    ne = g.shape[0] // dim
    I = np.eye(dim)
    Fbar = np.asarray(Fbar, float)
    F = np.broadcast_to(I, shape + (ne, dim, dim)).copy()
    Fb_prev = I
    newton_its = cg_its = 0
    for s in range(1, n_steps + 1):
        Fb = I + (s / n_steps) * (Fbar - I)
        F += Fb - Fb_prev
        Fb_prev = Fb
        for _ in range(max_newton):
            P = pk1(lam, mu, F)
            b = -apply_gradient_projection(g, P)
            nb, nP = np.sqrt(np.sum(b * b)), np.sqrt(np.sum(P * P))
            # G is idempotent: projecting again removes the rounding residue
            # (relative to ||P||, outside the compatible subspace) that keeps
            # CG from converging once ||G P|| << ||P||
            b = apply_gradient_projection(g, b)
            if nb <= equil_tol * nP:
                break  # equilibrium reached (also for a stress-free state)
            Fc = F.copy()

            def A(x, Fc=Fc):
                return apply_gradient_projection(g, tangent_apply(lam, mu, Fc, x))

            dF, it = _cg(A, b, cg_tol, maxit, floor=64.0 * np.finfo(float).eps * nP)
            F += dF
            newton_its += 1
            cg_its += it
            nrm = np.sqrt(np.sum(dF * dF) / np.sum(F * F))
            if history is not None:
                history.append((s, it, float(nrm), float(nb / max(nP, 1e-300))))
            if nrm <= newton_tol:
                break
    return F, newton_its, cg_its


def mean_stress(lam, mu, F):
    """Volume average of P over the evaluation points (equal weights)."""
    P = pk1(np.asarray(lam, float), np.asarray(mu, float), F)
    nd = np.ndim(lam)
    return P.mean(axis=tuple(range(nd + 1)))


# ---------------------------------------------------------------------------
# canonical nonlinear FE (the plain definition for the FE kind)
# ---------------------------------------------------------------------------
def fe_solve(lam, mu, Fbar, h=None, tol=1e-12, max_newton=50, n_steps=1):
    """Newton on the assembled nodal residual; returns F[grid..., n_e, D, D]."""
    lam = np.asarray(lam, float)
    mu = np.asarray(mu, float)
    shape = lam.shape
    dim = len(shape)
    hh = fe._default_h(dim, h)
    N = lam.size
    els = fe.elements(dim, hh)
    nodes = [[fe._node_index(shape, v) for v in verts] for verts, _, _ in els]
    lamf, muf = lam.ravel(), mu.ravel()
    u = np.zeros((N, dim))
    I = np.eye(dim)
    Fbar = np.asarray(Fbar, float)

    def element_F(u, Fb):
        Fs = []
        for e, (verts, gr, vol) in enumerate(els):
            Fe = np.broadcast_to(Fb, (N, dim, dim)).copy()
            for c in range(dim + 1):
                Fe += u[nodes[e][c]][:, :, None] * gr[c][None, None, :]
            Fs.append(Fe)
        return Fs

    for s in range(1, n_steps + 1):
        Fb = I + (s / n_steps) * (Fbar - I)
        for _ in range(max_newton):
            Fs = element_F(u, Fb)
            R = np.zeros((N, dim))
            rows, cols, vals = [], [], []
            for e, (verts, gr, vol) in enumerate(els):
                P = pk1(lamf, muf, Fs[e])                      # (N, D, D)
                K = tangent_matrix(lamf, muf, Fs[e])           # (N, D, D, D, D)
                for c in range(dim + 1):
                    np.add.at(R, nodes[e][c], vol * P @ gr[c])
                    for d in range(dim + 1):
                        blk = vol * np.einsum("a,niakb,b->nik", gr[c], K, gr[d])
                        for i in range(dim):
                            for k in range(dim):
                                rows.append(nodes[e][c] * dim + i)
                                cols.append(nodes[e][d] * dim + k)
                                vals.append(blk[:, i, k])
            Kt = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(N * dim, N * dim)).tocsr()
            free = np.arange(dim, N * dim)
            du = np.zeros(N * dim)
            du[free] = spla.splu(Kt[free][:, free].tocsc()).solve(-R.ravel()[free])
            du = fe.remove_mean(du, dim).reshape(N, dim)
            u += du
            if np.linalg.norm(du) <= tol * max(1.0, np.linalg.norm(u)):
                break
    Fs = element_F(u, Fbar)
    return np.stack(Fs, axis=1).reshape(shape + (len(els), dim, dim))
