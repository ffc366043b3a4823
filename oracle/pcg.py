"""The paper's projected conjugate gradients in strain space, FP64, CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. "Compatibility projection" poses equilibrium as G * (C : e) = 0 for a
strain field e = Ebar + e~ whose fluctuation e~ is compatible, and notes that
gradient-based solvers started from a compatible field stay compatible.  The
paper does not spell the solver out; the reading used here is plain conjugate
gradients on the compatible subspace with the Euclidean (Frobenius, equal
element weights) inner product:

    A e~ = G(C : e~),  b = -G(C : Ebar),  e~_0 = 0,

with G the small-strain projection of the small-strain appendix applied per
wavevector through the FFT (oracle.projection).  Stops when
||r_k|| <= tol ||r_0||.
"""
from __future__ import annotations

import numpy as np

from . import fe, projection


def _stress(lam, mu, e):
    # e[grid..., n_e, D, D]; lam, mu per voxel (grid)
    D = e.shape[-1]
    tr = np.trace(e, axis1=-2, axis2=-1)
    lam = lam[..., None, None, None]
    mu = mu[..., None, None, None]
    return lam * tr[..., None, None] * np.eye(D) + 2.0 * mu * e


def solve(lam, mu, Ebar, kind="fe", h=None, tol=1e-12, maxit=5000):
    """Returns (strain field e[grid..., n_e, D, D], iterations, residual history)."""
    lam = np.asarray(lam, float)
    mu = np.asarray(mu, float)
    shape = lam.shape
    dim = len(shape)
    Dhat = projection.symbols(kind, shape, h)
    G = projection.small_strain_operator(Dhat)
    ne = Dhat.shape[0]
    Eb = np.broadcast_to(np.asarray(Ebar, float), shape + (ne, dim, dim))

    def A(x):
        return projection.apply_small_strain(G, _stress(lam, mu, x))

    x = np.zeros(shape + (ne, dim, dim))
    r = -A(Eb)
    p = r.copy()
    rr = np.sum(r * r)
    rr0 = rr
    hist = [1.0]
    it = 0
    # The projected right-hand side -G sigma(Ebar) is computed from sigma(Ebar);
    # at or below that evaluation's rounding level (64 eps |sigma(Ebar)|) it is
    # zero, and so is the fluctuation.  The relative stop alone would iterate
    # on rounding noise, whose CG recurrences lose all accuracy.
    floor2 = (64.0 * np.finfo(float).eps) ** 2 * np.sum(_stress(lam, mu, Eb) ** 2)
    if rr0 <= floor2:
        return Eb + x, 0, hist
    while it < maxit:
        Ap = A(p)
        alpha = rr / np.sum(p * Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        rr_new = np.sum(r * r)
        hist.append(float(np.sqrt(rr_new / rr0)))
        if np.sqrt(rr_new / rr0) <= tol or rr_new <= floor2:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return Eb + x, it, hist


def flat_fields(e):
    """Reshape a grid-shaped element field to (N, n_e, D, D) (fe layout)."""
    D = e.shape[-1]
    ne = e.shape[-3]
    return e.reshape(-1, ne, D, D)


def stress_field(lam, mu, e):
    return _stress(np.asarray(lam, float), np.asarray(mu, float), e)


def average_stress(lam, mu, e):
    s = flat_fields(stress_field(lam, mu, e))
    return fe.average(s, e.shape[-1])
