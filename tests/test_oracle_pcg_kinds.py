"""Pins of the oracle's strain-space projected CG for the derivative kinds
other than linear finite elements (Sec. "Discrete projection": forward and
central differences, least squares, the Fourier derivative and the two-point
Fourier derivative).  The FE kind is pinned against the canonical FE solve in
test_oracle_fe.

  * Laminates (material varying along one axis): every field that depends on
    that axis only and has the right mean is compatible for a derivative whose
    symbol does not vanish on that axis (k != 0), so equilibrium makes the
    normal stress and the shear tractions uniform and C_eff equals the
    laminate closed form exactly (Reuss across, Voigt along for nu = 0).
  * Hill-Mandel at convergence: G(C : e) = 0 makes the stress orthogonal to
    every compatible fluctuation, so <e_l : C : e_m> = Ebar_l : <sigma_m>.
  * C_eff symmetric positive definite between the Reuss and Voigt bounds.
  * Uniform material: the right-hand side vanishes, e = Ebar.
"""
import numpy as np
import pytest

import microstructures as ms
from oracle import fe, pcg, projection

KINDS_2D = ["fd", "cd", "ls", "fourier", "fourier2"]


def _voigt_C(lam, mu, dim):
    nv = 3 if dim == 2 else 6
    C = np.zeros((nv, nv))
    C[:dim, :dim] = lam
    C[np.arange(dim), np.arange(dim)] += 2 * mu
    C[np.arange(dim, nv), np.arange(dim, nv)] = mu
    return C


def _solve_all(lam, mu, Ebars, kind, tol=1e-13):
    """Strain fields (N, n_e, D, D), stress means and energy matrix (equal
    weights per evaluation point)."""
    eps, smean = [], []
    for Eb in Ebars:
        e, it, _ = pcg.solve(lam, mu, Eb, kind=kind, tol=tol)
        eps.append(pcg.flat_fields(e))
        s = pcg.flat_fields(pcg.stress_field(lam, mu, e))
        smean.append(s.mean(axis=(0, 1)))
    L = len(Ebars)
    W = np.zeros((L, L))
    for l in range(L):
        s = pcg.flat_fields(pcg.stress_field(lam, mu, eps[l].reshape(lam.shape + eps[l].shape[1:])))
        for m in range(L):
            W[l, m] = np.einsum("neij,neij->", s, eps[m]) / (s.shape[0] * s.shape[1])
    return eps, np.array(smean), W


@pytest.mark.parametrize("kind,shape,axis", [
    ("fd", (8, 6), 0), ("fd", (6, 8), 1), ("fd", (6, 4, 5), 2),
    ("cd", (9, 7), 0), ("cd", (7, 9), 1), ("cd", (5, 7, 3), 1),
    ("ls", (8, 6), 0), ("ls", (6, 8), 1),
    ("fourier", (8, 6), 0), ("fourier", (7, 8), 1), ("fourier", (4, 5, 6), 0),
])
@pytest.mark.parametrize("nus", [(0.3, 0.2), (0.0, 0.0)])
def test_laminate_closed_form(kind, shape, axis, nus):
    dim = len(shape)
    nl = 3 if shape[axis] > 5 else 2
    m = ms.laminate(shape, axis, nl, E=(1.0, 7.0), nu=nus)
    lam, mu = fe.lame(m.E, m.nu)
    Ebars = ms.unit_loads(dim)
    _, smean, W = _solve_all(lam, mu, Ebars, kind)
    frac1 = nl / shape[axis]
    lam1, mu1 = fe.lame(7.0, nus[1])
    lam2, mu2 = fe.lame(1.0, nus[0])
    from test_oracle_fe import _laminate_closed_form
    ref = _laminate_closed_form(_voigt_C(lam1, mu1, dim), _voigt_C(lam2, mu2, dim), frac1, dim, axis)
    np.testing.assert_allclose(fe.c_eff_energy(W, Ebars), ref, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(fe.c_eff_stress(smean, Ebars), ref, atol=1e-11 * np.abs(ref).max())
    if nus == (0.0, 0.0):
        reuss = 1 / (frac1 / 7.0 + (1 - frac1) / 1.0)
        C = fe.c_eff_stress(smean, Ebars)
        assert C[axis, axis] == pytest.approx(reuss, rel=1e-11)


@pytest.mark.parametrize("kind", KINDS_2D + ["fe"])
def test_hill_mandel_bounds_symmetry(kind):
    # odd grids for the kinds whose symbol is not Hermitian at Nyquist
    # indices (Fourier: the real part of G there is the mean of two
    # projections, no longer idempotent) or vanishes there (cd, ls)
    shape = (8, 6) if kind in ("fd", "fe") else (9, 7)
    rng = np.random.default_rng(21)
    E = rng.uniform(1.0, 10.0, shape)
    nu = rng.uniform(0.1, 0.4, shape)
    lam, mu = fe.lame(E, nu)
    Ebars = ms.unit_loads(2)
    eps, smean, W = _solve_all(lam, mu, Ebars, kind)
    for l in range(3):
        for j in range(3):
            assert W[l, j] == pytest.approx(np.sum(Ebars[l] * smean[j]), rel=1e-9, abs=1e-12 * np.abs(W).max())
    C = fe.c_eff_energy(W, Ebars)
    np.testing.assert_allclose(C, C.T, atol=1e-10 * np.abs(C).max())
    Cs = [_voigt_C(a, b, 2) for a, b in zip(lam.ravel(), mu.ravel())]
    Cv = np.mean(Cs, axis=0)
    Cr = np.linalg.inv(np.mean([np.linalg.inv(c) for c in Cs], axis=0))
    assert np.linalg.eigvalsh(C).min() > 0
    assert np.linalg.eigvalsh(Cv - C).min() > -1e-10
    assert np.linalg.eigvalsh(C - Cr).min() > -1e-10
    # the fluctuation has zero mean and is compatible: G e~ = e~
    Dh = projection.symbols(kind, shape)
    G = projection.small_strain_operator(Dh)
    ef = eps[0].reshape(shape + eps[0].shape[1:]) - Ebars[0]
    np.testing.assert_allclose(ef.mean(axis=(0, 1)), 0.0, atol=1e-14)
    np.testing.assert_allclose(projection.apply_small_strain(G, ef), ef, atol=1e-12)


@pytest.mark.parametrize("kind", KINDS_2D)
def test_uniform_material_exact(kind):
    shape = (7, 6)
    lam, mu = fe.lame(np.full(shape, 3.0), np.full(shape, 0.25))
    Eb = np.array([[0.01, 0.003], [0.003, -0.02]])
    e, it, _ = pcg.solve(lam, mu, Eb, kind=kind, tol=1e-12)
    # the right-hand side is zero up to rounding of the transforms
    np.testing.assert_allclose(e, np.broadcast_to(Eb, e.shape), atol=1e-15)
