"""Pins of the sensitivity oracle: central finite differences of the direct
FE solve, Euler's identity for degree-one homogeneity, and the uniform-strain
closed form of a homogeneous cell."""
import numpy as np
import pytest

import microstructures as ms
from oracle import adjoint, fe


def _material(shape, seed):
    rng = np.random.default_rng(seed)
    E = np.exp(rng.standard_normal(shape))
    nu = 0.2 + 0.15 * rng.random(shape)
    return fe.lame(E, nu)


def _c_eff(lam, mu, Eb):
    return fe.homogenize(None, None, Eb, lam_mu=(lam, mu))["C_eff"]


@pytest.mark.parametrize("shape", [(6, 5), (3, 4, 3)])
def test_lame_sensitivity_matches_central_differences(shape):
    """dC_eff/dlambda_v, dC_eff/dmu_v of the direct FE solve by central
    differences (relative step 1e-4) on three voxels, every C_eff entry."""
    dim = len(shape)
    lam, mu = _material(shape, 3)
    Eb = ms.unit_loads(dim)
    out = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    nv = out["C_eff"].shape[0]
    N = lam.size
    for v in (0, N // 2 + 1, N - 1):
        for which in ("lam", "mu"):
            fd = np.zeros((nv, nv))
            base = lam if which == "lam" else mu
            step = 1e-4 * base.ravel()[v]
            for sgn in (1.0, -1.0):
                b = base.copy().ravel()
                b[v] += sgn * step
                b = b.reshape(shape)
                C = _c_eff(b, mu, Eb) if which == "lam" else _c_eff(lam, b, Eb)
                fd += sgn * C / (2.0 * step)
            for I in range(nv):
                for J in range(nv):
                    G = np.zeros((nv, nv))
                    G[I, J] = 1.0
                    gl, gm = adjoint.objective_gradient(out["eps"], Eb, G)
                    an = (gl if which == "lam" else gm)[v]
                    assert abs(an - fd[I, J]) <= 1e-7 * np.abs(fd).max() + 1e-13, (v, which, I, J, an, fd[I, J])


def test_e_sensitivity_matches_central_differences():
    """dJ/dE_v with a uniform Poisson ratio, J = sum of the diagonal of C_eff."""
    shape = (5, 4, 3)
    rng = np.random.default_rng(5)
    E = np.exp(rng.standard_normal(shape))
    nu = 0.3
    Eb = ms.unit_loads(3)
    out = fe.homogenize(E, np.full(shape, nu), Eb)
    G = np.eye(6)
    gE = adjoint.e_gradient(*adjoint.objective_gradient(out["eps"], Eb, G), nu)
    for v in (1, 17, 59):
        h = 1e-4 * E.ravel()[v]
        Jp, Jm = [], []
        for sgn, acc in ((1, Jp), (-1, Jm)):
            Ev = E.copy().ravel()
            Ev[v] += sgn * h
            acc.append(np.trace(fe.homogenize(Ev.reshape(shape), np.full(shape, nu), Eb)["C_eff"]))
        fd = (Jp[0] - Jm[0]) / (2 * h)
        assert abs(gE[v] - fd) <= 1e-7 * abs(fd), (v, gE[v], fd)


@pytest.mark.parametrize("shape", [(7, 6), (4, 3, 5)])
def test_euler_identity(shape):
    """C_eff is homogeneous of degree one in (lambda, mu) jointly (scaling the
    material scales every stress, not the strains), so
    sum_v lambda_v dW/dlambda_v + mu_v dW/dmu_v = W for every load pair."""
    dim = len(shape)
    lam, mu = _material(shape, 7)
    Eb = ms.unit_loads(dim)
    Eb[0] += 0.004 * np.eye(dim)[::-1] * 0.5  # a load with off-diagonal coupling
    Eb[0] = 0.5 * (Eb[0] + Eb[0].T)
    out = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    dl, dm = adjoint.energy_sensitivity(out["eps"])
    lhs = np.einsum("lmn,n->lm", dl, lam.ravel()) + np.einsum("lmn,n->lm", dm, mu.ravel())
    np.testing.assert_allclose(lhs, out["W"], rtol=1e-12, atol=1e-15 * np.abs(out["W"]).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneous_closed_form(dim):
    """Uniform material: e_l = Ebar_l in every element, so
    dW_lm/dlambda_v = tr Ebar_l tr Ebar_m / N and dW_lm/dmu_v = 2 Ebar_l : Ebar_m / N."""
    shape = (5, 4) if dim == 2 else (3, 4, 2)
    N = int(np.prod(shape))
    lam, mu = fe.lame(np.full(shape, 2.0), np.full(shape, 0.3))
    rng = np.random.default_rng(2)
    Eb = np.array([0.5 * (a + a.T) for a in rng.standard_normal((3, dim, dim))]) * 0.01
    out = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    dl, dm = adjoint.energy_sensitivity(out["eps"])
    for l in range(3):
        for m in range(3):
            np.testing.assert_allclose(dl[l, m], np.trace(Eb[l]) * np.trace(Eb[m]) / N, rtol=1e-12, atol=1e-20)
            np.testing.assert_allclose(dm[l, m], 2 * np.sum(Eb[l] * Eb[m]) / N, rtol=1e-12, atol=1e-20)


def test_objective_weights_diagonal_loads():
    """Unit Voigt loads: E is diagonal (0.01, ..., engineering shear 0.02), so
    E^-1 G E^-T keeps the sparsity of G."""
    Eb = ms.unit_loads(3)
    G = np.zeros((6, 6))
    G[0, 0] = 1.0
    G[4, 4] = 2.0
    Wt = adjoint.objective_weights(Eb, G)
    expect = np.zeros((6, 6))
    expect[0, 0] = 1.0 / 0.01 ** 2
    expect[4, 4] = 2.0 / 0.02 ** 2
    np.testing.assert_allclose(Wt, expect, rtol=1e-13)


def test_gradient_on_voxel_subset_equals_full():
    """The sensitivity formula evaluated from locally computed strains of a
    voxel subset (grids too large for whole fields) equals the full-field
    result at those voxels."""
    shape = (5, 4, 3)
    lam, mu = _material(shape, 8)
    Eb = ms.unit_loads(3)
    out = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    G = np.random.default_rng(4).standard_normal((6, 6))
    gl, gm = adjoint.objective_gradient(out["eps"], Eb, G)
    N = lam.size
    vox = np.array([0, 7, 31, N - 1])
    u = [x.reshape(-1) for x in out["u"]]
    eps_sub = [fe.element_strains_at(u[l], shape, vox, Eb[l]) for l in range(6)]
    sl, sm = adjoint.objective_gradient(eps_sub, Eb, G, n_voxels=N)
    np.testing.assert_allclose(sl, gl[vox], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(sm, gm[vox], rtol=1e-13, atol=1e-16)
