"""The remaining named configurations at their real sizes, and their recipes
at sizes the oracle solves completely.

  voronoi1024: 2D 1024^2 periodic Voronoi, 64 grains, two phases (contrast 100),
               3 load cases, FP64 at tol 1e-10 and FP32 at tol 1e-5.
  spheres128:  3D 128^3 random sequential addition of spheres (20 % volume,
               contrast 10), 6 load cases, FP32 at tol 1e-5 (FP64 at 1e-10 for
               the equilibrium check).

At full size the oracle cannot assemble the grid, so the checks use what it can
evaluate node by node or what holds at any size: the FE equilibrium
f - K u = 0 at sampled nodes for the returned displacement (local evaluation of
K and f), C_eff symmetric positive definite between the Reuss and Voigt bounds,
and FP32 against FP64 on the same input."""
import numpy as np
import pytest

import microstructures as ms
from gpu_util import rel, say

pytestmark = pytest.mark.gpu


def _voigt_C(lam, mu, dim):
    nv = 3 if dim == 2 else 6
    C = np.zeros(np.shape(lam) + (nv, nv))
    C[..., :dim, :dim] = np.asarray(lam)[..., None, None]
    for i in range(dim):
        C[..., i, i] += 2 * np.asarray(mu)
    for i in range(dim, nv):
        C[..., i, i] = mu
    return C


def _bounds(lam, mu, dim):
    """Voigt <C> and Reuss <C^-1>^-1 over the voxels (equal volumes)."""
    ul, il = np.unique(np.stack([np.ravel(lam), np.ravel(mu)], axis=1), axis=0, return_inverse=True)
    w = np.bincount(il.ravel()) / il.size
    Cs = _voigt_C(ul[:, 0], ul[:, 1], dim)
    Cv = np.tensordot(w, Cs, axes=1)
    Cr = np.linalg.inv(np.tensordot(w, np.linalg.inv(Cs), axes=1))
    return Cv, Cr


def _check_c(C, lam, mu, dim, tol=1e-9):
    np.testing.assert_allclose(C, C.T, rtol=0, atol=tol * np.abs(C).max())
    assert np.linalg.eigvalsh(C).min() > 0
    Cv, Cr = _bounds(lam, mu, dim)
    assert np.linalg.eigvalsh(Cv - C).min() > -tol * np.abs(C).max()
    assert np.linalg.eigvalsh(C - Cr).min() > -tol * np.abs(C).max()


def _equilibrium(lam, mu, Eb, u, n_samples=48, seed=0):
    """max over sampled nodes of |f - K u|, relative to the force scale
    max(lambda + 2 mu) max|Ebar| (local evaluation of K and f).  Half of the
    nodes are drawn next to material interfaces, where f does not vanish."""
    from oracle import fe
    N = lam.size
    rng = np.random.default_rng(seed)
    iface = np.zeros(lam.shape, bool)
    for ax in range(lam.ndim):
        for sh in (1, -1):
            iface |= np.roll(lam, sh, axis=ax) != lam
    iface = np.flatnonzero(iface.ravel())
    nodes = np.concatenate([rng.choice(N, n_samples // 2, replace=False),
                            rng.choice(iface, min(n_samples // 2, iface.size), replace=False), [0, N - 1]])
    scale = float((np.asarray(lam) + 2 * np.asarray(mu)).max() * np.abs(Eb).max())
    worst = 0.0
    for l in range(len(Eb)):
        f = fe.load_at_nodes(lam, mu, Eb[l], nodes)
        Ku = fe.apply_K_at_nodes(lam, mu, u[l], nodes)
        assert np.abs(f).max() > 1e-3 * scale  # the interface sample carries load
        worst = max(worst, float(np.abs(f - Ku).max() / scale))
    return worst


def _solve(shape, lam, mu, Eb, prec, tol, return_u=False):
    import paper_2105_03297_amd as feh
    h = feh.Homogenizer(shape, n_load=len(Eb), precision=prec)
    h.set_material(lam=lam, mu=mu)
    out = h.solve(Eb, tol=tol, max_iter=5000, return_u=return_u)
    if return_u:
        out["u"] = out["u"].double().cpu().numpy()
    h.close()
    return out


def _lame(m, prec):
    from oracle import fe
    lam, mu = fe.lame(m.E, m.nu)
    if prec == "fp32":
        lam = lam.astype(np.float32).astype(np.float64)
        mu = mu.astype(np.float32).astype(np.float64)
    return lam, mu


def test_voronoi1024_fullsize():
    say("voronoi1024 fp64 + fp32")
    m, Eb, tol, _ = ms.workload("voronoi1024")
    lam, mu = _lame(m, "fp64")
    o64 = _solve(m.shape, lam, mu, Eb, "fp64", tol, return_u=True)
    its = [r["iterations"] for r in o64["report"]]
    print("voronoi1024 fp64 iterations", its)
    assert o64["status"] == 0 and all(40 < i < 600 for i in its), its
    _check_c(o64["C_eff"], lam, mu, 2)
    eq = _equilibrium(lam, mu, Eb, o64["u"])
    print("equilibrium residual", eq)
    assert eq < 1e-6
    lam32, mu32 = _lame(m, "fp32")
    o32 = _solve(m.shape, lam32, mu32, Eb, "fp32", 1e-5)
    err = rel(o32["C_eff"], o64["C_eff"])
    print("voronoi1024 fp32 vs fp64", err, [r["iterations"] for r in o32["report"]])
    assert err < 1e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_voronoi_recipe_128_matches_oracle(prec):
    """The same recipe (64 grains, seed 1002, contrast 100) at 128^2 against
    the oracle's direct solve."""
    from oracle import fe
    say("voronoi recipe 128^2 vs oracle", prec)
    m = ms.voronoi((128, 128), 64, 1002)
    lam, mu = _lame(m, prec)
    Eb = ms.unit_loads(2)
    out = _solve(m.shape, lam, mu, Eb, prec, 1e-12 if prec == "fp64" else 1e-6)
    ref = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    err = rel(out["C_eff"], ref["C_eff"])
    print("C_eff rel err", err)
    assert err < (1e-10 if prec == "fp64" else 1e-5)


def test_spheres128_fullsize():
    say("spheres128 fp32 + fp64")
    m, Eb, tol, _ = ms.workload("spheres128")
    lam32, mu32 = _lame(m, "fp32")
    o32 = _solve(m.shape, lam32, mu32, Eb, "fp32", tol)
    its = [r["iterations"] for r in o32["report"]]
    print("spheres128 fp32 iterations", its)
    assert o32["status"] == 0 and all(10 < i < 200 for i in its), its
    _check_c(o32["C_eff"], lam32, mu32, 3, tol=1e-6)
    lam, mu = _lame(m, "fp64")
    o64 = _solve(m.shape, lam, mu, Eb, "fp64", 1e-10, return_u=True)
    eq = _equilibrium(lam, mu, Eb, o64["u"], n_samples=32)
    print("equilibrium residual", eq)
    assert eq < 1e-6
    err = rel(o32["C_eff"], o64["C_eff"])
    print("spheres128 fp32 vs fp64", err)
    assert err < 1e-5


def test_spheres_recipe_32_matches_oracle():
    """The sphere-packing recipe scaled to 32^3 (radii U[1, 2.5], 20 % volume)
    against the oracle's plain CG to 1e-13."""
    from oracle import fe
    say("spheres recipe 32^3 vs oracle")
    m = ms.rsa_spheres(32, 1003, (1.0, 2.5), 0.2)
    lam, mu = _lame(m, "fp64")
    Eb = ms.unit_loads(3)
    out = _solve(m.shape, lam, mu, Eb, "fp64", 1e-12)
    ref = fe.homogenize(None, None, Eb, method="ccg", tol=1e-13, lam_mu=(lam, mu))
    err = rel(out["C_eff"], ref["C_eff"])
    print("C_eff rel err", err)
    assert err < 1e-10
