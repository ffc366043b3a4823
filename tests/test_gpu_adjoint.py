"""Sensitivities of C_eff to the per-voxel material (adjoint row) through the
C ABI: parity with the oracle's formula on the oracle's fields, the
homogeneous closed form, the E-field entry point, the benchmark configuration
at 256^3 (the oracle's formula at sampled voxels, Euler's identity, central
differences of FP64 solves on 16 voxels), and the autograd gradient against
central differences of GPU FP64 solves."""
import numpy as np
import pytest

import microstructures as ms
from gpu_util import random_material, rel, say

pytestmark = pytest.mark.gpu


def _hz(shape, prec, L=None):
    import paper_2105_03297_amd as feh
    dim = len(shape)
    return feh.Homogenizer(shape, n_load=L or (3 if dim == 2 else 6), precision=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(14, 11), (7, 5, 6), (18, 4, 6)])
def test_sensitivity_matches_oracle(shape, prec):
    say("sensitivity vs oracle", shape, prec)
    from oracle import adjoint, fe
    dim = len(shape)
    lam, mu = random_material(shape, 21, prec)
    Eb = ms.unit_loads(dim)
    nv = len(Eb)
    G = np.random.default_rng(1).standard_normal((nv, nv))
    h = _hz(shape, prec)
    h.set_material(lam=lam, mu=mu)
    h.solve(Eb, tol=1e-12 if prec == "fp64" else 1e-6, max_iter=5000)
    gl, gm = (t.double().cpu().numpy().ravel() for t in h.c_eff_sensitivity(G))
    h.close()
    ref = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    rl, rm = adjoint.objective_gradient(ref["eps"], Eb, G)
    lim = 1e-9 if prec == "fp64" else 2e-4
    assert rel(gl, rl) < lim, rel(gl, rl)
    assert rel(gm, rm) < lim, rel(gm, rm)


@pytest.mark.parametrize("dim", [2, 3])
def test_sensitivity_homogeneous_closed_form(dim):
    say("sensitivity homogeneous", dim)
    from oracle import fe
    shape = (9, 7) if dim == 2 else (5, 4, 6)
    N = int(np.prod(shape))
    lam, mu = fe.lame(np.full(shape, 2.0), np.full(shape, 0.3))
    rng = np.random.default_rng(2)
    Eb = np.array([0.5 * (a + a.T) for a in rng.standard_normal((2, dim, dim))]) * 0.01
    h = _hz(shape, "fp64", L=2)
    h.set_material(lam=lam, mu=mu)
    h.solve(Eb, tol=1e-12)
    w = np.array([[1.0, 0.3], [-0.2, 2.0]])
    gl, gm = (t.cpu().numpy() for t in h.energy_sensitivity(w))
    h.close()
    el = sum(w[l, m] * np.trace(Eb[l]) * np.trace(Eb[m]) for l in range(2) for m in range(2)) / N
    em = sum(w[l, m] * 2 * np.sum(Eb[l] * Eb[m]) for l in range(2) for m in range(2)) / N
    np.testing.assert_allclose(gl, el, rtol=1e-12)
    np.testing.assert_allclose(gm, em, rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_sensitivity_E_entry_point(dim):
    """feh_energy_sensitivity_E (one kernel pass) equals the Lame pair combined
    with the plane-strain maps of the E-field setter, and refuses a material
    that was not set from an E field."""
    import torch
    import paper_2105_03297_amd as feh
    from oracle import adjoint
    say("sensitivity_E entry point", dim)
    shape = (13, 10) if dim == 2 else (7, 6, 9)
    nu = 0.27
    E = np.exp(np.random.default_rng(31).standard_normal(shape))
    h = _hz(shape, "fp64")
    h.set_material(E=torch.as_tensor(E), nu=nu)
    Eb = ms.unit_loads(dim)
    h.solve(Eb, tol=1e-12, max_iter=3000)
    G = np.random.default_rng(6).standard_normal((len(Eb), len(Eb)))
    W = feh.feh_effective_stiffness_weights(dim, Eb, G)
    gl, gm = (t.cpu().numpy() for t in h.energy_sensitivity(W))
    gE = h.energy_sensitivity_E(W).cpu().numpy()
    ref = adjoint.e_gradient(gl, gm, nu)
    assert rel(gE, ref) < 1e-14, rel(gE, ref)
    h.set_material(lam=E * nu / ((1 + nu) * (1 - 2 * nu)), mu=E / (2 * (1 + nu)))
    h.solve(Eb, tol=1e-12, max_iter=3000)
    with pytest.raises(feh.FehError) as ei:
        h.energy_sensitivity_E(W)
    assert ei.value.status == feh.FEH_EINVAL
    h.close()


def _sample_voxels(E, n_random, n_steep, seed):
    """Seeded random voxels plus the voxels where E changes most to a neighbour."""
    N = E.size
    steep = np.zeros(E.shape)
    for ax in range(E.ndim):
        steep = np.maximum(steep, np.abs(np.roll(E, -1, axis=ax) - E))
    top = np.argpartition(steep.ravel(), -n_steep)[-n_steep:]
    rnd = np.random.default_rng(seed).choice(N, n_random, replace=False)
    return np.unique(np.concatenate([rnd, top, [0, N - 1]]))


def test_sensitivity_fullsize_sampled_voxels_and_euler():
    """The benchmark configuration (256^3, E = exp(GRF), 6 load cases, FP32):
    dJ/dE_v of J = trace C_eff from feh_energy_sensitivity_E at 66 sampled
    voxels (32 seeded, 32 at the steepest changes of E, the first and last)
    against the oracle's formula evaluated from the GPU's own fluctuations at
    those voxels (local strains, FP64), element by element; and Euler's
    identity sum_v E_v dJ/dE_v = J over the whole grid (C_eff is homogeneous
    of degree one in E)."""
    import torch
    import paper_2105_03297_amd as feh
    from oracle import adjoint, fe
    say("sensitivity 256^3 fp32: sampled voxels vs oracle formula, Euler identity")
    shape = (256, 256, 256)
    N = int(np.prod(shape))
    m = ms.grf_modulus(shape, 16.0, 1004)
    E32 = m.E.astype(np.float32)
    h = _hz(shape, "fp32")
    h.set_material(E=torch.as_tensor(E32), nu=0.3)
    Eb = ms.unit_loads(3)
    out = h.solve(Eb, tol=1e-5, max_iter=2000, return_u=True)
    W = feh.feh_effective_stiffness_weights(3, Eb, np.eye(6))
    gE = h.energy_sensitivity_E(W).double().cpu().numpy().ravel()
    vox = _sample_voxels(E32.astype(np.float64), 32, 32, 2004)
    eps_sub = []
    for l in range(6):
        ul = out["u"][l].double().cpu().numpy()
        eps_sub.append(fe.element_strains_at(ul, shape, vox, Eb[l]))
    h.close()
    gl, gm = adjoint.objective_gradient(eps_sub, Eb, np.eye(6), n_voxels=N)
    ref = adjoint.e_gradient(gl, gm, 0.3)
    got = gE[vox]
    err = np.abs(got - ref) / np.abs(ref)
    print("sampled dJ/dE_v: max rel err per voxel %.3e, rel to max %.3e" % (err.max(), rel(got, ref)))
    assert rel(got, ref) < 1e-6 and err.max() < 1e-5
    lhs = float(np.sum(E32.astype(np.float64).ravel() * gE))
    J = float(np.trace(out["C_eff"]))
    print("Euler:", lhs, J)
    assert abs(lhs - J) < 1e-5 * J


@pytest.mark.timeout(900)
def test_sensitivity_fullsize_central_differences():
    """The benchmark recipe at 256^3 solved in FP64: dJ/dE_v of
    J = sum diag C_eff (feh_energy_sensitivity_E) against central differences
    on the 16 voxels drawn with seed 2004 (relative step 1e-2; each perturbed
    solve warm-started from the converged field, tol 1e-9: the energy form of
    C_eff is second order in the residual, so its solve error is far below the
    differences)."""
    import torch
    import paper_2105_03297_amd as feh
    say("sensitivity 256^3 fp64 vs central differences on 16 voxels")
    shape = (256, 256, 256)
    N = int(np.prod(shape))
    m = ms.grf_modulus(shape, 16.0, 1004)
    Eb = ms.unit_loads(3)
    h = _hz(shape, "fp64")
    Ed = torch.as_tensor(m.E, dtype=torch.float64, device="cuda")
    h.set_material(E=Ed, nu=0.3)
    base = h.solve(Eb, tol=1e-10, max_iter=5000, return_u=True)
    u0 = base["u"]
    W = feh.feh_effective_stiffness_weights(3, Eb, np.eye(6))
    gE = h.energy_sensitivity_E(W).cpu().numpy().ravel()
    vox = np.random.default_rng(2004).choice(N, 16, replace=False)
    Ef = Ed.view(-1)
    errs = []
    for v in vox:
        step = 1e-2 * float(m.E.ravel()[v])
        Js = []
        for sgn in (1.0, -1.0):
            Ef[v] = float(m.E.ravel()[v]) + sgn * step
            h.set_material(E=Ed, nu=0.3)
            o = h.solve(Eb, tol=1e-9, max_iter=5000, u0=u0)
            assert o["status"] == 0
            Js.append(float(np.trace(o["C_eff"])))
        Ef[v] = float(m.E.ravel()[v])
        fd = (Js[0] - Js[1]) / (2 * step)
        errs.append(abs(gE[v] - fd) / abs(fd))
        print("voxel", int(v), "adjoint", gE[v], "central difference", fd, "rel err", errs[-1], flush=True)
    h.close()
    print("max rel err over 16 voxels: %.3e" % max(errs))
    assert max(errs) < 1e-4


def test_autograd_matches_central_differences():
    """Autograd gradient of J = sum diag C_eff for the E = exp(GRF) recipe at
    24^3 (FP64, tol 1e-12) against central differences (step 1e-3 E_v) on 16
    voxels drawn with seed 2004."""
    import torch
    say("autograd vs central differences 24^3 fp64")
    from paper_2105_03297_amd.autograd import EffectiveStiffness
    n = 24
    m = ms.grf_modulus((n, n, n), 16.0 * n / 256.0, 1004)
    E = torch.as_tensor(m.E, dtype=torch.float64, device="cuda").requires_grad_(True)
    h = _hz((n, n, n), "fp64")
    C = EffectiveStiffness.apply(E, 0.3, h, 1e-12, 5000)
    J = torch.trace(C)
    J.backward()
    g = E.grad.cpu().numpy().ravel()
    vox = np.random.default_rng(2004).choice(n ** 3, 16, replace=False)
    Ef = m.E.ravel()
    for v in vox:
        step = 1e-3 * Ef[v]
        Js = []
        for sgn in (1.0, -1.0):
            Ep = Ef.copy()
            Ep[v] += sgn * step
            with torch.no_grad():
                Cp = EffectiveStiffness.apply(torch.as_tensor(Ep.reshape(m.E.shape), device="cuda"), 0.3, h, 1e-12, 5000)
            Js.append(float(torch.trace(Cp)))
        fd = (Js[0] - Js[1]) / (2 * step)
        assert abs(g[v] - fd) <= 1e-5 * abs(fd), (int(v), g[v], fd)
    h.close()
