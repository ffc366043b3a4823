"""Sensitivities of C_eff to the per-voxel material (adjoint row) through the
C ABI: parity with the oracle's formula on the oracle's fields, the
homogeneous closed form, Euler's identity at full size, and the autograd
gradient against central differences of GPU FP64 solves."""
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


def test_sensitivity_euler_identity_fullsize():
    """The benchmark recipe at 256^3 (FP32): sum_v E_v dJ/dE_v = J for
    J = trace C_eff (C_eff homogeneous of degree one in E)."""
    import torch
    say("sensitivity Euler identity 256^3 fp32")
    from paper_2105_03297_amd.autograd import lame_derivatives
    m = ms.grf_modulus((256, 256, 256), 16.0, 1004)
    E = torch.as_tensor(m.E.astype(np.float32))
    h = _hz((256, 256, 256), "fp32")
    h.set_material(E=E, nu=0.3)
    out = h.solve(ms.unit_loads(3), tol=1e-5, max_iter=2000)
    gl, gm = h.c_eff_sensitivity(np.eye(6))
    a, b = lame_derivatives(0.3)
    gE = (a * gl.double() + b * gm.double()).cpu().numpy()
    h.close()
    lhs = float(np.sum(m.E * gE))
    J = float(np.trace(out["C_eff"]))
    print("Euler:", lhs, J)
    assert abs(lhs - J) < 1e-5 * J


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
