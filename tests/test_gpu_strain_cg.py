"""Strain-space projected CG with a choice of derivative (Sec. "Discrete
projection") on the GPU against the oracle's projected CG, element by element.

Both sides run CG from e~ = 0 to a relative residual of 1e-12 in FP64, so the
strain fields agree to the solve tolerance times the conditioning (bound used:
1e-8 of max |e|) and the iteration counts to within one.  Even grids for the
kinds whose symbol is Hermitian or whose Nyquist handling both sides share
(the real part of the complex result), odd grids for central differences and
least squares (their symbol vanishes at Nyquist indices on even grids, where
the kernels project the mode out and the oracle keeps a rounding-level
direction).  The FE kind is also checked against the factored
displacement-space solver (same canonical FE solution), and FP32 against the
FP64 oracle."""
import zlib

import numpy as np
import pytest

import microstructures as ms
from gpu_util import random_material, rel, say

pytestmark = pytest.mark.gpu


def _ebars(dim, L, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((L, dim, dim)) * 0.01
    return 0.5 * (A + np.swapaxes(A, 1, 2))


def _oracle(lam, mu, Ebars, kind, h=None):
    from oracle import pcg
    eps, its = [], []
    for Eb in Ebars:
        e, it, _ = pcg.solve(lam, mu, Eb, kind=kind, h=h, tol=1e-12)
        eps.append(pcg.flat_fields(e))
        its.append(it)
    return np.array(eps), its


def _energy(lam, mu, eps):
    """W_lm = mean over points of e_l : C : e_m (equal weights)."""
    L = eps.shape[0]
    lam = np.asarray(lam).ravel()[:, None]
    mu = np.asarray(mu).ravel()[:, None]
    tr = np.trace(eps, axis1=3, axis2=4)
    W = np.zeros((L, L))
    for l in range(L):
        for m in range(L):
            W[l, m] = np.mean(lam * tr[l] * tr[m] + 2 * mu * np.einsum("nejk,nejk->ne", eps[l], eps[m]))
    return W


CASES = [
    ("fe", (16, 12), None), ("fe", (9, 7), (1.0, 0.7)), ("fd", (16, 12), None), ("fd", (10, 9), (0.8, 1.3)),
    ("cd", (15, 13), None), ("ls", (15, 13), None), ("fourier", (16, 12), None), ("fourier", (15, 11), None),
    ("fourier2", (16, 12), None), ("fourier2", (9, 13), None),
    ("fe", (8, 6, 10), None), ("fd", (10, 8, 6), None), ("cd", (7, 9, 5), None), ("fourier", (8, 8, 6), None),
    ("fourier", (7, 5, 9), (1.0, 1.2, 0.9)),
    # smallest grids: axes of 2 and 3 points (single-butterfly transforms,
    # symbols that vanish on whole axes)
    ("fe", (2, 3), None), ("fd", (2, 2), None), ("cd", (2, 3), None), ("ls", (3, 2), None),
    ("fourier", (3, 3), None), ("fourier2", (3, 3), None), ("fe", (2, 2, 2), None), ("fd", (3, 2, 2), None),
    ("cd", (3, 3, 3), None),
    # even grids: central-difference and least-squares symbols vanish exactly
    # at Nyquist wavevectors
    ("cd", (8, 6), None), ("ls", (8, 6), None), ("cd", (6, 4, 8), None),
]


@pytest.mark.parametrize("kind,shape,h", CASES)
def test_strain_cg_matches_oracle(kind, shape, h):
    import torch
    from paper_2105_03297_amd import Homogenizer
    dim = len(shape)
    L = 3 if dim == 2 else 6
    say("strain_cg", kind, shape, h)
    lam, mu = random_material(shape, seed=zlib.crc32(repr((kind, shape)).encode()) % 1000)
    Eb = _ebars(dim, L, 5)
    hz = Homogenizer(shape, n_load=L, precision="fp64", h=h)
    hz.set_material(lam=lam, mu=mu)
    out = hz.strain_cg_solve(Eb, kind=kind, tol=1e-12, max_iter=2000, fields=True)
    torch.cuda.synchronize()
    ref, its = _oracle(lam, mu, Eb, kind, h)
    got = out["strain"].cpu().numpy()
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-8 * np.abs(ref).max())
    for l in range(L):
        assert out["report"][l]["status"] == 0
        assert abs(out["report"][l]["iterations"] - its[l]) <= 1, (out["report"][l], its[l])
    W = _energy(lam, mu, ref)
    np.testing.assert_allclose(out["energy"], W, rtol=0, atol=1e-9 * np.abs(W).max())
    lamf, muf = lam.ravel()[:, None, None, None], mu.ravel()[:, None, None, None]
    tr = np.trace(ref, axis1=3, axis2=4)[..., None, None]
    sig = lamf * tr * np.eye(dim) + 2 * muf * ref
    np.testing.assert_allclose(out["stress_mean"], sig.mean(axis=(1, 2)), rtol=0,
                               atol=1e-9 * np.abs(sig).max())
    hz.close()


@pytest.mark.parametrize("shape", [(64, 48), (24, 20, 16)])
def test_fe_strain_space_equals_factored_solver(shape):
    """Both solvers reach the canonical FE solution: same strain fields and
    effective stiffness."""
    import torch
    from paper_2105_03297_amd import Homogenizer
    dim = len(shape)
    say("strain_cg vs factored", shape)
    m = ms.voronoi(shape, 12, seed=31, E=(1.0, 20.0))
    from oracle import fe
    lam, mu = fe.lame(m.E, m.nu)
    loads = ms.unit_loads(dim)
    hz = Homogenizer(shape, n_load=len(loads), precision="fp64")
    hz.set_material(lam=lam, mu=mu)
    a = hz.solve(loads, tol=1e-12, max_iter=3000, fields=True)
    b = hz.strain_cg_solve(loads, kind="fe", tol=1e-12, max_iter=3000, fields=True)
    torch.cuda.synchronize()
    ea, eb = a["strain"].cpu().numpy(), b["strain"].cpu().numpy()
    np.testing.assert_allclose(eb, ea, rtol=0, atol=1e-8 * np.abs(ea).max())
    np.testing.assert_allclose(b["C_eff"], a["C_eff"], rtol=0, atol=1e-9 * np.abs(a["C_eff"]).max())
    hz.close()


@pytest.mark.parametrize("kind,shape", [("fe", (32, 24)), ("fourier", (33, 25)), ("fe", (12, 10, 8))])
def test_fp32_against_fp64_oracle(kind, shape):
    import torch
    from paper_2105_03297_amd import Homogenizer
    dim = len(shape)
    L = 3 if dim == 2 else 6
    say("strain_cg fp32", kind, shape)
    lam, mu = random_material(shape, seed=17, prec="fp32")
    Eb = _ebars(dim, L, 6)
    hz = Homogenizer(shape, n_load=L, precision="fp32")
    hz.set_material(lam=lam, mu=mu)
    out = hz.strain_cg_solve(Eb, kind=kind, tol=1e-6, max_iter=2000, fields=True)
    torch.cuda.synchronize()
    ref, _ = _oracle(lam, mu, Eb, kind)
    got = out["strain"].cpu().numpy().astype(np.float64)
    assert rel(got, ref) < 1e-4
    W = _energy(lam, mu, ref)
    assert rel(out["energy"], W) < 1e-6
    hz.close()


def test_uniform_material_and_edge_cases():
    """Uniform material: zero right-hand side (up to the rounding of the
    transforms), e = Ebar; max_iter = 1 reports FEH_ENOCONV with outputs;
    workspace too small, kinds outside their dimension and batched plans are
    rejected."""
    import torch
    import paper_2105_03297_amd as m
    from paper_2105_03297_amd import Homogenizer
    say("strain_cg edge cases")
    shape = (12, 10)
    hz = Homogenizer(shape, n_load=2, precision="fp64")
    hz.set_material(lam=np.full(shape, 2.0), mu=np.full(shape, 1.5))
    Eb = _ebars(2, 2, 8)
    for kind in ("fe", "fd", "fourier2"):
        out = hz.strain_cg_solve(Eb, kind=kind, tol=1e-10, fields=True)
        got = out["strain"].cpu().numpy()
        np.testing.assert_allclose(got, np.broadcast_to(Eb[:, None, None], got.shape), atol=1e-15)
        for l in range(2):
            s = 2.0 * np.trace(Eb[l]) * np.eye(2) + 3.0 * Eb[l]
            np.testing.assert_allclose(out["stress_mean"][l], s, atol=1e-15)
    # non-convergence within max_iter
    lam, mu = random_material(shape, seed=3)
    hz.set_material(lam=lam, mu=mu)
    out = hz.strain_cg_solve(Eb, kind="fe", tol=1e-14, max_iter=1, fields=False)
    assert out["status"] == m.FEH_ENOCONV
    assert all(r["iterations"] == 1 for r in out["report"])
    # workspace too small
    nbytes = m.feh_strain_cg_workspace_bytes(hz.plan, m.FEH_DERIV_FE)
    work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(m.FehError) as ei:
        m.feh_strain_cg_solve(hz.plan, m.FEH_DERIV_FE, Eb, 1e-8, 10, work.data_ptr(), nbytes - 256)
    assert ei.value.status == m.FEH_ENOMEM
    hz.close()
    h3 = Homogenizer((4, 4, 4), n_load=1, precision="fp64")
    with pytest.raises(m.FehError) as ei:
        m.feh_strain_cg_workspace_bytes(h3.plan, m.FEH_DERIV_LS)
    assert ei.value.status == m.FEH_ENOTSUP
    h3.close()
    hb = Homogenizer((8, 8), n_load=1, n_batch=2, precision="fp64")
    hb.set_material(lam=np.full((2, 8, 8), 1.0), mu=np.full((2, 8, 8), 1.0))
    with pytest.raises(m.FehError) as ei:
        hb.strain_cg_solve(_ebars(2, 2, 1), kind="fe")
    assert ei.value.status == m.FEH_EINVAL
    hb.close()


def test_spheres128_bench_configuration_equals_factored_solver():
    """The configuration the benchmark times (128^3 sphere packing, FE kind in
    strain space, FP32, 6 unit load cases, tol 1e-5), at full size where the
    oracle cannot follow: it reaches the FE solution of the factored solver on
    the same plan (C_eff and <sigma> to the FP32 solve accuracy), its energy
    matrix is symmetric, and <sigma> equals the energy form's columns
    (Hill-Mandel: <sigma_l> : Ebar_m = W_lm)."""
    import torch
    from paper_2105_03297_amd import Homogenizer
    say("strain_cg spheres128 bench configuration")
    m, Eb, _, _ = ms.workload("spheres128")
    lam = m.E * m.nu / ((1 + m.nu) * (1 - 2 * m.nu))
    mu = m.E / (2 * (1 + m.nu))
    hz = Homogenizer(m.shape, n_load=len(Eb), precision="fp32")
    hz.set_material(lam=lam, mu=mu)
    b = hz.strain_cg_solve(Eb, kind="fe", tol=1e-5, max_iter=5000)
    a = hz.solve(Eb, tol=1e-6, max_iter=5000)
    torch.cuda.synchronize()
    assert b["status"] == 0 and a["status"] == 0
    assert all(r["rel_residual"] <= 1e-5 for r in b["report"])
    scale = np.abs(a["C_eff"]).max()
    np.testing.assert_allclose(b["C_eff"], a["C_eff"], rtol=0, atol=2e-4 * scale)
    np.testing.assert_allclose(b["stress_mean"], a["stress_mean"], rtol=0,
                               atol=2e-4 * np.abs(a["stress_mean"]).max())
    W = b["energy"]
    np.testing.assert_allclose(W, W.T, rtol=0, atol=1e-5 * np.abs(W).max())
    HM = np.einsum("lij,mij->lm", b["stress_mean"], Eb)
    np.testing.assert_allclose(HM, W, rtol=0, atol=2e-4 * np.abs(W).max())
    hz.close()


@pytest.mark.parametrize("kind,shape,axis", [
    ("fd", (8, 6), 0), ("fd", (6, 4, 5), 2), ("cd", (9, 7), 0), ("cd", (5, 7, 3), 1),
    ("ls", (8, 6), 0), ("ls", (6, 8), 1), ("fourier", (7, 8), 1), ("fourier", (4, 5, 6), 0), ("fe", (8, 6), 0),
    ("fe", (4, 6, 5), 1),
])
@pytest.mark.parametrize("nus", [(0.3, 0.2), (0.0, 0.0)])
def test_laminate_closed_form(kind, shape, axis, nus):
    """Laminates (layers normal to `axis`) have the exact effective stiffness
    of the layered closed form with every discrete derivative (central
    differences on odd grids only: on an even axis their symbol vanishes at
    the Nyquist wavevector, which a layering of that axis needs); with nu = 0
    the loads along the layers have a zero right-hand side (the uniform
    strain is the solution), which must stop at once rather than iterate on
    rounding noise."""
    import torch
    from test_oracle_fe import _laminate_closed_form
    from test_oracle_pcg_kinds import _voigt_C
    from oracle import fe
    from paper_2105_03297_amd import Homogenizer
    say("strain_cg laminate", kind, shape, axis, nus)
    dim = len(shape)
    nl = 3 if shape[axis] > 5 else 2
    m = ms.laminate(shape, axis, nl, E=(1.0, 7.0), nu=nus)
    lam, mu = fe.lame(m.E, m.nu)
    Eb = ms.unit_loads(dim)
    hz = Homogenizer(shape, n_load=len(Eb), precision="fp64")
    hz.set_material(lam=lam, mu=mu)
    out = hz.strain_cg_solve(Eb, kind=kind, tol=1e-12, max_iter=2000)
    torch.cuda.synchronize()
    assert out["status"] == 0, [r for r in out["report"]]
    frac1 = nl / shape[axis]
    ref = _laminate_closed_form(_voigt_C(*fe.lame(7.0, nus[1]), dim), _voigt_C(*fe.lame(1.0, nus[0]), dim),
                                frac1, dim, axis)
    np.testing.assert_allclose(out["C_eff"], ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    hz.close()


@pytest.mark.parametrize("kind,shape,L", [("fe", (12, 10), 20), ("fd", (5, 4, 3), 9)])
def test_many_load_cases_match_oracle(kind, shape, L):
    """Many load cases in one strain-space solve: every strain field and the
    full energy matrix (L (L + 1) / 2 pair quantities) against the oracle."""
    import torch
    from paper_2105_03297_amd import Homogenizer
    say("strain_cg many load cases", kind, shape, L)
    dim = len(shape)
    lam, mu = random_material(shape, seed=44)
    Eb = _ebars(dim, L, 8)
    hz = Homogenizer(shape, n_load=L, precision="fp64")
    hz.set_material(lam=lam, mu=mu)
    out = hz.strain_cg_solve(Eb, kind=kind, tol=1e-12, max_iter=2000, fields=True)
    torch.cuda.synchronize()
    ref, its = _oracle(lam, mu, Eb, kind)
    got = out["strain"].cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-8 * np.abs(ref).max())
    W = _energy(lam, mu, ref)
    np.testing.assert_allclose(out["energy"], W, rtol=0, atol=1e-9 * np.abs(W).max())
    assert all(r["status"] == 0 for r in out["report"])
    hz.close()
