"""GPU solve parity through the C ABI against the CPU FP64 oracle (canonical
FE direct / plain-CG solve), plus the method's exact special cases.

Tolerances (relative, max-abs over max-abs): FP64 <= 1e-10 on C_eff and
<sigma> at tol 1e-12; FP32-bulk/FP64-scalar <= 1e-5 on C_eff."""
import numpy as np
import pytest

import microstructures as ms
from gpu_util import random_material, rel, say

pytestmark = pytest.mark.gpu


def _solve(shape, lam, mu, Ebars, prec, tol, fields=False, return_u=False, max_iter=2000, h=None, u0=None):
    import paper_2105_03297_amd as feh
    hz = feh.Homogenizer(shape, n_load=len(Ebars), precision=prec, h=h)
    hz.set_material(lam=lam, mu=mu)
    out = hz.solve(Ebars, tol=tol, max_iter=max_iter, fields=fields, return_u=return_u, u0=u0)
    for k in ("u", "strain", "stress"):
        if out[k] is not None:
            out[k] = out[k].cpu().numpy().astype(np.float64)
    hz.close()
    return out


def test_circle32_fp64_matches_oracle():
    say("circle32 fp64")
    from oracle import fe
    m, _, _, _ = ms.workload("circle32")
    lam, mu = fe.lame(m.E, m.nu)
    Eb = ms.unit_loads(2)
    out = _solve(m.shape, lam, mu, Eb, "fp64", 1e-12, fields=True, return_u=True)
    ref = fe.homogenize(m.E, m.nu, Eb)
    assert out["status"] == 0
    assert rel(out["C_eff"], ref["C_eff"]) < 1e-10
    errs = {k: max(rel(out[k][l], ref[r][l]) for l in range(3))
            for k, r in (("stress_mean", "sig_mean"), ("strain", "eps"), ("stress", "sig"), ("u", "u"))}
    print("circle32 fp64 tol 1e-12, max rel err over the load cases:", errs)
    for k, e in errs.items():
        assert e < 1e-10, (k, e)
    np.testing.assert_allclose(out["energy"], out["energy"].T, rtol=0, atol=1e-15)


def test_circle32_iterations_at_paper_tolerance():
    """rel residual 1e-10 in FP64: about 40-45 iterations, C_eff already at
    rounding level (energy form is second order in the residual)."""
    say("circle32 tol 1e-10")
    from oracle import fe
    m, Eb, tol, _ = ms.workload("circle32")
    lam, mu = fe.lame(m.E, m.nu)
    out = _solve(m.shape, lam, mu, Eb, "fp64", tol)
    it = out["report"][0]["iterations"]
    assert 30 <= it <= 55, it
    assert out["report"][0]["rel_residual"] <= tol
    ref = fe.homogenize(m.E, m.nu, Eb)
    e = rel(out["stress_mean"][0], ref["sig_mean"][0])
    print("circle32 fp64 tol 1e-10: <sigma> rel err %.3e" % e)
    assert e < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(24, 20), (9, 300), (6, 5, 7), (10, 8, 70), (18, 4, 6),
                                   (17, 17), (151, 34), (17, 6, 5)])
def test_random_material_matches_oracle(shape, prec):
    say("random material", shape, prec)
    from oracle import fe
    dim = len(shape)
    lam, mu = random_material(shape, 11, prec)
    Eb = ms.unit_loads(dim)
    hvox = (1.0, 1.2, 0.9)[:dim]
    tol = 1e-12 if prec == "fp64" else 1e-6
    out = _solve(shape, lam, mu, Eb, prec, tol, h=hvox)
    ref = fe.homogenize(None, None, Eb, h=hvox, lam_mu=(lam, mu))
    lim = 1e-10 if prec == "fp64" else 1e-5
    assert rel(out["C_eff"], ref["C_eff"]) < lim
    for l in range(len(Eb)):
        assert rel(out["stress_mean"][l], ref["sig_mean"][l]) < (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("shape,prec", [((2048, 16), "fp64"), ((3072, 16), "fp32"),
                                        ((1365, 3, 2), "fp64"), ((2048, 2, 3), "fp32")])
def test_longest_first_axis_matches_oracle(shape, prec):
    """The longest first axis whose pencils fill one workgroup's LDS tile
    (one pencil block of all D components): the fused first-axis pass at its
    largest LDS footprint, against the direct solve."""
    say("longest first axis", shape, prec)
    from oracle import fe
    dim = len(shape)
    lam, mu = random_material(shape, 11, prec)
    Eb = ms.unit_loads(dim)
    tol = 1e-12 if prec == "fp64" else 1e-6
    out = _solve(shape, lam, mu, Eb, prec, tol, max_iter=5000)
    assert out["status"] == 0
    ref = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    assert rel(out["C_eff"], ref["C_eff"]) < (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("shape", [(2, 2), (2, 3), (3, 2), (2, 2, 2), (3, 2, 2), (2, 5, 2), (2, 2, 3)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_smallest_grids_match_oracle(shape, prec):
    """Grids with axes of 2 or 3 voxels: every periodic neighbour wraps, the
    stencil tiles and halos cover the cell several times over and the FFTs are
    a single butterfly.  The solve matches the direct solve."""
    say("smallest grid", shape, prec)
    from oracle import fe
    dim = len(shape)
    lam, mu = random_material(shape, 21, prec)
    Eb = ms.unit_loads(dim)
    tol = 1e-12 if prec == "fp64" else 1e-6
    out = _solve(shape, lam, mu, Eb, prec, tol, max_iter=500)
    assert out["status"] == 0
    ref = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    assert rel(out["C_eff"], ref["C_eff"]) < (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("shape,L", [((20, 16), 64), ((6, 5, 4), 13)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_many_load_cases_match_oracle(shape, L, prec):
    """Up to the plan's maximum of 64 load cases in one batched solve: every
    load case's <sigma> and the full energy matrix W_lm = <e_l : C : e_m>
    (L (L + 1) / 2 pair quantities in the post pass) against the direct
    solve."""
    say("many load cases", shape, L, prec)
    from oracle import fe
    dim = len(shape)
    lam, mu = random_material(shape, 33, prec)
    rng = np.random.default_rng(L)
    A = rng.standard_normal((L, dim, dim)) * 0.01
    Eb = 0.5 * (A + np.swapaxes(A, 1, 2))
    tol = 1e-12 if prec == "fp64" else 1e-6
    out = _solve(shape, lam, mu, Eb, prec, tol, max_iter=2000)
    assert out["status"] == 0 and len(out["report"]) == L
    ref = fe.homogenize(None, None, Eb, lam_mu=(lam, mu))
    lim = 1e-10 if prec == "fp64" else 1e-4
    for l in range(L):
        assert rel(out["stress_mean"][l], ref["sig_mean"][l]) < lim, l
    W = out["energy"]
    Wr = ref["W"]
    np.testing.assert_allclose(W, W.T, rtol=0, atol=1e-12 * np.abs(W).max())
    np.testing.assert_allclose(W, Wr, rtol=0, atol=(1e-9 if prec == "fp64" else 1e-4) * np.abs(Wr).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_laminate_exact(dim):
    """Laminate with interfaces on voxel faces: FE exact, C_eff equals the
    oracle (pinned to the closed form)."""
    say("laminate", dim)
    from oracle import fe
    shape = (12, 8) if dim == 2 else (8, 6, 4)
    m = ms.laminate(shape, 0, 5, E=(1.0, 9.0), nu=(0.3, 0.2))
    lam, mu = fe.lame(m.E, m.nu)
    Eb = ms.unit_loads(dim)
    out = _solve(shape, lam, mu, Eb, "fp64", 1e-13)
    ref = fe.homogenize(m.E, m.nu, Eb)
    assert rel(out["C_eff"], ref["C_eff"]) < 1e-11


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_homogeneous_zero_iterations(dim, prec):
    """Uniform material: the right-hand side vanishes exactly (difference
    stencils), the solve stops at 0 iterations with e = Ebar."""
    say("homogeneous", dim, prec)
    from oracle import fe
    shape = (16, 12) if dim == 2 else (8, 6, 10)
    lam, mu = fe.lame(np.full(shape, 3.0), np.full(shape, 0.25))
    Eb = ms.unit_loads(dim)
    out = _solve(shape, lam, mu, Eb, prec, 1e-10, fields=True)
    assert all(r["iterations"] == 0 for r in out["report"])
    dt = np.float64 if prec == "fp64" else np.float32
    for l in range(len(Eb)):
        # the strain field is stored in the plan precision
        assert np.abs(out["strain"][l] - Eb[l].astype(dt).astype(np.float64)).max() == 0.0
    lam0, mu0 = fe.lame(3.0, 0.25)
    nv = 3 if dim == 2 else 6
    C = np.zeros((nv, nv))
    C[:dim, :dim] = lam0
    C[np.arange(dim), np.arange(dim)] += 2 * mu0
    C[np.arange(dim, nv), np.arange(dim, nv)] = mu0
    assert rel(out["C_eff"], C) < (1e-14 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("dim", [2, 3])
def test_identity_material_one_iteration(dim):
    """lambda = 0, mu = 1/2: K equals the preconditioner M, so from any warm
    start the preconditioned CG converges in exactly one iteration to the
    zero fluctuation (pins the scaling of (B^*B)^-1 and of the FFT pair)."""
    say("identity material", dim)
    shape = (12, 10) if dim == 2 else (6, 8, 4)
    N = int(np.prod(shape))
    rng = np.random.default_rng(8)
    u0 = rng.standard_normal((1, N, dim))
    Eb = np.zeros((1, dim, dim))
    Eb[0, 0, 0] = 0.01
    out = _solve(shape, np.zeros(shape), np.full(shape, 0.5), Eb, "fp64", 1e-12, return_u=True, u0=u0)
    assert out["report"][0]["iterations"] == 1
    umax = float(np.abs(out["u"][0]).max())
    assert umax < 1e-12, umax


@pytest.mark.parametrize("shape", [(16, 12), (6, 5, 7)])
def test_warm_starts(shape):
    """Warm starts (u0): from the converged u shifted by a constant (the mean
    is removed) the solve stops at once with the same fields; from a
    perturbed u it converges to the same C_eff; with Ebar = 0 and a random u0
    the solution is the zero fluctuation."""
    say("warm starts", shape)
    dim = len(shape)
    lam, mu = random_material(shape, 19, "fp64")
    Eb = ms.unit_loads(dim)
    cold = _solve(shape, lam, mu, Eb, "fp64", 1e-12, return_u=True)
    u = cold["u"]
    again = _solve(shape, lam, mu, Eb, "fp64", 1e-12, return_u=True, u0=u + 0.3)
    assert max(r["iterations"] for r in again["report"]) <= 1
    np.testing.assert_allclose(again["u"], u, rtol=0, atol=1e-9 * np.abs(u).max())
    assert rel(again["C_eff"], cold["C_eff"]) < 1e-12
    rng = np.random.default_rng(3)
    pert = _solve(shape, lam, mu, Eb, "fp64", 1e-12, return_u=True, u0=u + 1e-3 * rng.standard_normal(u.shape))
    assert pert["status"] == 0 and rel(pert["C_eff"], cold["C_eff"]) < 1e-10
    np.testing.assert_allclose(pert["u"], u, rtol=0, atol=1e-8 * np.abs(u).max())
    u0 = rng.standard_normal(u.shape[1:])[None]
    zero = _solve(shape, lam, mu, np.zeros((1, dim, dim)), "fp64", 1e-12, return_u=True, u0=u0)
    assert zero["status"] == 0
    assert np.abs(zero["u"]).max() < 1e-10 * np.abs(u0).max()
    assert np.abs(zero["stress_mean"]).max() < 1e-10


def test_two_plans_two_streams_two_threads():
    """Plans share no device or host state (the error message is per thread):
    two plans on their own streams, solved at the same time from two host
    threads, give bitwise the results of the same solves run one after the
    other."""
    import threading
    import torch
    from paper_2105_03297_amd import Homogenizer
    say("two plans, two streams, two threads")
    cases = [((16, 12), 5, "fp64"), ((6, 5, 7), 6, "fp32")]
    mats = [random_material(s, seed, prec) for s, seed, prec in cases]
    loads = [ms.unit_loads(len(s)) for s, _, _ in cases]

    def run(i, stream, out):
        shape, _, prec = cases[i]
        h = Homogenizer(shape, n_load=len(loads[i]), precision=prec, stream=stream)
        h.set_material(lam=mats[i][0], mu=mats[i][1])
        r = h.solve(loads[i], tol=1e-10 if prec == "fp64" else 1e-6, max_iter=3000)
        out[i] = (r["C_eff"], [x["iterations"] for x in r["report"]])
        h.close()

    seq = [None, None]
    for i in range(2):
        run(i, None, seq)
    conc = [None, None]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    threads = [threading.Thread(target=run, args=(i, streams[i], conc)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    for i in range(2):
        assert conc[i] is not None, i
        assert np.array_equal(conc[i][0], seq[i][0]) and conc[i][1] == seq[i][1], i


def test_max_iter_reports_noconv_and_keeps_last_iterate():
    say("max_iter")
    from oracle import fe
    m, Eb, _, _ = ms.workload("circle32")
    lam, mu = fe.lame(m.E, m.nu)
    out = _solve(m.shape, lam, mu, Eb, "fp64", 1e-14, max_iter=3)
    import paper_2105_03297_amd as feh
    assert out["status"] == feh.FEH_ENOCONV
    assert out["report"][0]["iterations"] == 3
    assert out["report"][0]["status"] == feh.FEH_ENOCONV
    ref = fe.homogenize(m.E, m.nu, Eb)
    # the last iterate is already a reasonable approximation
    assert rel(out["stress_mean"][0], ref["sig_mean"][0]) < 0.05


def test_repeat_solves_bitwise_identical():
    say("determinism")
    lam, mu = random_material((10, 12, 9), 3, "fp32")
    Eb = ms.unit_loads(3)
    a = _solve((10, 12, 9), lam, mu, Eb, "fp32", 1e-6, fields=True)
    b = _solve((10, 12, 9), lam, mu, Eb, "fp32", 1e-6, fields=True)
    assert np.array_equal(a["energy"], b["energy"])
    assert np.array_equal(a["strain"], b["strain"])
    assert [r["iterations"] for r in a["report"]] == [r["iterations"] for r in b["report"]]


def test_batched_load_cases_independent():
    """Load cases batched in one solve stop independently and reproduce the
    single-load-case solves."""
    say("batch independence")
    lam, mu = random_material((14, 10), 5, "fp64")
    Eb = ms.unit_loads(2)
    Eb[2] *= 7.0
    allc = _solve((14, 10), lam, mu, Eb, "fp64", 1e-11)
    for l in range(3):
        one = _solve((14, 10), lam, mu, Eb[l:l + 1], "fp64", 1e-11)
        assert one["report"][0]["iterations"] == allc["report"][l]["iterations"]
        assert rel(one["stress_mean"][0], allc["stress_mean"][l]) < 1e-13


def test_fp32_vs_fp64_circle32():
    say("fp32 vs fp64 circle32")
    from oracle import fe
    m, _, _, _ = ms.workload("circle32")
    lam, mu = fe.lame(m.E, m.nu)
    Eb = ms.unit_loads(2)
    o32 = _solve(m.shape, lam.astype(np.float32).astype(np.float64), mu.astype(np.float32).astype(np.float64),
                 Eb, "fp32", 1e-5)
    ref = fe.homogenize(m.E, m.nu, Eb)
    assert rel(o32["C_eff"], ref["C_eff"]) < 1e-5


@pytest.mark.parametrize("shape", [(48, 24), (8, 5, 48)])
@pytest.mark.parametrize("scale", [1e-12, 1e-3, 1e3, 1e12])
def test_fp32_voxel_scale_invariance(shape, scale):
    """C_eff does not depend on a uniform scaling of the voxel (the element
    stiffness and the load both scale out of the energy balance).  FP32 plans
    form M(k)^-1 in FP32 away from k = 0; M itself has entries of order h and
    a determinant of order h^3 in 3D (up to about 1.7e39 at h = 1e12, beyond
    the FP32 range), so the kernel forms it from the dimensionless factors
    a_a h_max, and the CG paths scale K, f and M by the voxel volume (element
    volume 1/6 of the voxel), whose h^3 / 6 would leave the FP32 normal range
    below h = 1e-12 (sigma |e| of order 1e-39).  Scaled voxels must leave
    C_eff, and the iteration count to within a few, unchanged.  The grids hold
    wavevectors on both sides of the FP64 long-wavelength shell."""
    say("fp32 voxel scale", shape, scale)
    from oracle import fe
    dim = len(shape)
    lam, mu = random_material(shape, 5, "fp32")
    Eb = ms.unit_loads(dim)
    hvox = np.array((1.0, 1.3, 0.8)[:dim])
    base = _solve(shape, lam, mu, Eb, "fp32", 1e-6, h=tuple(hvox))
    out = _solve(shape, lam, mu, Eb, "fp32", 1e-6, h=tuple(scale * hvox))
    ref = fe.homogenize(None, None, Eb, h=tuple(hvox), lam_mu=(lam, mu))
    assert out["status"] == 0 and base["status"] == 0
    assert rel(out["C_eff"], ref["C_eff"]) < 1e-5
    assert rel(base["C_eff"], ref["C_eff"]) < 1e-5
    for l in range(len(Eb)):
        assert abs(out["report"][l]["iterations"] - base["report"][l]["iterations"]) <= 3
