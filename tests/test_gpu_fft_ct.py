"""The compile-time transforms (power-of-two axes of 64 to 512 points in the
default radix order: the middle-axis pass, the CG's fused first-axis pass
and, in FP32, the last-axis passes of 128 to 512 points with their fused CG
updates) against the run-time passes they replace, on the same plan: the CG
solution, its iteration counts and C_eff, and the FFT export against the DFT
definition.  Both use the same butterflies and twiddles in the same order,
so they agree to rounding (the compiler may contract multiply-adds
differently in the two instruction streams)."""
import numpy as np
import pytest

import microstructures as ms
from gpu_util import random_material, rel, say

pytestmark = pytest.mark.gpu


def _solve(shape, lam, mu, prec, ct):
    import paper_2105_03297_amd as feh
    dim = len(shape)
    h = feh.Homogenizer(shape, n_load=3 if dim == 2 else 6, precision=prec)
    t = feh.feh_plan_tuning(h.plan)
    t["compile_time_transforms"] = ct
    feh.feh_plan_set_tuning(h.plan, t)
    assert feh.feh_plan_tuning(h.plan)["compile_time_transforms"] == ct
    h.set_material(lam=lam, mu=mu)
    out = h.solve(ms.unit_loads(dim), tol=1e-10 if prec == "fp64" else 1e-5, max_iter=3000, return_u=True)
    out["u"] = out["u"].double().cpu().numpy()
    h.close()
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (128, 64, 20), (256, 128, 12), (40, 256, 18), (64, 12, 64),
                                   (256, 90), (64, 128),
                                   # last axis of 128 / 256 points, with a partial row block (rows % 16 != 0)
                                   (9, 7, 256), (24, 10, 128), (33, 128), (40, 256),
                                   # 512-point axes: first, middle, last (3D and 2D)
                                   (512, 6, 10), (5, 512, 12), (6, 9, 512), (512, 40), (21, 512), (512, 512)])
def test_compile_time_transforms_match_runtime_passes(shape, prec):
    say("compile-time vs run-time transforms", shape, prec)
    lam, mu = random_material(shape, 17, prec)
    a = _solve(shape, lam, mu, prec, 1)
    b = _solve(shape, lam, mu, prec, 0)
    ia = [r["iterations"] for r in a["report"]]
    ib = [r["iterations"] for r in b["report"]]
    eu = max(rel(a["u"][l], b["u"][l]) for l in range(len(ia)))
    ec = rel(a["C_eff"], b["C_eff"])
    print(shape, prec, "iterations", ia, ib, "u rel diff %.3e, C_eff rel diff %.3e, bitwise %s"
          % (eu, ec, bool(np.array_equal(a["u"], b["u"]))))
    assert all(abs(x - y) <= 1 for x, y in zip(ia, ib))
    bar = 1e-12 if prec == "fp64" else 1e-5
    assert ec < bar and eu < (1e-10 if prec == "fp64" else 1e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(8, 64, 16), (4, 128, 8), (3, 256, 10), (5, 64, 9), (3, 5, 256), (2, 6, 128),
                                   (3, 512, 6), (2, 5, 512)])
def test_fft_with_compile_time_passes_matches_dft(shape, prec):
    import paper_2105_03297_amd as feh
    say("fft compile-time middle", shape, prec)
    L = 2
    h = feh.Homogenizer(shape, n_load=L, precision=prec)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((L * 3,) + shape)
    X = h.fft_forward(x.reshape(L * 3, -1)).cpu().numpy()
    ref = np.fft.rfftn(x, axes=(1, 2, 3))
    tol = 1e-13 if prec == "fp64" else 3e-6
    assert np.abs(X - ref).max() / np.abs(ref).max() < tol
    back = h.fft_inverse(ref.astype(np.complex128 if prec == "fp64" else np.complex64))
    np.testing.assert_allclose(back.cpu().numpy().reshape(x.shape), x, atol=tol * np.abs(x).max() * 10)
    h.close()


def test_spectral_residual_warm_start_batches():
    """The CG with its residual kept as a last-axis half spectrum (FP32,
    compile-time last-axis passes) against the real-field residual on the same
    plans: a warm start from a perturbed solution, a batched plan of two
    microstructures, and an uneven batch of two grids (graph replay); 2D warm
    start and uneven batch as well."""
    import paper_2105_03297_amd as feh
    say("spectral residual: warm start, batched plan, uneven batch")
    shape = (10, 12, 128)
    Eb = ms.unit_loads(3)
    lam, mu = random_material(shape, 23, "fp32")

    def plan(ct, n_batch=1, shp=shape):
        h = feh.Homogenizer(shp, n_load=6, precision="fp32", n_batch=n_batch)
        t = feh.feh_plan_tuning(h.plan)
        t["compile_time_transforms"] = ct
        feh.feh_plan_set_tuning(h.plan, t)
        assert feh.feh_plan_cg_residual_spectral(h.plan) == bool(ct)
        return h

    cold = {}
    for ct in (1, 0):
        h = plan(ct)
        h.set_material(lam=lam, mu=mu)
        o = h.solve(Eb, tol=1e-6, max_iter=3000, return_u=True)
        u = o["u"].double().cpu().numpy()
        pert = u + 1e-3 * np.abs(u).max() * np.random.default_rng(5).standard_normal(u.shape)
        w = h.solve(Eb, tol=1e-6, max_iter=3000, return_u=True, u0=pert)
        h.close()
        cold[ct] = (o, w)
    (o1, w1), (o0, w0) = cold[1], cold[0]
    print("cold C_eff rel diff %.3e, warm %.3e, warm iterations %s / %s" % (
        rel(o1["C_eff"], o0["C_eff"]), rel(w1["C_eff"], w0["C_eff"]),
        [r["iterations"] for r in w1["report"]], [r["iterations"] for r in w0["report"]]))
    assert rel(o1["C_eff"], o0["C_eff"]) < 1e-5
    assert w1["status"] == 0 and rel(w1["C_eff"], o1["C_eff"]) < 1e-5 and rel(w1["C_eff"], w0["C_eff"]) < 1e-5
    assert all(abs(a["iterations"] - b["iterations"]) <= 1 for a, b in zip(w1["report"], w0["report"]))

    # batched plan of two microstructures
    lam2, mu2 = random_material(shape, 24, "fp32")
    res = {}
    for ct in (1, 0):
        h = plan(ct, n_batch=2)
        h.set_material(lam=np.stack([lam, lam2]), mu=np.stack([mu, mu2]))
        o = h.solve(np.concatenate([Eb, Eb]), tol=1e-6, max_iter=3000)
        W = o["energy"]
        res[ct] = [feh.feh_effective_stiffness(3, Eb, W[6 * b:6 * b + 6, 6 * b:6 * b + 6]) for b in range(2)]
        h.close()
    for b in range(2):
        assert rel(res[1][b], res[0][b]) < 1e-5, b
    assert rel(res[1][0], o1["C_eff"]) < 1e-5

    # uneven batch of two grids, each with a compile-time last axis
    shapes = [(8, 6, 128), (6, 4, 256)]
    maps = []
    for i, shp in enumerate(shapes):
        E = np.exp(np.random.default_rng(40 + i).standard_normal(shp))
        maps.append((E, 0.3))
    ub = feh.UnevenBatch(maps, precision="fp32")
    assert all(feh.feh_plan_cg_residual_spectral(hz.plan) for hz, _ in ub.plans)
    out = ub.solve(Eb, tol=1e-6, max_iter=3000, use_graph=True)
    ub.close()
    for (E, nu), o in zip(maps, out):
        h = plan(0, shp=E.shape)
        h.set_material(E=E, nu=nu)
        ref = h.solve(Eb, tol=1e-6, max_iter=3000)
        h.close()
        assert rel(o["C_eff"], ref["C_eff"]) < 1e-5, (E.shape, rel(o["C_eff"], ref["C_eff"]))



def test_spectral_residual_2d():
    """2D plans with a 128- or 256-point last axis keep the residual as its
    last-axis half spectrum (the first-axis pass reads it): warm start and
    an uneven batch against the real-field residual."""
    import paper_2105_03297_amd as feh
    say("spectral residual 2D")
    Eb = ms.unit_loads(2)
    shape = (40, 128)
    lam, mu = random_material(shape, 29, "fp32")
    res = {}
    for ct in (1, 0):
        h = feh.Homogenizer(shape, n_load=3, precision="fp32")
        t = feh.feh_plan_tuning(h.plan)
        t["compile_time_transforms"] = ct
        feh.feh_plan_set_tuning(h.plan, t)
        assert feh.feh_plan_cg_residual_spectral(h.plan) == bool(ct)
        h.set_material(lam=lam, mu=mu)
        o = h.solve(Eb, tol=1e-6, max_iter=3000, return_u=True)
        u = o["u"].double().cpu().numpy()
        w = h.solve(Eb, tol=1e-6, max_iter=3000, u0=u + 1e-3 * np.abs(u).max())
        h.close()
        res[ct] = (o, w)
    assert rel(res[1][0]["C_eff"], res[0][0]["C_eff"]) < 1e-5
    assert all(abs(a["iterations"] - b["iterations"]) <= 1 for a, b in zip(res[1][0]["report"], res[0][0]["report"]))
    assert res[1][1]["status"] == 0 and rel(res[1][1]["C_eff"], res[0][0]["C_eff"]) < 1e-5
    maps = [(np.exp(np.random.default_rng(50 + i).standard_normal(s)), 0.3) for i, s in enumerate([(64, 256), (30, 128)])]
    ub = feh.UnevenBatch(maps, precision="fp32")
    assert all(feh.feh_plan_cg_residual_spectral(hz.plan) for hz, _ in ub.plans)
    out = ub.solve(Eb, tol=1e-6, max_iter=3000, use_graph=True)
    ub.close()
    for (E, nu), o in zip(maps, out):
        h = feh.Homogenizer(E.shape, n_load=3, precision="fp32")
        t = feh.feh_plan_tuning(h.plan)
        t["compile_time_transforms"] = 0
        feh.feh_plan_set_tuning(h.plan, t)
        h.set_material(E=E, nu=nu)
        ref = h.solve(Eb, tol=1e-6, max_iter=3000)
        h.close()
        assert rel(o["C_eff"], ref["C_eff"]) < 1e-5, (E.shape, rel(o["C_eff"], ref["C_eff"]))
