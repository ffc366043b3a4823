"""Batched plans and uneven batches (several grids solved together, CG chunks
replayed as captured HIP graphs).

  * a batched plan of several microstructures of one shape reproduces the
    single-microstructure solves (FP64, bitwise iteration counts, C_eff to
    1e-13) and keeps load cases of different microstructures apart;
  * sensitivities of a batched plan equal the single-plan ones;
  * the uneven-batch workload (48 two-phase 2D maps of sizes 64^2 .. 512^2,
    laminates and circular inclusions, contrast log-uniform in [2, 1000],
    3 load cases each, FP32): laminates against their closed form, a sample of
    circle maps against the oracle's direct solve, graph replay against
    eager launches (bitwise), and C_eff_1111 sensitivities against separate
    single-map plans."""
import numpy as np
import pytest

import microstructures as ms
from gpu_util import random_material, rel, say

pytestmark = pytest.mark.gpu


def _single(shape, lam, mu, Eb, prec, tol):
    import paper_2105_03297_amd as feh
    h = feh.Homogenizer(shape, n_load=len(Eb), precision=prec)
    h.set_material(lam=lam, mu=mu)
    out = h.solve(Eb, tol=tol, max_iter=5000)
    h.close()
    return out


@pytest.mark.parametrize("shape", [(20, 14), (6, 7, 5)])
def test_batched_plan_matches_single_plans(shape):
    import paper_2105_03297_amd as feh
    say("batched plan vs single", shape)
    dim = len(shape)
    Eb = ms.unit_loads(dim)
    mats = [random_material(shape, 30 + b) for b in range(3)]
    h = feh.Homogenizer(shape, n_load=len(Eb), precision="fp64", n_batch=3)
    h.set_material(lam=np.stack([m[0] for m in mats]), mu=np.stack([m[1] for m in mats]))
    out = h.solve(np.concatenate([Eb] * 3), tol=1e-12, max_iter=5000)
    W = out["energy"]
    G = len(Eb)
    for b in range(3):
        one = _single(shape, mats[b][0], mats[b][1], Eb, "fp64", 1e-12)
        assert rel(out["C_eff_batch"][b], one["C_eff"]) < 1e-13
        assert [r["iterations"] for r in out["report"][b * G:(b + 1) * G]] == [r["iterations"] for r in one["report"]]
        for c in range(3):
            if c != b:
                assert np.all(W[b * G:(b + 1) * G, c * G:(c + 1) * G] == 0.0)
    # sensitivities of microstructure b equal the single-plan ones
    Gm = np.random.default_rng(3).standard_normal((G, G))
    gl, gm = h.c_eff_sensitivity(Gm)
    h.close()
    for b in range(3):
        h1 = feh.Homogenizer(shape, n_load=G, precision="fp64")
        h1.set_material(lam=mats[b][0], mu=mats[b][1])
        h1.solve(Eb, tol=1e-12, max_iter=5000)
        l1, m1 = h1.c_eff_sensitivity(Gm)
        h1.close()
        assert rel(gl[b].cpu().numpy(), l1.cpu().numpy()) < 1e-11
        assert rel(gm[b].cpu().numpy(), m1.cpu().numpy()) < 1e-11


def _c5_maps():
    from oracle import fe
    maps = ms.uneven_batch()
    return maps, [fe.lame(m.E, m.nu) for m in maps]


@pytest.fixture(scope="module")
def c5():
    import paper_2105_03297_amd as feh
    maps, lm = _c5_maps()
    lm32 = [(l.astype(np.float32).astype(np.float64), m.astype(np.float32).astype(np.float64)) for l, m in lm]
    ub = feh.UnevenBatch(lm32, precision="fp32")
    out = ub.solve(ms.unit_loads(2)[:, :, :], tol=1e-5, max_iter=5000, use_graph=True)
    yield maps, lm32, ub, out
    ub.close()


def test_uneven_batch_laminates_closed_form(c5):
    from test_oracle_fe import _laminate_closed_form, _voigt_C
    from oracle import fe
    say("uneven batch laminates")
    maps, lm, ub, out = c5
    n_lam = 0
    for m, o in zip(maps, out):
        assert o["status"] in (0,)
        if m.extra["kind"] != "laminate":
            continue
        n_lam += 1
        c = m.extra["contrast"]
        lam1, mu1 = fe.lame(c, 0.3)
        lam2, mu2 = fe.lame(1.0, 0.3)
        C1, C2 = _voigt_C(np.float32(lam1), np.float32(mu1), 2), _voigt_C(np.float32(lam2), np.float32(mu2), 2)
        ref = _laminate_closed_form(C1, C2, 0.5, 2, m.extra["axis"])
        assert rel(o["C_eff"], ref) < 1e-5, (m.recipe, rel(o["C_eff"], ref))
    assert n_lam > 5


def test_uneven_batch_circles_match_oracle(c5):
    from oracle import fe
    say("uneven batch circles vs oracle")
    maps, lm, ub, out = c5
    checked = 0
    for i, (m, o) in enumerate(zip(maps, out)):
        if m.extra["kind"] != "circle" or m.shape[0] > 128:
            continue
        ref = fe.homogenize(None, None, ms.unit_loads(2), lam_mu=lm[i])
        assert rel(o["C_eff"], ref["C_eff"]) < 1e-5, (m.recipe, rel(o["C_eff"], ref["C_eff"]))
        checked += 1
    assert checked >= 3


def test_uneven_batch_graph_replay_equals_eager(c5):
    say("uneven batch graph vs eager")
    maps, lm, ub, out = c5
    eager = ub.solve(ms.unit_loads(2), tol=1e-5, max_iter=5000, use_graph=False)
    again = ub.solve(ms.unit_loads(2), tol=1e-5, max_iter=5000, use_graph=True)
    for a, b, c in zip(out, eager, again):
        assert np.array_equal(a["C_eff"], b["C_eff"])
        assert np.array_equal(a["C_eff"], c["C_eff"])
        assert [r["iterations"] for r in a["report"]] == [r["iterations"] for r in b["report"]]
    assert ub.graph_launches() >= 1


def test_uneven_batch_sensitivity_matches_single_plans(c5):
    """Per-pixel d C_eff_1111 / d(lambda, mu) of a few maps from the batch
    equal those of separate single-map plans."""
    import paper_2105_03297_amd as feh
    say("uneven batch sensitivities")
    maps, lm, ub, out = c5
    G = np.zeros((3, 3))
    G[0, 0] = 1.0
    sens = ub.c_eff_sensitivity(G)
    for i in (0, 7, 23, 41):
        h = feh.Homogenizer(maps[i].shape, n_load=3, precision="fp32")
        h.set_material(lam=lm[i][0], mu=lm[i][1])
        h.solve(ms.unit_loads(2), tol=1e-5, max_iter=5000)
        gl, gm = h.c_eff_sensitivity(G)
        h.close()
        assert rel(sens[i][0].cpu().numpy(), gl.cpu().numpy()) < 1e-4
        assert rel(sens[i][1].cpu().numpy(), gm.cpu().numpy()) < 1e-4


@pytest.mark.parametrize("shape,prec", [((24, 20, 18), "fp64"), ((64, 48, 32), "fp32"), ((96, 80), "fp64")])
def test_autotuned_plan_matches_default(shape, prec):
    """After autotuning (any radix order and launch geometry) the solve equals
    the default plan's to rounding, and repeats bitwise."""
    import paper_2105_03297_amd as feh
    say("autotune", shape, prec)
    dim = len(shape)
    lam, mu = random_material(shape, 12, prec)
    Eb = ms.unit_loads(dim)
    tol = 1e-12 if prec == "fp64" else 1e-6
    ref = _single(shape, lam, mu, Eb, prec, tol)
    h = feh.Homogenizer(shape, n_load=len(Eb), precision=prec)
    h.set_material(lam=lam, mu=mu)
    tun = h.autotune(reps=2)
    print("tuning", tun)
    assert all(np.prod(r) == n for r, n in zip(tun["radices"], shape[:-1] + (shape[-1] // 2,)))
    a = h.solve(Eb, tol=tol, max_iter=5000)
    b = h.solve(Eb, tol=tol, max_iter=5000)
    h.close()
    assert np.array_equal(a["C_eff"], b["C_eff"])
    assert rel(a["C_eff"], ref["C_eff"]) < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("shape,prec", [((24, 20, 18), "fp64"), ((40, 36, 34), "fp32"), ((33, 17, 20), "fp64")])
def test_explicit_schedules_match_default(shape, prec):
    """Every schedule feh_plan_set_tuning accepts gives the default plan's
    solution to rounding: 16-row stencil tiles (ragged tiles included), the
    first-axis layout the default does not use (one workgroup per load case,
    or every load case in one workgroup with the inverses in registers), other
    radix orders and smaller workgroups; the CG iteration counts agree."""
    import paper_2105_03297_amd as feh
    say("explicit schedules", shape, prec)
    dim = len(shape)
    lam, mu = random_material(shape, 14, prec)
    Eb = ms.unit_loads(dim)
    tol = 1e-12 if prec == "fp64" else 1e-6
    ref = _single(shape, lam, mu, Eb, prec, tol)
    h = feh.Homogenizer(shape, n_load=len(Eb), precision=prec)
    h.set_material(lam=lam, mu=mu)
    base = feh.feh_plan_tuning(h.plan)
    PPT = 16 if prec == "fp64" else 24
    first_default = min(32, max(1, PPT * 256 // (shape[0] * dim)))
    other = 1 - base["first_per_load_case"]  # the first-axis layout the default does not use
    variants = [dict(base, stencil_rows=16), dict(base, first_per_load_case=other),
                dict(base, stencil_rows=16, first_per_load_case=other, rows_last=2, pencils_mid=2,
                     pencils_first=max(1, first_default // 4), radices=[list(reversed(r)) for r in base["radices"]])]
    for v in variants:
        feh.feh_plan_set_tuning(h.plan, v)
        assert feh.feh_plan_tuning(h.plan) == v
        out = h.solve(Eb, tol=tol, max_iter=5000)
        assert rel(out["C_eff"], ref["C_eff"]) < (1e-11 if prec == "fp64" else 1e-5), v
        its = [r["iterations"] for r in out["report"]]
        its_ref = [r["iterations"] for r in ref["report"]]
        assert max(abs(x - y) for x, y in zip(its, its_ref)) <= (1 if prec == "fp64" else 2), (v, its, its_ref)
    h.close()


def test_uneven_batch_streams_do_not_change_results():
    """The plans of an uneven batch on one shared stream or on separate
    streams (concurrent kernels, forked graph branches) give bitwise the same
    results, with graph replay and with eager launches."""
    import paper_2105_03297_amd as feh
    say("uneven batch one vs several streams")
    rng = np.random.default_rng(12)
    shapes = [(24, 20), (9, 31), (16, 16), (24, 20), (9, 31), (40, 8)]
    maps = [random_material(s, int(rng.integers(1000)), "fp32") for s in shapes]
    res = {}
    for ns in (1, 4):
        for graph in (True, False):
            ub = feh.UnevenBatch(maps, precision="fp32", n_streams=ns)
            assert len(ub.streams) == min(ns, 4)
            out = ub.solve(ms.unit_loads(2), tol=1e-6, max_iter=3000, use_graph=graph)
            res[(ns, graph)] = [(o["C_eff"], [r["iterations"] for r in o["report"]]) for o in out]
            ub.close()
    ref = res[(1, False)]
    for key, val in res.items():
        for (c, it), (cr, itr) in zip(val, ref):
            assert np.array_equal(c, cr) and it == itr, key


@pytest.mark.parametrize("max_iter", [1, 5, 13])
def test_uneven_batch_iteration_cap(c5, max_iter):
    """A cap below convergence for most load cases (chunks of 4 then 8
    iterations, stop checks one chunk behind): every load case stops at
    exactly max_iter with FEH_ENOCONV unless it converged first (laminates
    and homogeneous maps converge in a few iterations), with graph replay and
    eagerly, and a map's capped result (iteration counts, energies) equals
    the same map solved alone with the same cap."""
    import paper_2105_03297_amd as feh
    from oracle import fe
    say("uneven batch iteration cap", max_iter)
    maps, lm, ub, out = c5
    res = {}
    for graph in (True, False):
        got = ub.solve(ms.unit_loads(2), tol=1e-12, max_iter=max_iter, use_graph=graph)
        assert got[0]["status"] == feh.FEH_ENOCONV
        for o in got:
            for r in o["report"]:
                assert r["iterations"] <= max_iter
                assert (r["status"] == feh.FEH_ENOCONV) == (r["iterations"] == max_iter and r["rel_residual"] > 1e-12)
        res[graph] = got
    for a, b in zip(res[True], res[False]):
        assert np.array_equal(a["energy"], b["energy"])
    for i in (0, len(lm) - 1):
        lam, mu = lm[i]
        h = feh.Homogenizer(lam.shape, n_load=3, precision="fp32")
        h.set_material(lam=lam, mu=mu)
        ref = h.solve(ms.unit_loads(2), tol=1e-12, max_iter=max_iter)
        h.close()
        assert [r["iterations"] for r in ref["report"]] == [r["iterations"] for r in res[True][i]["report"]]
        assert rel(res[True][i]["energy"], ref["energy"]) < 1e-6, (i, rel(res[True][i]["energy"], ref["energy"]))
