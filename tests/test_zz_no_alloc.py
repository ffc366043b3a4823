"""The allocation-free solve (feh_solve_noalloc, the library's static device
workspace) through the C ABI against feh_solve on a torch workspace: two
calls in a row, the second on a smaller grid, each compared field by field;
and the size limit of the static workspace."""
import numpy as np
import pytest

import microstructures as ms
from gpu_util import random_material, rel, say

pytestmark = pytest.mark.gpu


def _reference(shape, lam, mu, Eb, prec, tol):
    import paper_2105_03297_amd as feh
    h = feh.Homogenizer(shape, n_load=len(Eb), precision=prec)
    h.set_material(lam=lam, mu=mu)
    out = h.solve(Eb, tol=tol, max_iter=3000, return_u=True)
    out["u"] = out["u"].double().cpu().numpy()
    h.close()
    return out


def _noalloc(shape, lam, mu, Eb, prec, tol):
    import torch
    import paper_2105_03297_amd as feh
    dt = torch.float64 if prec == "fp64" else torch.float32
    L, D, N = len(Eb), len(shape), int(np.prod(shape))
    stream = torch.cuda.current_stream()
    plan = feh.feh_plan_create(D, shape, None, L, feh.FEH_FP64 if prec == "fp64" else feh.FEH_FP32,
                               stream.cuda_stream)
    lt = torch.as_tensor(lam, dtype=dt, device="cuda").contiguous()
    mt = torch.as_tensor(mu, dtype=dt, device="cuda").contiguous()
    u = torch.empty((L, N, D), dtype=dt, device="cuda")
    rc, smean, W, rep = feh.feh_solve_noalloc(plan, lt.data_ptr(), mt.data_ptr(), Eb, tol, 3000, 0, u.data_ptr())
    feh.feh_plan_destroy(plan)
    return dict(status=rc, stress_mean=smean, energy=W, report=rep, u=u.double().cpu().numpy())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_solve_twice(prec):
    tol = 1e-12 if prec == "fp64" else 1e-6
    bar = 1e-10 if prec == "fp64" else 1e-5
    for shape, seed in (((40, 36, 44), 3), ((24, 20, 18), 4)):  # the second call is smaller
        say("noalloc vs feh_solve", shape, prec)
        lam, mu = random_material(shape, seed, prec)
        Eb = ms.unit_loads(3)
        ref = _reference(shape, lam, mu, Eb, prec, tol)
        got = _noalloc(shape, lam, mu, Eb, prec, tol)
        assert got["status"] == 0 and ref["status"] == 0
        assert [r["iterations"] for r in got["report"]] == [r["iterations"] for r in ref["report"]]
        assert rel(got["energy"], ref["energy"]) < bar
        assert rel(got["stress_mean"], ref["stress_mean"]) < bar
        for l in range(len(Eb)):
            assert rel(got["u"][l], ref["u"][l]) < bar


def test_noalloc_rejects_plans_beyond_the_static_workspace():
    import torch
    import paper_2105_03297_amd as feh
    say("noalloc size limit")
    plan = feh.feh_plan_create(3, (128, 128, 128), None, 6, feh.FEH_FP32, torch.cuda.current_stream().cuda_stream)
    assert feh.feh_plan_workspace_bytes(plan) > 256 << 20
    x = torch.ones(4, device="cuda")
    with pytest.raises(feh.FehError) as ei:
        feh.feh_solve_noalloc(plan, x.data_ptr(), x.data_ptr(), ms.unit_loads(3), 1e-5, 10)
    assert ei.value.status == feh.FEH_ENOMEM
    assert "static scratch" in ei.value.message
    feh.feh_plan_destroy(plan)
