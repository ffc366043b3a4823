"""The 2D Eshelby-inhomogeneity setup (151 x 151, soft disc of radius 10 % of
the edge, stiffness ratio 10, biaxial 1 % strain) with every derivative kind
of Sec. "Discrete projection": the GPU strain-space solver against the
oracle's projected CG element by element, the FE kind against the factored
solver and the canonical FE solve, and the square symmetry of the fields.
The 1661 x 1661 refinement (11 x 151: a radix-11 and a direct 151 pass per
axis) runs the FE kind in both solvers against each other."""
import numpy as np
import pytest

import microstructures as ms
from gpu_util import rel, say

pytestmark = pytest.mark.gpu


def _setup(n):
    from oracle import fe
    m, Eb, tol, _ = ms.workload(f"eshelby{n}")
    lam, mu = fe.lame(m.E, m.nu)
    return m, lam, mu, Eb


@pytest.mark.parametrize("kind", ["fe", "fd", "cd", "ls", "fourier", "fourier2"])
def test_eshelby151_kinds_match_oracle(kind):
    import torch
    from oracle import pcg
    from paper_2105_03297_amd import Homogenizer
    say("eshelby151", kind)
    m, lam, mu, Eb = _setup(151)
    hz = Homogenizer(m.shape, n_load=1, precision="fp64")
    hz.set_material(lam=lam, mu=mu)
    out = hz.strain_cg_solve(Eb, kind=kind, tol=1e-12, max_iter=5000, fields=True)
    torch.cuda.synchronize()
    got = out["strain"].cpu().numpy()[0]
    e, it, _ = pcg.solve(lam, mu, Eb[0], kind=kind, tol=1e-12)
    ref = pcg.flat_fields(e)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    assert abs(out["report"][0]["iterations"] - it) <= 2
    # the disc is centred on a voxel and every discretisation maps onto
    # itself under the diagonal mirror (x <-> y; each triangle onto itself):
    # e_xx(x, y) = e_yy(y, x) per evaluation point
    ne = got.shape[1]
    g = got.reshape(151, 151, ne, 2, 2)
    for t in range(ne):
        np.testing.assert_allclose(g[:, :, t, 0, 0], g[:, :, t, 1, 1].T, rtol=0, atol=1e-9 * np.abs(g).max())
        np.testing.assert_allclose(g[:, :, t, 0, 1], g[:, :, t, 0, 1].T, rtol=0, atol=1e-9 * np.abs(g).max())
    hz.close()


def test_eshelby151_fe_equals_factored_and_fe_solve():
    import torch
    from oracle import fe
    from paper_2105_03297_amd import Homogenizer
    say("eshelby151 fe: strain space vs factored vs FE solve")
    m, lam, mu, Eb = _setup(151)
    hz = Homogenizer(m.shape, n_load=1, precision="fp64")
    hz.set_material(lam=lam, mu=mu)
    a = hz.solve(Eb, tol=1e-12, max_iter=5000, fields=True)
    b = hz.strain_cg_solve(Eb, kind="fe", tol=1e-12, max_iter=5000, fields=True)
    torch.cuda.synchronize()
    ref = fe.homogenize(m.E, m.nu, Eb)
    ea, eb = a["strain"].cpu().numpy()[0], b["strain"].cpu().numpy()[0]
    np.testing.assert_allclose(ea, ref["eps"][0], rtol=0, atol=1e-9 * np.abs(ref["eps"][0]).max())
    np.testing.assert_allclose(eb, ref["eps"][0], rtol=0, atol=1e-9 * np.abs(ref["eps"][0]).max())
    assert rel(b["stress_mean"][0], ref["sig_mean"][0]) < 1e-10
    hz.close()


def test_eshelby1661_fe_two_solvers_agree():
    import torch
    from paper_2105_03297_amd import Homogenizer
    say("eshelby1661 fe")
    m, lam, mu, Eb = _setup(1661)
    hz = Homogenizer(m.shape, n_load=1, precision="fp64")
    hz.set_material(lam=lam, mu=mu)
    a = hz.solve(Eb, tol=1e-10, max_iter=5000, fields=True)
    b = hz.strain_cg_solve(Eb, kind="fe", tol=1e-10, max_iter=5000, fields=True)
    torch.cuda.synchronize()
    ea, eb = a["strain"].cpu().numpy()[0], b["strain"].cpu().numpy()[0]
    assert np.abs(ea - eb).max() < 1e-7 * np.abs(ea).max()
    assert rel(b["stress_mean"][0], a["stress_mean"][0]) < 1e-9
    # iteration counts of the FE projection do not grow with the refinement
    its = a["report"][0]["iterations"]
    hz.close()
    hz = Homogenizer((151, 151), n_load=1, precision="fp64")
    m1, lam1, mu1, _ = _setup(151)
    hz.set_material(lam=lam1, mu=mu1)
    c = hz.solve(Eb, tol=1e-10, max_iter=5000)
    assert abs(its - c["report"][0]["iterations"]) <= 0.2 * its + 5
    hz.close()
