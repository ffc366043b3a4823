"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every entry point the header declares, validates arguments, and its host
helper for the effective stiffness agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import microstructures as ms
import paper_2105_03297_amd as feh
from oracle import fe

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "feh.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(feh_\w+)\s*\(", txt, re.M)))


def test_header_symbols_exported():
    names = _declared()
    assert len(names) >= 16
    lib = ctypes.CDLL(feh.library_path())
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps every declared entry point under the same name
    for n in names:
        assert callable(getattr(feh, n)), n


def test_version_and_error_string():
    assert feh.feh_version() == 10000
    assert isinstance(feh.feh_last_error(), str)


@pytest.mark.parametrize("dim,n,nl,prec,code", [
    (1, (8,), 1, 0, feh.FEH_EINVAL),
    (2, (8, 1), 1, 0, feh.FEH_EINVAL),
    (2, (8, 8), 0, 0, feh.FEH_EINVAL),
    (2, (8, 8), 65, 0, feh.FEH_EINVAL),
    (2, (8, 8), 1, 7, feh.FEH_EINVAL),
    (2, (4096, 8), 1, 0, feh.FEH_ENOTSUP),
    (3, (8, 8, 8192), 1, 0, feh.FEH_EINVAL),
])
def test_plan_validation(dim, n, nl, prec, code):
    with pytest.raises(feh.FehError) as ei:
        feh.feh_plan_create(dim, n, None, nl, prec)
    assert ei.value.status == code


@pytest.mark.parametrize("n,passes", [((34, 8), [[2, 17], [4]]), ((151, 302), [[151], [151]]),
                                      ((17, 17), [[17], [17]]), ((26, 39), [[2, 13], [3, 13]])])
def test_prime_sizes_factorise(n, passes):
    """Prime factors above 13 become single direct-DFT passes; the last axis
    of even length is transformed at half length (two reals per point)."""
    p = feh.feh_plan_create(2, n, None, 1, feh.FEH_FP64)
    t = feh.feh_plan_tuning(p)
    got = [sorted(r) for r in t["radices"][:2]]
    assert got == [sorted(r) for r in passes]
    feh.feh_plan_destroy(p)


def test_cg_residual_form_follows_the_schedule():
    """The CG keeps its residual as a last-axis half spectrum exactly when the
    last-axis passes of an FP32 plan take the compile-time transform."""
    cases = [((64, 32, 256), feh.FEH_FP32, True), ((16, 8, 128), feh.FEH_FP32, True),
             ((8, 8, 512), feh.FEH_FP32, True), ((64, 64, 64), feh.FEH_FP32, False),
             ((16, 8, 256), feh.FEH_FP64, False), ((64, 256), feh.FEH_FP32, True),
             ((30, 512), feh.FEH_FP32, True), ((64, 64), feh.FEH_FP32, False),
             ((64, 250), feh.FEH_FP32, False), ((16, 8, 250), feh.FEH_FP32, False)]
    for n, prec, want in cases:
        p = feh.feh_plan_create(len(n), n, None, 2, prec)
        assert feh.feh_plan_cg_residual_spectral(p) is want, (n, prec)
        if want:
            t = feh.feh_plan_tuning(p)
            t["compile_time_transforms"] = 0
            feh.feh_plan_set_tuning(p, t)
            assert feh.feh_plan_cg_residual_spectral(p) is False
            t["compile_time_transforms"] = 1
            t["rows_last"] = 4
            feh.feh_plan_set_tuning(p, t)
            assert feh.feh_plan_cg_residual_spectral(p) is False
        feh.feh_plan_destroy(p)
    assert load_rc_null() < 0


def load_rc_null():
    return feh.load().feh_plan_cg_residual_spectral(None)


def test_bad_voxel_size():
    with pytest.raises(feh.FehError) as ei:
        feh.feh_plan_create(2, (8, 8), (1.0, -1.0), 1, 0)
    assert ei.value.status == feh.FEH_EINVAL


def test_plan_sizes_and_workspace_checks():
    p = feh.feh_plan_create(3, (256, 256, 256), None, 6, feh.FEH_FP32)
    b = feh.feh_plan_workspace_bytes(p)
    # 4 nodal vectors (u, r, p, q) + half spectrum + material: about 6.2 GB at
    # 256^3 x 6 load cases in FP32
    assert 5.8e9 < b < 6.6e9
    # calls that need a workspace fail before touching the device
    Eb = ms.unit_loads(3)
    with pytest.raises(feh.FehError) as ei:
        feh.feh_solve(p, Eb, 1e-5, 10)
    assert ei.value.status == feh.FEH_ENOMEM
    with pytest.raises(feh.FehError) as ei:
        feh.feh_plan_set_workspace(p, 0, b)
    assert ei.value.status == feh.FEH_EINVAL
    with pytest.raises(feh.FehError) as ei:
        feh.feh_plan_set_workspace(p, 4096, b - 1)
    assert ei.value.status == feh.FEH_ENOMEM
    feh.feh_plan_destroy(p)


@pytest.mark.parametrize("dim", [2, 3])
def test_effective_stiffness_helper_matches_oracle(dim):
    rng = np.random.default_rng(3)
    nv = 3 if dim == 2 else 6
    A = rng.standard_normal((nv, nv))
    C = A @ A.T + nv * np.eye(nv)
    Ebars = []
    for _ in range(nv):
        E = rng.standard_normal((dim, dim)) * 0.01
        Ebars.append(0.5 * (E + E.T))
    Ebars = np.array(Ebars)
    Ev = np.stack([fe.voigt_strain(E) for E in Ebars], axis=1)
    W = Ev.T @ C @ Ev
    got = feh.feh_effective_stiffness(dim, Ebars, W)
    np.testing.assert_allclose(got, fe.c_eff_energy(W, Ebars), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(got, C, rtol=1e-9, atol=1e-10)
    with pytest.raises(feh.FehError):
        feh.feh_effective_stiffness(dim, np.zeros((nv, dim, dim)), W)


def test_effective_stiffness_weights_match_oracle():
    """Host helper E^-1 G E^-T against the oracle's chain rule, general loads."""
    from oracle import adjoint
    rng = np.random.default_rng(4)
    for dim in (2, 3):
        nv = 3 if dim == 2 else 6
        Eb = np.array([0.5 * (a + a.T) for a in rng.standard_normal((nv, dim, dim))])
        G = rng.standard_normal((nv, nv))
        W = feh.feh_effective_stiffness_weights(dim, Eb, G)
        np.testing.assert_allclose(W, adjoint.objective_weights(Eb, G), rtol=1e-10, atol=1e-12)


def test_energy_sensitivity_needs_workspace_and_solution():
    p = feh.feh_plan_create(2, (8, 6), None, 3, feh.FEH_FP64)
    with pytest.raises(feh.FehError) as ei:
        feh.feh_energy_sensitivity(p, np.eye(3), 0, 0)
    assert ei.value.status in (feh.FEH_ENOMEM, feh.FEH_EINVAL)
    feh.feh_plan_destroy(p)


def test_plan_tuning_reports_default_schedule():
    p = feh.feh_plan_create(3, (256, 96, 30), None, 2, feh.FEH_FP32)
    t = feh.feh_plan_tuning(p)
    feh.feh_plan_destroy(p)
    assert (t["rows_last"], t["pencils_mid"], t["pencils_first"]) == (0, 0, 0)
    assert np.prod(t["radices"][0]) == 256 and np.prod(t["radices"][1]) == 96 and np.prod(t["radices"][2]) == 15
    assert t["radices"][0] == [8, 8, 4]


def test_set_tuning_validates_and_round_trips():
    p = feh.feh_plan_create(3, (16, 12, 10), None, 2, feh.FEH_FP32)
    t = feh.feh_plan_tuning(p)
    # default axis-0 layout: one workgroup per load case for a power-of-two axis 0
    assert t["stencil_rows"] == 8 and t["first_per_load_case"] == 1
    q = feh.feh_plan_create(3, (15, 12, 10), None, 2, feh.FEH_FP32)
    assert feh.feh_plan_tuning(q)["first_per_load_case"] == 0
    feh.feh_plan_destroy(q)
    t2 = dict(t, stencil_rows=16, first_per_load_case=0, radices=[[4, 4], [3, 4], [5]])
    feh.feh_plan_set_tuning(p, t2)
    assert feh.feh_plan_tuning(p) == t2
    for bad in (dict(t2, radices=[[4, 2], [3, 4], [5]]), dict(t2, radices=[[16], [3, 4], [5]]),
                dict(t2, stencil_rows=4), dict(t2, first_per_load_case=2), dict(t2, pencils_first=1)):
        with pytest.raises(feh.FehError) as ei:
            feh.feh_plan_set_tuning(p, bad)
        assert ei.value.status == feh.FEH_EINVAL
        assert feh.feh_plan_tuning(p) == t2
    feh.feh_plan_destroy(p)
