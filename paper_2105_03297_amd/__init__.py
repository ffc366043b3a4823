"""FE-projection FFT homogenization on MI355X (gfx950): Python binding.

A thin ctypes binding of ``libfeh.so`` (declared in ``include/feh.h``).  The
functions ``feh_*`` below carry the C names and only marshal arguments; every
step of the computation runs in the library's HIP kernels.  PyTorch provides
device memory and the stream (``Homogenizer`` is a convenience wrapper that
allocates the workspace and outputs as torch tensors).

The library refuses to load if it has not been built (``build.py``); there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "FEH_OK", "FEH_EINVAL", "FEH_ENOMEM", "FEH_EHIP", "FEH_ENOCONV", "FEH_EBREAKDOWN", "FEH_ENOTSUP",
    "FEH_FP64", "FEH_FP32", "FehError", "feh_report", "library_path", "load",
    "feh_plan_create", "feh_plan_create_batch", "feh_plan_destroy", "feh_plan_workspace_bytes", "feh_plan_set_workspace",
    "feh_set_material_lame", "feh_set_material_phases", "feh_set_material_field", "feh_solve", "feh_solve_noalloc",
    "feh_effective_stiffness", "feh_effective_stiffness_weights", "feh_energy_sensitivity", "feh_energy_sensitivity_E",
    "unit_loads", "UNIT_STRAIN",
    "feh_apply_operator", "feh_apply_preconditioner", "feh_apply_projection",
    "feh_fft_forward", "feh_fft_inverse", "feh_profile_enable", "feh_profile_read", "feh_stream_copy", "PROFILE_KINDS",
    "feh_batch_create", "feh_batch_destroy", "feh_batch_solve", "feh_batch_graph_launches",
    "feh_plan_autotune", "feh_plan_tuning", "feh_plan_set_tuning", "feh_plan_cg_residual_spectral",
    "FEH_DERIV_FE", "FEH_DERIV_FD", "FEH_DERIV_CD", "FEH_DERIV_LS", "FEH_DERIV_FOURIER", "FEH_DERIV_FOURIER2",
    "DERIV_KINDS", "feh_strain_cg_points", "feh_strain_cg_workspace_bytes", "feh_strain_cg_solve",
    "feh_finite_report", "feh_finite_strain_workspace_bytes", "feh_finite_strain_solve",
    "feh_last_error", "feh_version", "Homogenizer", "UnevenBatch",
]

FEH_OK, FEH_EINVAL, FEH_ENOMEM, FEH_EHIP, FEH_ENOCONV, FEH_EBREAKDOWN, FEH_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
FEH_FP64, FEH_FP32 = 0, 1
FEH_DERIV_FE, FEH_DERIV_FD, FEH_DERIV_CD, FEH_DERIV_LS, FEH_DERIV_FOURIER, FEH_DERIV_FOURIER2 = 0, 1, 2, 3, 4, 5
DERIV_KINDS = {"fe": FEH_DERIV_FE, "fd": FEH_DERIV_FD, "cd": FEH_DERIV_CD, "ls": FEH_DERIV_LS,
               "fourier": FEH_DERIV_FOURIER, "fourier2": FEH_DERIV_FOURIER2}

# The unit load set whose energy matrix gives C_eff: tensor strain 0.01 per
# normal component and per shear pair (engineering shear 0.02), in Voigt
# order (xx, yy, xy) / (xx, yy, zz, yz, xz, xy).
UNIT_STRAIN = 0.01


def unit_loads(dim):
    """[nv][D][D] unit macroscopic strains (the load cases C_eff is defined on)."""
    pairs = [(0, 0), (1, 1), (0, 1)] if dim == 2 else [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    Eb = np.zeros((len(pairs), dim, dim))
    for k, (a, b) in enumerate(pairs):
        Eb[k, a, b] = Eb[k, b, a] = UNIT_STRAIN
    return Eb


_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfeh.so")


class FehError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"feh error {status}: {message}")
        self.status = status
        self.message = message


class feh_report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]


def _report_dict(r):
    return dict(iterations=r.iterations, status=r.status, rel_residual=r.rel_residual, seconds=r.seconds)


class feh_finite_report(ctypes.Structure):
    _fields_ = [("newton_iterations", ctypes.c_int32), ("cg_iterations", ctypes.c_int32),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("rel_equilibrium", ctypes.c_double), ("rel_increment", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "feh_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                       _dp, ctypes.c_int, ctypes.c_int, _vp]),
    "feh_plan_create_batch": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                             _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "feh_plan_destroy": (ctypes.c_int, [_vp]),
    "feh_plan_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "feh_plan_set_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "feh_set_material_lame": (ctypes.c_int, [_vp, _vp, _vp]),
    "feh_set_material_phases": (ctypes.c_int, [_vp, _vp, _dp, ctypes.c_int]),
    "feh_set_material_field": (ctypes.c_int, [_vp, _vp, ctypes.c_double]),
    "feh_solve": (ctypes.c_int, [_vp, _dp, ctypes.c_double, ctypes.c_int, _vp, _vp, _vp, _vp, _dp, _dp,
                                 ctypes.POINTER(feh_report)]),
    "feh_solve_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _dp, ctypes.c_double, ctypes.c_int, _vp, _vp, _vp, _vp,
                                         _dp, _dp, ctypes.POINTER(feh_report)]),
    "feh_effective_stiffness": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]),
    "feh_effective_stiffness_weights": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]),
    "feh_energy_sensitivity": (ctypes.c_int, [_vp, _dp, _vp, _vp]),
    "feh_energy_sensitivity_E": (ctypes.c_int, [_vp, _dp, _vp]),
    "feh_apply_operator": (ctypes.c_int, [_vp, _vp, _vp]),
    "feh_apply_preconditioner": (ctypes.c_int, [_vp, _vp, _vp]),
    "feh_apply_projection": (ctypes.c_int, [_vp, _vp, _vp]),
    "feh_fft_forward": (ctypes.c_int, [_vp, _vp, _vp]),
    "feh_fft_inverse": (ctypes.c_int, [_vp, _vp, _vp]),
    "feh_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "feh_profile_read": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    "feh_stream_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp]),
    "feh_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int]),
    "feh_batch_destroy": (ctypes.c_int, [_vp]),
    "feh_batch_solve": (ctypes.c_int, [_vp, ctypes.POINTER(_dp), ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(_dp), ctypes.POINTER(_dp), ctypes.POINTER(ctypes.POINTER(feh_report))]),
    "feh_batch_graph_launches": (ctypes.c_int, [_vp]),
    "feh_plan_autotune": (ctypes.c_int, [_vp, ctypes.c_int]),
    "feh_plan_cg_residual_spectral": (ctypes.c_int, [_vp]),
    "feh_plan_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "feh_plan_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "feh_strain_cg_points": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "feh_strain_cg_workspace_bytes": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "feh_strain_cg_solve": (ctypes.c_int, [_vp, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _vp,
                                           ctypes.c_size_t, _vp, _dp, _dp, ctypes.POINTER(feh_report)]),
    "feh_finite_strain_workspace_bytes": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "feh_finite_strain_solve": (ctypes.c_int, [_vp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t,
                                               _vp, _vp, _dp, ctypes.POINTER(feh_finite_report)]),
    "feh_last_error": (ctypes.c_char_p, []),
    "feh_version": (ctypes.c_int, []),
}


def library_path():
    return _LIB_PATH


def load():
    """Load libfeh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python paper_2105_03297_amd/build.py` (no CPU fallback exists)")
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc, allow=()):
    if rc != FEH_OK and rc not in allow:
        raise FehError(rc, load().feh_last_error().decode())
    return rc


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


# --------------------------------------------------------------------------
# same-name wrappers (argument marshalling only)
# --------------------------------------------------------------------------
def feh_last_error():
    return load().feh_last_error().decode()


def feh_version():
    return load().feh_version()


def feh_plan_create(dim, n, h=None, n_load=1, precision=FEH_FP64, stream=0):
    n_arr = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))
    if h is None:
        h_ptr = None
    else:
        h_keep = (ctypes.c_double * 3)(*(list(h) + [1.0] * (3 - len(h))))
        h_ptr = ctypes.cast(h_keep, _dp)
    plan = _vp()
    _check(load().feh_plan_create(ctypes.byref(plan), int(dim), n_arr, h_ptr, int(n_load), int(precision),
                                  _vp(stream or 0)))
    return plan


def feh_plan_create_batch(dim, n, h=None, n_batch=1, n_load=1, precision=FEH_FP64, stream=0):
    n_arr = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))
    h_ptr = None
    if h is not None:
        h_keep = (ctypes.c_double * 3)(*(list(h) + [1.0] * (3 - len(h))))
        h_ptr = ctypes.cast(h_keep, _dp)
    plan = _vp()
    _check(load().feh_plan_create_batch(ctypes.byref(plan), int(dim), n_arr, h_ptr, int(n_batch), int(n_load),
                                        int(precision), _vp(stream or 0)))
    return plan


def feh_plan_destroy(plan):
    return _check(load().feh_plan_destroy(plan))


def feh_plan_workspace_bytes(plan):
    b = ctypes.c_size_t(0)
    _check(load().feh_plan_workspace_bytes(plan, ctypes.byref(b)))
    return b.value


def feh_plan_set_workspace(plan, dev_ptr, nbytes):
    return _check(load().feh_plan_set_workspace(plan, _vp(dev_ptr), ctypes.c_size_t(nbytes)))


def feh_set_material_lame(plan, lam_ptr, mu_ptr):
    return _check(load().feh_set_material_lame(plan, _vp(lam_ptr), _vp(mu_ptr)))


def feh_set_material_phases(plan, phase_ptr, E_nu):
    t, tp = _f64(E_nu)
    return _check(load().feh_set_material_phases(plan, _vp(phase_ptr), tp, int(t.shape[0])))


def feh_set_material_field(plan, E_ptr, nu):
    return _check(load().feh_set_material_field(plan, _vp(E_ptr), float(nu)))


def feh_solve(plan, Ebar, tol, max_iter, u0_ptr=0, u_ptr=0, strain_ptr=0, stress_ptr=0, allow_noconv=True):
    """Returns (status, stress_mean[L,D,D], energy[L,L], reports)."""
    Eb, Ebp = _f64(Ebar)
    L, D = Eb.shape[0], Eb.shape[1]
    smean = np.zeros((L, D, D))
    W = np.zeros((L, L))
    rep = (feh_report * L)()
    rc = load().feh_solve(plan, Ebp, float(tol), int(max_iter), _vp(u0_ptr or 0), _vp(u_ptr or 0),
                          _vp(strain_ptr or 0), _vp(stress_ptr or 0), smean.ctypes.data_as(_dp),
                          W.ctypes.data_as(_dp), rep)
    _check(rc, allow=(FEH_ENOCONV,) if allow_noconv else ())
    return rc, smean, W, [_report_dict(r) for r in rep]


def feh_solve_noalloc(plan, lam_ptr, mu_ptr, Ebar, tol, max_iter, u0_ptr=0, u_ptr=0, strain_ptr=0, stress_ptr=0,
                      allow_noconv=True):
    """feh_solve on the library's static workspace with the material passed in;
    returns (status, stress_mean[L,D,D], energy[L,L], reports)."""
    Eb, Ebp = _f64(Ebar)
    L, D = Eb.shape[0], Eb.shape[1]
    smean = np.zeros((L, D, D))
    W = np.zeros((L, L))
    rep = (feh_report * L)()
    rc = load().feh_solve_noalloc(plan, _vp(lam_ptr), _vp(mu_ptr), Ebp, float(tol), int(max_iter), _vp(u0_ptr or 0),
                                  _vp(u_ptr or 0), _vp(strain_ptr or 0), _vp(stress_ptr or 0),
                                  smean.ctypes.data_as(_dp), W.ctypes.data_as(_dp), rep)
    _check(rc, allow=(FEH_ENOCONV,) if allow_noconv else ())
    return rc, smean, W, [_report_dict(r) for r in rep]


def feh_strain_cg_points(kind, dim):
    n = ctypes.c_int(0)
    _check(load().feh_strain_cg_points(int(kind), int(dim), ctypes.byref(n)))
    return n.value


def feh_strain_cg_workspace_bytes(plan, kind):
    n = ctypes.c_size_t(0)
    _check(load().feh_strain_cg_workspace_bytes(plan, int(kind), ctypes.byref(n)))
    return n.value


def feh_strain_cg_solve(plan, kind, Ebar, tol, max_iter, work_ptr, work_bytes, strain_ptr=0, allow_noconv=True):
    """Returns (status, stress_mean[L,D,D], energy[L,L], reports)."""
    Eb, Ebp = _f64(Ebar)
    L, D = Eb.shape[0], Eb.shape[1]
    smean = np.zeros((L, D, D))
    W = np.zeros((L, L))
    rep = (feh_report * L)()
    rc = load().feh_strain_cg_solve(plan, int(kind), Ebp, float(tol), int(max_iter), _vp(work_ptr),
                                    ctypes.c_size_t(int(work_bytes)), _vp(strain_ptr or 0),
                                    smean.ctypes.data_as(_dp), W.ctypes.data_as(_dp), rep)
    _check(rc, allow=(FEH_ENOCONV,) if allow_noconv else ())
    return rc, smean, W, [_report_dict(r) for r in rep]


def feh_finite_strain_workspace_bytes(plan, kind):
    n = ctypes.c_size_t(0)
    _check(load().feh_finite_strain_workspace_bytes(plan, int(kind), ctypes.byref(n)))
    return n.value


def feh_finite_strain_solve(plan, kind, Fbar, n_steps, newton_tol, equil_tol, cg_tol, max_newton, max_cg,
                            work_ptr, work_bytes, F_ptr=0, P_ptr=0, allow_noconv=True):
    """Returns (status, P_mean[L,D,D], reports)."""
    Fb, Fbp = _f64(Fbar)
    L, D = Fb.shape[0], Fb.shape[1]
    pm = np.zeros((L, D, D))
    rep = (feh_finite_report * L)()
    rc = load().feh_finite_strain_solve(plan, int(kind), Fbp, int(n_steps), float(newton_tol), float(equil_tol),
                                        float(cg_tol), int(max_newton), int(max_cg), _vp(work_ptr),
                                        ctypes.c_size_t(int(work_bytes)), _vp(F_ptr or 0), _vp(P_ptr or 0),
                                        pm.ctypes.data_as(_dp), rep)
    _check(rc, allow=(FEH_ENOCONV,) if allow_noconv else ())
    return rc, pm, [dict(newton_iterations=r.newton_iterations, cg_iterations=r.cg_iterations, status=r.status,
                         rel_equilibrium=r.rel_equilibrium, rel_increment=r.rel_increment) for r in rep]


def feh_effective_stiffness(dim, Ebar, W):
    Eb, Ebp = _f64(Ebar)
    Wm, Wp = _f64(W)
    nv = 3 if dim == 2 else 6
    C = np.zeros((nv, nv))
    _check(load().feh_effective_stiffness(int(dim), int(Eb.shape[0]), Ebp, Wp, C.ctypes.data_as(_dp)))
    return C


def feh_batch_create(plans):
    arr = (_vp * len(plans))(*[p.value if isinstance(p, _vp) else p for p in plans])
    b = _vp()
    _check(load().feh_batch_create(ctypes.byref(b), arr, len(plans)))
    return b


def feh_batch_destroy(batch):
    return _check(load().feh_batch_destroy(batch))


def feh_batch_solve(batch, Ebars, tol, max_iter, use_graph=True, allow_noconv=True):
    """Ebars: per plan [L][D][D].  Returns (status, stress_means, energies, reports) per plan."""
    n = len(Ebars)
    keep = [np.ascontiguousarray(e, dtype=np.float64) for e in Ebars]
    eb = (_dp * n)(*[k.ctypes.data_as(_dp) for k in keep])
    sm = [np.zeros((k.shape[0], k.shape[1], k.shape[2])) for k in keep]
    W = [np.zeros((k.shape[0], k.shape[0])) for k in keep]
    reps = [(feh_report * k.shape[0])() for k in keep]
    smp = (_dp * n)(*[a.ctypes.data_as(_dp) for a in sm])
    Wp = (_dp * n)(*[a.ctypes.data_as(_dp) for a in W])
    rp = (ctypes.POINTER(feh_report) * n)(*[ctypes.cast(r, ctypes.POINTER(feh_report)) for r in reps])
    rc = load().feh_batch_solve(batch, eb, float(tol), int(max_iter), 1 if use_graph else 0, smp, Wp, rp)
    _check(rc, allow=(FEH_ENOCONV,) if allow_noconv else ())
    out_rep = [[_report_dict(r) for r in rr] for rr in reps]
    return rc, sm, W, out_rep


def feh_batch_graph_launches(batch):
    return load().feh_batch_graph_launches(batch)


def feh_plan_autotune(plan, reps=3):
    return _check(load().feh_plan_autotune(plan, int(reps)))


def feh_plan_cg_residual_spectral(plan):
    """True when the plan's CG keeps its residual as a last-axis half spectrum."""
    rc = load().feh_plan_cg_residual_spectral(plan)
    if rc < 0:
        raise FehError(rc, feh_last_error())
    return bool(rc)


def feh_plan_tuning(plan):
    """{'rows_last', 'pencils_mid', 'pencils_first', 'first_per_load_case', 'radices': [[..] per axis]}"""
    buf = (ctypes.c_int * 64)()
    n = load().feh_plan_tuning(plan, buf, 64)
    if n < 0:
        raise FehError(n, feh_last_error())
    v = list(buf[:n])
    rad, i = [], 5
    for _ in range(3):
        k = v[i]
        rad.append(v[i + 1:i + 1 + k])
        i += 1 + k
    return {"rows_last": v[0], "pencils_mid": v[1], "pencils_first": v[2], "first_per_load_case": v[3],
            "stencil_rows": v[4], "radices": rad, "compile_time_transforms": v[i]}


def feh_plan_set_tuning(plan, tuning):
    """Inverse of feh_plan_tuning: a dict with the same keys."""
    v = [int(tuning.get("rows_last", 0)), int(tuning.get("pencils_mid", 0)), int(tuning.get("pencils_first", 0)),
         int(tuning.get("first_per_load_case", 0)), int(tuning["stencil_rows"])]
    for r in list(tuning["radices"]) + [[]] * (3 - len(tuning["radices"])):
        v.append(len(r))
        v.extend(int(x) for x in r)
    if "compile_time_transforms" in tuning:
        v.append(int(tuning["compile_time_transforms"]))
    buf = (ctypes.c_int * len(v))(*v)
    return _check(load().feh_plan_set_tuning(plan, buf, len(v)))


PROFILE_KINDS = ["stencil", "alpha", "fft_last_fwd", "fft_middle_fwd", "fft_first_ksolve", "fft_middle_inv",
                 "fft_last_inv", "beta"]


def feh_profile_enable(plan, enable=True):
    return _check(load().feh_profile_enable(plan, 1 if enable else 0))


def feh_stream_copy(dst_ptr, src_ptr, nbytes, stream=None):
    """Nontemporal streaming copy of nbytes between device buffers (measurement)."""
    return _check(load().feh_stream_copy(dst_ptr, src_ptr, nbytes, stream))


def feh_profile_read(plan):
    """Returns {kind: (total_ms, launches)}."""
    n = len(PROFILE_KINDS)
    ms = np.zeros(n)
    cnt = (ctypes.c_int64 * n)()
    _check(load().feh_profile_read(plan, ms.ctypes.data_as(_dp), cnt, n))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROFILE_KINDS)}


def feh_effective_stiffness_weights(dim, Ebar, G):
    """dJ/dW for J = sum G_IJ C_eff_IJ (host helper of the C ABI)."""
    nv = 3 if dim == 2 else 6
    Eb = np.ascontiguousarray(Ebar, dtype=np.float64).reshape(nv, dim, dim)
    Gm = np.ascontiguousarray(G, dtype=np.float64).reshape(nv, nv)
    W = np.zeros((nv, nv))
    _check(load().feh_effective_stiffness_weights(dim, nv, Eb.ctypes.data_as(_dp), Gm.ctypes.data_as(_dp),
                                                  W.ctypes.data_as(_dp)))
    return W


def feh_energy_sensitivity(plan, weight, glam_ptr, gmu_ptr):
    w = np.ascontiguousarray(weight, dtype=np.float64)
    return _check(load().feh_energy_sensitivity(plan, w.ctypes.data_as(_dp), _vp(glam_ptr), _vp(gmu_ptr)))


def feh_energy_sensitivity_E(plan, weight, gE_ptr):
    w = np.ascontiguousarray(weight, dtype=np.float64)
    return _check(load().feh_energy_sensitivity_E(plan, w.ctypes.data_as(_dp), _vp(gE_ptr)))


def feh_apply_operator(plan, p_ptr, q_ptr):
    return _check(load().feh_apply_operator(plan, _vp(p_ptr), _vp(q_ptr)))


def feh_apply_preconditioner(plan, r_ptr, z_ptr):
    return _check(load().feh_apply_preconditioner(plan, _vp(r_ptr), _vp(z_ptr)))


def feh_apply_projection(plan, e_ptr, Ge_ptr):
    return _check(load().feh_apply_projection(plan, _vp(e_ptr), _vp(Ge_ptr)))


def feh_fft_forward(plan, x_ptr, X_ptr):
    return _check(load().feh_fft_forward(plan, _vp(x_ptr), _vp(X_ptr)))


def feh_fft_inverse(plan, X_ptr, x_ptr):
    return _check(load().feh_fft_inverse(plan, _vp(X_ptr), _vp(x_ptr)))


# --------------------------------------------------------------------------
# torch convenience wrapper
# --------------------------------------------------------------------------
class Homogenizer:
    """One plan bound to a torch device and stream, with a torch-owned workspace.

    shape: grid (Nx, Ny[, Nz]); n_load: load cases solved together (per
    microstructure); n_batch: microstructures of this shape in one plan (their
    materials stacked along a leading axis, load cases numbered
    b * n_load + j); precision: "fp64" or "fp32" (FP32 fields/FFT/stencils,
    FP64 CG scalars and per-wavevector inverses); h: voxel sizes (default 1).
    """

    def __init__(self, shape, n_load=1, precision="fp64", h=None, device="cuda", stream=None, n_batch=1):
        import torch
        self.torch = torch
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        self.N = int(np.prod(self.shape))
        self.n_batch = int(n_batch)
        self.n_per = int(n_load)
        self.n_load = self.n_batch * self.n_per  # load cases in the plan
        self.precision = precision
        self.prec = FEH_FP64 if precision == "fp64" else FEH_FP32
        self.dtype = torch.float64 if self.prec == FEH_FP64 else torch.float32
        self.device = torch.device(device)
        self.ne = 2 if self.dim == 2 else 6
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.plan = feh_plan_create_batch(self.dim, self.shape, h, self.n_batch, self.n_per, self.prec,
                                          stream.cuda_stream)
        nbytes = feh_plan_workspace_bytes(self.plan)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        feh_plan_set_workspace(self.plan, self.workspace.data_ptr(), self.workspace.numel())
        self._keep = []

    def _dev(self, x, dtype=None):
        t = self.torch.as_tensor(x, device=self.device, dtype=dtype or self.dtype)
        return t.contiguous()

    def set_material(self, E=None, nu=None, phases=None, table=None, lam=None, mu=None):
        """Either (E field, uniform nu), (phases, table[(E, nu)]), or (lam, mu) fields."""
        if lam is not None:
            l, m = self._dev(lam), self._dev(mu)
            feh_set_material_lame(self.plan, l.data_ptr(), m.data_ptr())
        elif phases is not None:
            ph = self._dev(phases, self.torch.int32)
            feh_set_material_phases(self.plan, ph.data_ptr(), np.asarray(table, dtype=np.float64))
        else:
            e = self._dev(E)
            feh_set_material_field(self.plan, e.data_ptr(), float(nu))
        self.stream.synchronize()

    def solve(self, Ebar, tol=1e-10, max_iter=1000, u0=None, fields=False, return_u=False):
        torch = self.torch
        Ebar = np.asarray(Ebar, dtype=np.float64).reshape(self.n_load, self.dim, self.dim)
        L, D, N, ne = self.n_load, self.dim, self.N, self.ne
        u = torch.empty((L, N, D), dtype=self.dtype, device=self.device) if return_u else None
        strain = stress = None
        if fields:
            strain = torch.empty((L, N, ne, D, D), dtype=self.dtype, device=self.device)
            stress = torch.empty_like(strain)
        u0t = self._dev(u0).reshape(L, N, D) if u0 is not None else None
        rc, smean, W, rep = feh_solve(self.plan, Ebar, tol, max_iter,
                                      u0t.data_ptr() if u0t is not None else 0,
                                      u.data_ptr() if u is not None else 0,
                                      strain.data_ptr() if strain is not None else 0,
                                      stress.data_ptr() if stress is not None else 0)
        out = dict(status=rc, stress_mean=smean, energy=W, report=rep, u=u, strain=strain, stress=stress)
        self._last_Ebar = Ebar
        nv = 3 if D == 2 else 6
        if self.n_per == nv:
            G = self.n_per
            Cs = []
            for b in range(self.n_batch):
                sl = slice(b * G, (b + 1) * G)
                try:
                    Cs.append(feh_effective_stiffness(D, Ebar[sl], W[sl, sl]))
                except FehError:
                    Cs.append(None)
            if self.n_batch == 1:
                if Cs[0] is not None:
                    out["C_eff"] = Cs[0]
            else:
                out["C_eff_batch"] = Cs
        return out

    def strain_cg_solve(self, Ebar, kind="fe", tol=1e-10, max_iter=1000, fields=False):
        """Projected CG in strain space with the derivative `kind` (one of
        DERIV_KINDS); the plan's material.  Returns a dict like solve (strain
        field [L, N, n_e, D, D] when fields) plus C_eff for nv load cases."""
        torch = self.torch
        k = DERIV_KINDS[kind] if isinstance(kind, str) else int(kind)
        Ebar = np.asarray(Ebar, dtype=np.float64).reshape(self.n_load, self.dim, self.dim)
        L, D, N = self.n_load, self.dim, self.N
        ne = feh_strain_cg_points(k, D)
        nbytes = feh_strain_cg_workspace_bytes(self.plan, k)
        work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        strain = torch.empty((L, N, ne, D, D), dtype=self.dtype, device=self.device) if fields else None
        rc, smean, W, rep = feh_strain_cg_solve(self.plan, k, Ebar, tol, max_iter, work.data_ptr(), nbytes,
                                                strain.data_ptr() if strain is not None else 0)
        out = dict(status=rc, stress_mean=smean, energy=W, report=rep, strain=strain)
        if self.n_per == (3 if D == 2 else 6) and self.n_batch == 1:
            try:
                out["C_eff"] = feh_effective_stiffness(D, Ebar, W)
            except FehError:
                pass
        return out

    def finite_strain_solve(self, Fbar, kind="fe", n_steps=1, newton_tol=1e-10, equil_tol=1e-11, cg_tol=1e-10,
                            max_newton=50, max_cg=5000, fields=False):
        """Finite-strain (Saint Venant-Kirchhoff) Newton + projected CG with the
        derivative `kind`; the plan's Lame constants.  Returns a dict with
        status, P_mean [L, D, D], report and, when fields, F and P
        [L, N, n_e, D, D]."""
        torch = self.torch
        k = DERIV_KINDS[kind] if isinstance(kind, str) else int(kind)
        Fbar = np.asarray(Fbar, dtype=np.float64).reshape(self.n_load, self.dim, self.dim)
        L, D, N = self.n_load, self.dim, self.N
        ne = feh_strain_cg_points(k, D)
        nbytes = feh_finite_strain_workspace_bytes(self.plan, k)
        work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        F = P = None
        if fields:
            F = torch.empty((L, N, ne, D, D), dtype=self.dtype, device=self.device)
            P = torch.empty_like(F)
        rc, pm, rep = feh_finite_strain_solve(self.plan, k, Fbar, n_steps, newton_tol, equil_tol, cg_tol, max_newton,
                                              max_cg, work.data_ptr(), nbytes,
                                              F.data_ptr() if F is not None else 0, P.data_ptr() if P is not None else 0)
        return dict(status=rc, P_mean=pm, report=rep, F=F, P=P)

    def autotune(self, reps=3):
        """Pick the FFT radix orders and launch geometry by timing (see feh_plan_autotune)."""
        feh_plan_autotune(self.plan, reps)
        return feh_plan_tuning(self.plan)

    def energy_sensitivity(self, weight):
        """Per-voxel (dJ/dlambda, dJ/dmu) for J = sum weight_lm W_lm of the last solve."""
        gshape = self.shape if self.n_batch == 1 else (self.n_batch,) + self.shape
        g_lam = self.torch.empty(gshape, dtype=self.dtype, device=self.device)
        g_mu = self.torch.empty_like(g_lam)
        feh_energy_sensitivity(self.plan, np.asarray(weight, dtype=np.float64).reshape(self.n_load, self.n_load),
                               g_lam.data_ptr(), g_mu.data_ptr())
        return g_lam, g_mu

    def energy_sensitivity_E(self, weight):
        """Per-voxel dJ/dE for J = sum weight_lm W_lm of the last solve (material
        set from an E field with a uniform nu)."""
        gshape = self.shape if self.n_batch == 1 else (self.n_batch,) + self.shape
        g_E = self.torch.empty(gshape, dtype=self.dtype, device=self.device)
        feh_energy_sensitivity_E(self.plan, np.asarray(weight, dtype=np.float64).reshape(self.n_load, self.n_load),
                                 g_E.data_ptr())
        return g_E

    def c_eff_sensitivity(self, G):
        """Per-voxel (dJ/dlambda, dJ/dmu) for J = sum G_IJ C_eff_IJ of the last solve
        (nv load cases per microstructure); G one nv x nv matrix, or one per
        microstructure for a batched plan."""
        nv, Gp = self.n_per, self.n_per
        Gs = np.asarray(G, dtype=np.float64)
        if Gs.ndim == 2:
            Gs = np.broadcast_to(Gs, (self.n_batch, nv, nv))
        W = np.zeros((self.n_load, self.n_load))
        for b in range(self.n_batch):
            sl = slice(b * Gp, (b + 1) * Gp)
            W[sl, sl] = feh_effective_stiffness_weights(self.dim, self._last_Ebar[sl], Gs[b])
        return self.energy_sensitivity(W)

    def apply_operator(self, p):
        p = self._dev(p).reshape(self.n_load, self.N, self.dim)
        q = self.torch.empty_like(p)
        feh_apply_operator(self.plan, p.data_ptr(), q.data_ptr())
        return q

    def apply_preconditioner(self, r):
        r = self._dev(r).reshape(self.n_load, self.N, self.dim)
        z = self.torch.empty_like(r)
        feh_apply_preconditioner(self.plan, r.data_ptr(), z.data_ptr())
        return z

    def apply_projection(self, e):
        e = self._dev(e).reshape(self.n_load, self.N, self.ne, self.dim, self.dim)
        g = self.torch.empty_like(e)
        feh_apply_projection(self.plan, e.data_ptr(), g.data_ptr())
        return g

    def fft_forward(self, x):
        x = self._dev(x).reshape(self.n_load * self.dim, self.N)
        nh = self.shape[-1] // 2 + 1
        cd = self.torch.complex128 if self.prec == FEH_FP64 else self.torch.complex64
        X = self.torch.empty((self.n_load * self.dim,) + self.shape[:-1] + (nh,), dtype=cd, device=self.device)
        feh_fft_forward(self.plan, x.data_ptr(), X.data_ptr())
        return X

    def fft_inverse(self, X):
        cd = self.torch.complex128 if self.prec == FEH_FP64 else self.torch.complex64
        X = self.torch.as_tensor(X, device=self.device, dtype=cd).contiguous()
        x = self.torch.empty((self.n_load * self.dim, self.N), dtype=self.dtype, device=self.device)
        feh_fft_inverse(self.plan, X.data_ptr(), x.data_ptr())
        return x

    def close(self):
        if self.plan is not None:
            feh_plan_destroy(self.plan)
            self.plan = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UnevenBatch:
    """Microstructures of uneven sizes solved together.

    maps: list of per-map materials (any grid shapes, one dimension), each
    either (E, nu) with a per-voxel Young's modulus array and a uniform
    Poisson ratio (set through feh_set_material_field), or (lam, mu) per-voxel
    Lame arrays (feh_set_material_lame); maps of one group must use one kind,
    and (E, nu) maps of a group one nu;
    maps of the same shape share a batched plan (at most 64 load cases per
    plan), and all plans form one ``feh_batch`` whose CG chunks run as
    captured HIP graphs.  The plans take up to ``n_streams`` dedicated streams
    in turn (default 4, the hardware queues a process gets by default), so
    the short kernels of different grids overlap; the plan with the most
    voxel-load-cases comes first (its kernels are enqueued first in every
    iteration: the batch's time is its chain's).  n_load load cases per map
    (default: the nv unit Voigt loads)."""

    def __init__(self, maps, n_load=None, precision="fp32", device="cuda", n_streams=4):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.dim = np.ndim(maps[0][0])
        nv = 3 if self.dim == 2 else 6
        self.n_load = int(n_load or nv)
        self.stream = torch.cuda.Stream(device=self.device)  # default priority
        cap = max(1, 64 // self.n_load)
        groups = {}
        for i, (lam, mu) in enumerate(maps):
            groups.setdefault(tuple(np.shape(lam)), []).append(i)
        n_plans = sum((len(idx) + cap - 1) // cap for idx in groups.values())
        self.streams = [self.stream] + [torch.cuda.Stream(device=self.device)  # default priority
                                        for _ in range(max(1, min(int(n_streams), n_plans)) - 1)]
        self.plans = []   # (Homogenizer, [map indices])
        self.where = {}   # map index -> (plan number, slot)
        # largest plans first (voxels x maps), ties by shape
        chunks = [(shape, idx[k:k + cap]) for shape, idx in groups.items() for k in range(0, len(idx), cap)]
        chunks.sort(key=lambda c: (-int(np.prod(c[0])) * len(c[1]), c[0]))
        with torch.cuda.stream(self.stream):
            for shape, part in chunks:
                hz = Homogenizer(shape, n_load=self.n_load, precision=precision, device=self.device,
                                 stream=self.streams[len(self.plans) % len(self.streams)],
                                 n_batch=len(part))
                a = np.stack([np.asarray(maps[i][0], dtype=np.float64) for i in part])
                if np.ndim(maps[part[0]][1]) == 0:
                    nus = {float(maps[i][1]) for i in part}
                    if len(nus) != 1:
                        raise ValueError("(E, nu) maps of one shape group need one nu")
                    hz.set_material(E=a, nu=nus.pop())
                else:
                    b = np.stack([np.asarray(maps[i][1], dtype=np.float64) for i in part])
                    hz.set_material(lam=a, mu=b)
                for s_, i in enumerate(part):
                    self.where[i] = (len(self.plans), s_)
                self.plans.append((hz, part))
        self.n_maps = len(maps)
        self.batch = feh_batch_create([hz.plan for hz, _ in self.plans])

    def solve(self, Ebar, tol=1e-5, max_iter=5000, use_graph=True):
        """Ebar: [n_load][D][D] for every map.  Returns a list per map with
        C_eff (when n_load = nv), stress_mean, energy block and reports."""
        Ebar = np.asarray(Ebar, dtype=np.float64).reshape(self.n_load, self.dim, self.dim)
        Ebs = [np.concatenate([Ebar] * hz.n_batch) for hz, _ in self.plans]
        for (hz, _), e in zip(self.plans, Ebs):
            hz._last_Ebar = e
        rc, sm, W, rep = feh_batch_solve(self.batch, Ebs, tol, max_iter, use_graph)
        for s in self.streams:
            s.synchronize()
        G = self.n_load
        nv = 3 if self.dim == 2 else 6
        out = [None] * self.n_maps
        for p, (hz, part) in enumerate(self.plans):
            for s_, i in enumerate(part):
                sl = slice(s_ * G, (s_ + 1) * G)
                r = dict(stress_mean=sm[p][sl], energy=W[p][sl, sl], report=rep[p][sl], status=rc)
                if G == nv:
                    r["C_eff"] = feh_effective_stiffness(self.dim, Ebar, W[p][sl, sl])
                out[i] = r
        return out

    def graph_launches(self):
        return feh_batch_graph_launches(self.batch)

    def energy_sensitivity_E(self, weight):
        """Per-voxel dJ/dE for J = sum weight_lm W_lm of the last solve (material
        set from an E field with a uniform nu)."""
        gshape = self.shape if self.n_batch == 1 else (self.n_batch,) + self.shape
        g_E = self.torch.empty(gshape, dtype=self.dtype, device=self.device)
        feh_energy_sensitivity_E(self.plan, np.asarray(weight, dtype=np.float64).reshape(self.n_load, self.n_load),
                                 g_E.data_ptr())
        return g_E

    def c_eff_sensitivity(self, G):
        """Per map (dJ/dlambda, dJ/dmu) for J = sum G_IJ C_eff_IJ (one nv x nv G
        for every map) after solve()."""
        res = [None] * self.n_maps
        for hz, part in self.plans:
            gl, gm = hz.c_eff_sensitivity(G)
            if hz.n_batch == 1:
                gl, gm = gl[None], gm[None]
            for s_, i in enumerate(part):
                res[i] = (gl[s_], gm[s_])
        return res

    def close(self):
        if self.batch is not None:
            feh_batch_destroy(self.batch)
            self.batch = None
        for hz, _ in self.plans:
            hz.close()
        self.plans = []

