"""Pins of the finite-strain oracle (material law, gradient projection,
Newton + projected CG) against definitions it does not share code with:

  * P is the derivative of the strain energy W(F) (central differences) and
    the tangent action is the derivative of P; P(R F) = R P(F) for rotations.
  * The gradient projection is idempotent and self-adjoint, leaves gradients
    of periodic displacements unchanged, and for the FE kind its range is the
    element gradients of nodal fields (brute force on a tiny grid).
  * The FE kind reaches the canonical nonlinear FE solution (assembled
    residual and tangent, sparse LU Newton) field by field.
  * Uniform material: F = Fbar.  Laminates: the rank-one closed form (layer
    gradients Fbar + (1 - f) a (x) n and Fbar - f a (x) n with continuous
    traction P n, solved for a by a small Newton) for every kind whose symbol
    is non-zero on the laminate axis.
  * Objectivity of the whole solve: Fbar -> R Fbar gives F -> R F.
  * Small-strain limit: (F - I) / delta tends to the small-strain solution.
  * Load stepping does not change the converged solution.
"""
import numpy as np
import pytest

import microstructures as ms
from oracle import fe, finite, pcg, projection


def _rand_F(rng, shape, amp=0.15):
    return np.eye(shape[-1]) + amp * rng.standard_normal(shape)


def _rot2(t):
    return np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])


def _rot3(a, b):
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(b), -np.sin(b)], [0, np.sin(b), np.cos(b)]])
    return Rz @ Rx


@pytest.mark.parametrize("D", [2, 3])
def test_pk1_is_energy_derivative_and_tangent_is_its_derivative(D):
    rng = np.random.default_rng(D)
    lam, mu = np.array([1.3]), np.array([0.7])
    F = _rand_F(rng, (1, D, D))
    P = finite.pk1(lam, mu, F)
    eps = 1e-6
    for i in range(D):
        for a in range(D):
            dF = np.zeros_like(F)
            dF[0, i, a] = eps
            num = (finite.energy(lam, mu, F + dF) - finite.energy(lam, mu, F - dF)) / (2 * eps)
            assert num[0] == pytest.approx(P[0, i, a], rel=1e-7, abs=1e-9)
    X = rng.standard_normal((1, D, D))
    num = (finite.pk1(lam, mu, F + eps * X) - finite.pk1(lam, mu, F - eps * X)) / (2 * eps)
    np.testing.assert_allclose(finite.tangent_apply(lam, mu, F, X), num, rtol=1e-7, atol=1e-9)
    K = finite.tangent_matrix(lam, mu, F)
    np.testing.assert_allclose(np.einsum("niakb,nkb->nia", K, X), num, rtol=1e-7, atol=1e-9)
    R = _rot2(0.4) if D == 2 else _rot3(0.4, -0.9)
    np.testing.assert_allclose(finite.pk1(lam, mu, R @ F), R @ P, atol=1e-13)
    # small strain: P linearises to C : sym(H)
    H = 1e-7 * rng.standard_normal((1, D, D))
    sig = fe.stress_of(lam, mu, 0.5 * (H + np.swapaxes(H, 1, 2)))
    np.testing.assert_allclose(finite.pk1(lam, mu, np.eye(D) + H), sig, rtol=0, atol=1e-5 * np.abs(sig).max())


@pytest.mark.parametrize("kind,shape", [("fe", (5, 4)), ("fd", (6, 5)), ("fourier", (5, 7)), ("fourier2", (5, 5)),
                                        ("fe", (3, 4, 3)), ("cd", (5, 5))])
def test_gradient_projection_properties(kind, shape):
    rng = np.random.default_rng(3)
    D = len(shape)
    g = finite.projector(kind, shape)
    ne = g.shape[0] // D
    X = rng.standard_normal(shape + (ne, D, D))
    Y = rng.standard_normal(shape + (ne, D, D))
    GX = finite.apply_gradient_projection(g, X)
    np.testing.assert_allclose(finite.apply_gradient_projection(g, GX), GX, atol=1e-12)
    assert np.sum(GX * Y) == pytest.approx(np.sum(X * finite.apply_gradient_projection(g, Y)), rel=1e-11)
    np.testing.assert_allclose(GX.mean(axis=tuple(range(D))), 0.0, atol=1e-13)
    if kind == "fe":
        # element gradients of a nodal field are compatible: G leaves them unchanged
        u = rng.standard_normal((int(np.prod(shape)), D))
        Ge = fe.element_gradients(u, shape).reshape(shape + (ne, D, D))
        np.testing.assert_allclose(finite.apply_gradient_projection(g, Ge), Ge, atol=1e-12)
        # and the range has the dimension of the zero-mean nodal fields
        B = []
        for j in range(int(np.prod(shape)) * D):
            e = np.zeros(int(np.prod(shape)) * D)
            e[j] = 1.0
            B.append(fe.element_gradients(e, shape).ravel())
        rank = np.linalg.matrix_rank(np.array(B), tol=1e-9)
        assert rank == (int(np.prod(shape)) - 1) * D
        tr = sum(np.sum(finite.apply_gradient_projection(g, np.eye(ne * D * D * int(np.prod(shape)))[j]
                                                         .reshape(shape + (ne, D, D))).ravel()[j])
                 for j in range(ne * D * D * int(np.prod(shape))))
        assert tr == pytest.approx(rank, abs=1e-8)


@pytest.mark.parametrize("shape", [(6, 5), (4, 3, 5)])
def test_fe_kind_equals_canonical_nonlinear_fe(shape):
    rng = np.random.default_rng(5)
    D = len(shape)
    E = rng.uniform(1.0, 10.0, shape)
    nu = rng.uniform(0.1, 0.4, shape)
    lam, mu = fe.lame(E, nu)
    Fbar = np.eye(D) + np.diag(rng.uniform(-0.1, 0.1, D)) + 0.05 * rng.standard_normal((D, D))
    F, nit, cit = finite.solve(lam, mu, Fbar, "fe", newton_tol=1e-12, equil_tol=1e-13, cg_tol=1e-10)
    Fref = finite.fe_solve(lam, mu, Fbar, tol=1e-13)
    np.testing.assert_allclose(F, Fref, atol=1e-10)
    assert nit < 12
    np.testing.assert_allclose(F.mean(axis=tuple(range(D + 1))), Fbar, atol=1e-13)


@pytest.mark.parametrize("kind", ["fe", "fd", "cd", "ls", "fourier", "fourier2"])
def test_uniform_material_gives_uniform_F(kind):
    shape = (5, 6) if kind in ("fe", "fd") else (5, 7)
    lam, mu = fe.lame(np.full(shape, 2.0), np.full(shape, 0.3))
    Fbar = np.array([[1.1, 0.03], [-0.02, 0.95]])
    F, _, _ = finite.solve(lam, mu, Fbar, kind)
    np.testing.assert_allclose(F, np.broadcast_to(Fbar, F.shape), atol=1e-14)


def _laminate_rank_one(P1, P2, Fbar, f, n, D):
    """a with P1(Fbar + (1-f) a n) n = P2(Fbar - f a n) n (Newton, FD Jacobian)."""
    a = np.zeros(D)
    for _ in range(50):
        def res(a):
            F1 = Fbar + (1 - f) * np.outer(a, n)
            F2 = Fbar - f * np.outer(a, n)
            return P1(F1) @ n - P2(F2) @ n
        r = res(a)
        J = np.zeros((D, D))
        for k in range(D):
            e = np.zeros(D)
            e[k] = 1e-7
            J[:, k] = (res(a + e) - res(a - e)) / 2e-7
        da = np.linalg.solve(J, -r)
        a += da
        if np.linalg.norm(da) < 1e-15:
            break
    return Fbar + (1 - f) * np.outer(a, n), Fbar - f * np.outer(a, n)


@pytest.mark.parametrize("kind,shape,axis", [("fe", (6, 5), 0), ("fe", (5, 6), 1), ("fd", (6, 5), 0),
                                             ("fourier", (7, 5), 0), ("ls", (6, 5), 1), ("cd", (7, 5), 0),
                                             ("fe", (4, 3, 5), 2), ("fd", (5, 4, 3), 0)])
def test_laminate_rank_one_closed_form(kind, shape, axis):
    D = len(shape)
    nl = 2
    m = ms.laminate(shape, axis, nl, E=(1.0, 6.0), nu=(0.3, 0.2))
    lam, mu = fe.lame(m.E, m.nu)
    rng = np.random.default_rng(axis + 10 * D)
    Fbar = np.eye(D) + 0.08 * rng.standard_normal((D, D))
    F, _, _ = finite.solve(lam, mu, Fbar, kind, newton_tol=1e-12, equil_tol=1e-13, cg_tol=1e-10)
    l1, m1 = fe.lame(6.0, 0.2)
    l2, m2 = fe.lame(1.0, 0.3)
    P1 = lambda X: finite.pk1(np.array([l1]), np.array([m1]), X[None])[0]
    P2 = lambda X: finite.pk1(np.array([l2]), np.array([m2]), X[None])[0]
    n = np.zeros(D)
    n[axis] = 1.0
    F1, F2 = _laminate_rank_one(P1, P2, Fbar, nl / shape[axis], n, D)
    idx = [slice(None)] * D
    idx[axis] = slice(0, nl)
    layer1 = F[tuple(idx)]
    idx[axis] = slice(nl, None)
    layer2 = F[tuple(idx)]
    np.testing.assert_allclose(layer1, np.broadcast_to(F1, layer1.shape), atol=1e-11)
    np.testing.assert_allclose(layer2, np.broadcast_to(F2, layer2.shape), atol=1e-11)


@pytest.mark.parametrize("kind,shape", [("fe", (5, 4)), ("fourier", (5, 5)), ("fe", (3, 3, 4))])
def test_objectivity_of_the_solution(kind, shape):
    rng = np.random.default_rng(8)
    D = len(shape)
    lam, mu = fe.lame(rng.uniform(1, 5, shape), np.full(shape, 0.3))
    Fbar = np.eye(D) + 0.07 * rng.standard_normal((D, D))
    R = _rot2(0.7) if D == 2 else _rot3(0.7, 0.3)
    F, _, _ = finite.solve(lam, mu, Fbar, kind, newton_tol=1e-12, equil_tol=1e-13, cg_tol=1e-10)
    FR, _, _ = finite.solve(lam, mu, R @ Fbar, kind, newton_tol=1e-12, equil_tol=1e-13, cg_tol=1e-10)
    np.testing.assert_allclose(FR, R @ F, atol=1e-10)


@pytest.mark.parametrize("kind", ["fe", "fd", "fourier"])
def test_small_strain_limit(kind):
    # odd grid for the Fourier derivative (its real-field operator is not a
    # projection at Nyquist indices of even axes)
    shape = (7, 5) if kind == "fourier" else (6, 5)
    rng = np.random.default_rng(4)
    lam, mu = fe.lame(rng.uniform(1, 5, shape), rng.uniform(0.1, 0.4, shape))
    Eb = np.array([[0.4, 0.3], [0.3, -0.2]])
    delta = 1e-6
    F, _, _ = finite.solve(lam, mu, np.eye(2) + delta * Eb, kind, newton_tol=1e-13, equil_tol=1e-14, cg_tol=1e-11)
    e, _, _ = pcg.solve(lam, mu, Eb, kind=kind, tol=1e-14)
    H = (F - np.eye(2)) / delta
    np.testing.assert_allclose(0.5 * (H + np.swapaxes(H, -1, -2)), e, atol=1e-5)


def test_load_steps_reach_the_same_solution():
    shape = (5, 6)
    rng = np.random.default_rng(6)
    lam, mu = fe.lame(rng.uniform(1, 5, shape), np.full(shape, 0.33))
    Fbar = np.diag([1.1, 1.1])
    F1, _, _ = finite.solve(lam, mu, Fbar, "fe", n_steps=1, newton_tol=1e-12, equil_tol=1e-13, cg_tol=1e-10)
    F4, _, _ = finite.solve(lam, mu, Fbar, "fe", n_steps=4, newton_tol=1e-12, equil_tol=1e-13, cg_tol=1e-10)
    np.testing.assert_allclose(F4, F1, atol=1e-11)


# ---------------------------------------------------------------------------
# the paper's finite-strain examples (Sec. "Single voxel inhomogeneity",
# Sec. "Two pillars and vacuum"): the qualitative statements it makes
# ---------------------------------------------------------------------------
def test_single_voxel_symmetry_lines():
    """17 x 17, soft centre voxel (E/10, nu = 0.33), 10 % biaxial stretch: the
    one-point symmetric stencils (Fourier, central differences, least squares)
    give P_xy = 0 on the row and column through the inhomogeneity; forward
    differences (asymmetric stencil), the two-point Fourier derivative and FE
    (two evaluation points per voxel) do not."""
    m = ms.single_voxel()
    lam, mu = fe.lame(m.E, m.nu)
    Fbar = np.diag([1.1, 1.1])
    for kind in ("fe", "fd", "cd", "ls", "fourier", "fourier2"):
        F, _, _ = finite.solve(lam, mu, Fbar, kind)
        P = finite.pk1(lam, mu, F)
        line = max(np.abs(P[8, :, :, 0, 1]).max(), np.abs(P[:, 8, :, 0, 1]).max())
        if kind in ("cd", "ls", "fourier"):
            assert line < 1e-14, (kind, line)
        else:
            assert line > 1e-3, (kind, line)


def test_two_pillars_decoupling():
    """17 x 17: vacuum columns (E = 0) at x = 0 and x = 8, a 7-column pillar
    with a soft 3-voxel line and an 8-column pillar, 10 % stretch along y at
    fixed width: forward differences, least squares and FE decouple the
    pillars through the vacuum (no shear stress in the right pillar); the
    Fourier derivatives and central differences (stencils reaching across the
    vacuum column) do not.  The vacuum carries no stress."""
    m = ms.two_pillars()
    lam, mu = fe.lame(m.E, m.nu)
    Fbar = np.diag([1.0, 1.1])
    for kind in ("fe", "fd", "cd", "ls", "fourier", "fourier2"):
        F, _, _ = finite.solve(lam, mu, Fbar, kind, equil_tol=1e-8)
        P = finite.pk1(lam, mu, F)
        right = np.abs(P[9:, :, :, 0, 1]).max()
        assert np.abs(P[0]).max() == 0.0 and np.abs(P[8]).max() == 0.0
        assert np.abs(P[1:8, :, :, 0, 1]).max() > 1e-3
        if kind in ("fe", "fd", "ls"):
            assert right < 1e-9, (kind, right)
        else:
            assert right > 1e-4, (kind, right)


def test_fourier_kinds_need_odd_grids():
    """Sec. "Even vs. odd number of grid points": the Fourier-derivative
    projection is exact only on odd grids; finite strain refuses even axes."""
    lam, mu = np.full((6, 5), 1.0), np.full((6, 5), 1.0)
    for kind in ("fourier", "fourier2"):
        with pytest.raises(ValueError):
            finite.solve(lam, mu, np.eye(2), kind)
    F, _, _ = finite.solve(np.full((5, 5), 1.0), np.full((5, 5), 1.0), np.diag([1.05, 1.0]), "fourier")
    np.testing.assert_allclose(F.mean(axis=(0, 1, 2)), np.diag([1.05, 1.0]), atol=1e-14)
