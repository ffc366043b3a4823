"""Pins of the FE oracle (assembly, solve, post-processing) against exact
solutions, closed forms, brute force and the paper's projected CG."""
import itertools
import json
import os

import numpy as np
import pytest

import microstructures as ms
from oracle import fe, pcg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _voigt_C(lam, mu, dim):
    nv = 3 if dim == 2 else 6
    C = np.zeros((nv, nv))
    C[:dim, :dim] = lam
    C[np.arange(dim), np.arange(dim)] += 2 * mu
    C[np.arange(dim, nv), np.arange(dim, nv)] = mu
    return C


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(6, 5), (4, 3, 5)])
def test_homogeneous_exact(shape):
    """Uniform material: f = 0, the fluctuation vanishes, e = Ebar, s = C Ebar."""
    dim = len(shape)
    E = np.full(shape, 2.5)
    nu = np.full(shape, 0.27)
    Eb = ms.unit_loads(dim)
    rng = np.random.default_rng(0)
    Eb = Eb + 0.003 * np.array([0.5 * (a + a.T) for a in rng.standard_normal(Eb.shape)])
    out = fe.homogenize(E, nu, Eb)
    lam, mu = fe.lame(2.5, 0.27)
    for l in range(len(Eb)):
        f = fe.load_vector(fe.lame(E, nu)[0], fe.lame(E, nu)[1], Eb[l])
        assert np.abs(f).max() < 1e-15
        assert np.abs(out["u"][l]).max() < 1e-15
        np.testing.assert_allclose(out["eps"][l], np.broadcast_to(Eb[l], out["eps"][l].shape), atol=1e-16)
        s = lam * np.trace(Eb[l]) * np.eye(dim) + 2 * mu * Eb[l]
        np.testing.assert_allclose(out["sig_mean"][l], s, atol=1e-15)
    np.testing.assert_allclose(out["C_eff"], _voigt_C(lam, mu, dim), atol=1e-13)


@pytest.mark.parametrize("shape", [(4, 4), (3, 4, 3)])
def test_stiffness_symmetric_psd_translation_kernel(shape):
    dim = len(shape)
    rng = np.random.default_rng(3)
    lam, mu = fe.lame(rng.uniform(1, 3, shape), np.full(shape, 0.3))
    K = fe.assemble(lam, mu).toarray()
    np.testing.assert_allclose(K, K.T, atol=1e-14)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-12) == dim
    assert ev.min() > -1e-12
    for i in range(dim):
        t = np.zeros((K.shape[0] // dim, dim))
        t[:, i] = 1
        assert np.abs(K @ t.ravel()).max() < 1e-13


def _affine_gradient(X, U):
    """Gradient of the affine map through simplex vertices X -> values U,
    solved from the D+1 interpolation conditions (independent of the
    shape-function gradients used by the oracle)."""
    dim = X.shape[1]
    A = np.hstack([X, np.ones((dim + 1, 1))])
    coef = np.linalg.solve(A, U)          # U = X grad^T + c
    return coef[:dim].T                   # grad[i, a]


def _energy(u, lam, mu, shape, h):
    """Total strain energy 1/2 sum_e |e| e:C:e, strains by affine fit."""
    dim = len(shape)
    u = u.reshape(-1, dim)
    tot = 0.0
    for vox in itertools.product(*[range(n) for n in shape]):
        vidx = np.ravel_multi_index(vox, shape)
        for verts in fe.element_vertices(dim):
            X = verts * h
            nodes = [np.ravel_multi_index(tuple((np.array(vox) + v) % shape), shape) for v in verts]
            G = _affine_gradient(X, u[nodes])
            e = 0.5 * (G + G.T)
            s = lam[vidx] * np.trace(e) * np.eye(dim) + 2 * mu[vidx] * e
            vol = abs(np.linalg.det((X[1:] - X[0]).T)) / (2 if dim == 2 else 6)
            tot += 0.5 * vol * np.sum(e * s)
    return tot


@pytest.mark.parametrize("shape,h", [((3, 4), (1.0, 1.3)), ((2, 3, 2), (1.0, 0.8, 1.2))])
def test_stiffness_brute_force_energy(shape, h):
    """K_ij = Pi(e_i + e_j) - Pi(e_i) - Pi(e_j) for the quadratic energy Pi,
    evaluated element by element with strains from an affine fit."""
    dim = len(shape)
    h = np.array(h)
    rng = np.random.default_rng(7)
    lam, mu = fe.lame(rng.uniform(1, 4, shape), rng.uniform(0.1, 0.4, shape))
    lamf, muf = lam.ravel(), mu.ravel()
    n = int(np.prod(shape)) * dim
    K = fe.assemble(lam, mu, h).toarray()
    Pi1 = np.zeros(n)
    I = np.eye(n)
    for i in range(n):
        Pi1[i] = _energy(I[i], lamf, muf, shape, h)
    Kb = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            Kb[i, j] = Kb[j, i] = _energy(I[i] + I[j], lamf, muf, shape, h) - Pi1[i] - Pi1[j]
    np.testing.assert_allclose(K, Kb, atol=1e-12 * np.abs(K).max())
    # load vector: f = -dPi(u; Ebar)/du at u = 0 with the strain Ebar added
    Eb = np.array([[0.3, 0.1, 0.05], [0.1, -0.2, 0.07], [0.05, 0.07, 0.11]])[:dim, :dim]
    f = fe.load_vector(lam, mu, Eb, h)
    pos = np.stack(np.indices(shape), axis=-1).reshape(-1, dim) * h
    # Pi(Ebar x + u) restricted to one element is the energy of the affine
    # field; its gradient in u is K u - f (no periodic seam for the uniform
    # strain because only gradients enter).  Check K u - f by central
    # differences of the energy of (u + Ebar-strain) built per element:
    def Pi_shift(u):
        tot = 0.0
        uu = u.reshape(-1, dim)
        for vox in itertools.product(*[range(nn) for nn in shape]):
            vidx = np.ravel_multi_index(vox, shape)
            for verts in fe.element_vertices(dim):
                X = verts * h
                nodes = [np.ravel_multi_index(tuple((np.array(vox) + v) % shape), shape) for v in verts]
                G = _affine_gradient(X, uu[nodes]) + Eb
                e = 0.5 * (G + G.T)
                s = lamf[vidx] * np.trace(e) * np.eye(dim) + 2 * muf[vidx] * e
                vol = abs(np.linalg.det((X[1:] - X[0]).T)) / (2 if dim == 2 else 6)
                tot += 0.5 * vol * np.sum(e * s)
        return tot
    grad = np.array([(Pi_shift(0.5 * I[i]) - Pi_shift(-0.5 * I[i])) for i in range(n)])
    np.testing.assert_allclose(grad, -f, atol=1e-12 * np.abs(f).max())
    del pos


def _laminate_closed_form(C1, C2, frac1, dim, axis):
    """Partial-inversion closed form of a layered medium with normal e_axis:
    continuity of the tangential strains and of the normal tractions."""
    pairs = fe.VOIGT_PAIRS[dim]
    Nset = [v for v, (a, b) in enumerate(pairs) if axis in (a, b)]
    Tset = [v for v in range(len(pairs)) if v not in Nset]
    def blocks(C):
        return (C[np.ix_(Nset, Nset)], C[np.ix_(Nset, Tset)], C[np.ix_(Tset, Nset)], C[np.ix_(Tset, Tset)])
    fr = [frac1, 1 - frac1]
    Bs = [blocks(C1), blocks(C2)]
    avg = lambda f: sum(w * f(*b) for w, b in zip(fr, Bs))
    A = np.linalg.inv(avg(lambda nn, nt, tn, tt: np.linalg.inv(nn)))
    Q = avg(lambda nn, nt, tn, tt: np.linalg.inv(nn) @ nt)
    P = avg(lambda nn, nt, tn, tt: tn @ np.linalg.inv(nn))
    Ctt = avg(lambda nn, nt, tn, tt: tt - tn @ np.linalg.inv(nn) @ nt) + P @ A @ Q
    C = np.zeros_like(C1)
    C[np.ix_(Nset, Nset)] = A
    C[np.ix_(Nset, Tset)] = A @ Q
    C[np.ix_(Tset, Nset)] = (A @ Q).T
    C[np.ix_(Tset, Tset)] = Ctt
    return C


@pytest.mark.parametrize("shape,axis", [((8, 6), 0), ((6, 8), 1), ((6, 4, 5), 0), ((4, 6, 5), 1),
                                        ((4, 5, 6), 2)])
@pytest.mark.parametrize("nus", [(0.3, 0.2), (0.0, 0.0)])
def test_laminate_closed_form(shape, axis, nus):
    """Layers with interfaces on voxel faces: the FE solution is exact, so
    C_eff equals the laminate closed form; with nu = 0 the normal stiffness is
    the Reuss (harmonic) and the in-plane stiffness the Voigt (arithmetic)
    mean, and the shear across the layers the harmonic mean of mu."""
    dim = len(shape)
    nl = 3 if shape[axis] > 5 else 2
    m = ms.laminate(shape, axis, nl, E=(1.0, 7.0), nu=nus)
    out = fe.homogenize(m.E, m.nu, ms.unit_loads(dim))
    frac1 = nl / shape[axis]
    lam1, mu1 = fe.lame(7.0, nus[1])
    lam2, mu2 = fe.lame(1.0, nus[0])
    C1, C2 = _voigt_C(lam1, mu1, dim), _voigt_C(lam2, mu2, dim)
    ref = _laminate_closed_form(C1, C2, frac1, dim, axis)
    np.testing.assert_allclose(out["C_eff"], ref, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(out["C_eff_stress"], ref, atol=1e-12 * np.abs(ref).max())
    if nus == (0.0, 0.0):
        reuss = 1 / (frac1 / 7.0 + (1 - frac1) / 1.0)
        voigt = frac1 * 7.0 + (1 - frac1) * 1.0
        assert out["C_eff"][axis, axis] == pytest.approx(reuss, rel=1e-12)
        for t in range(dim):
            if t != axis:
                assert out["C_eff"][t, t] == pytest.approx(voigt, rel=1e-12)
        mu_h = 1 / (frac1 / mu1 + (1 - frac1) / mu2)
        pairs = fe.VOIGT_PAIRS[dim]
        for v, (a, b) in enumerate(pairs):
            if a != b and axis in (a, b):
                assert out["C_eff"][v, v] == pytest.approx(mu_h, rel=1e-12)


def test_circle_anchor_and_symmetry():
    """32x32 circle (R = 8, contrast 10, nu = 0.3, plane strain): square
    symmetry of the anti-diagonal split gives C11 = C22 and C13 = C23; C_eff is
    symmetric positive definite, inside the Voigt/Reuss bounds; both C_eff
    forms agree.  The anchor values were computed independently (separate
    scratch code, same conventions) before this oracle existed; they are not
    from the paper."""
    m, Eb1, _, _ = ms.workload("circle32")
    out = fe.homogenize(m.E, m.nu, ms.unit_loads(2))
    C = out["C_eff"]
    anchor = json.load(open(os.path.join(GOLDEN, "circle32_anchor.json")))
    np.testing.assert_allclose(C, np.array(anchor["C_eff"]), rtol=0, atol=2e-9)
    np.testing.assert_allclose(out["sig_mean"][0], np.array(anchor["sig_mean_exx"]), rtol=0, atol=2e-11)
    assert C[0, 0] == pytest.approx(C[1, 1], rel=1e-13)
    assert C[0, 2] == pytest.approx(C[1, 2], rel=1e-11)
    np.testing.assert_allclose(C, C.T, atol=1e-13)
    assert np.linalg.eigvalsh(C).min() > 0
    np.testing.assert_allclose(out["C_eff_stress"], C, atol=1e-11)
    _check_bounds(m, C, 2)


def _check_bounds(m, C, dim):
    lam, mu = fe.lame(m.E, m.nu)
    Cs = [_voigt_C(l, u, dim) for l, u in zip(lam.ravel(), mu.ravel())]
    Cv = np.mean(Cs, axis=0)
    Cr = np.linalg.inv(np.mean([np.linalg.inv(c) for c in Cs], axis=0))
    assert np.linalg.eigvalsh(Cv - C).min() > -1e-12
    assert np.linalg.eigvalsh(C - Cr).min() > -1e-12


def test_3d_bounds_and_symmetry():
    m = ms.rsa_spheres(10, 7, (1.5, 2.5), 0.15)
    out = fe.homogenize(m.E, m.nu, ms.unit_loads(3))
    C = out["C_eff"]
    np.testing.assert_allclose(C, C.T, atol=1e-13)
    np.testing.assert_allclose(out["C_eff_stress"], C, atol=1e-10)
    _check_bounds(m, C, 3)


@pytest.mark.parametrize("case", ["circle8", "odd6x5", "cube4", "box543"])
def test_projected_cg_equals_fe(case):
    """The paper's method (projected CG in strain space with the small-strain
    FE projection) reaches the canonical FE solution (abstract; Sec. "Linear
    finite elements"), field by field."""
    rng = np.random.default_rng(9)
    if case == "circle8":
        m = ms.circle(8, 2.5)
    elif case == "odd6x5":
        m = ms.Micro(E=rng.uniform(1, 10, (6, 5)), nu=rng.uniform(0.1, 0.4, (6, 5)), phase=None, recipe="")
    elif case == "cube4":
        m = ms.sphere(4, 1.2)
    else:
        m = ms.Micro(E=rng.uniform(1, 10, (5, 4, 3)), nu=np.full((5, 4, 3), 0.3), phase=None, recipe="")
    dim = m.dim
    lam, mu = fe.lame(m.E, m.nu)
    A = rng.standard_normal((dim, dim)) * 0.01
    Eb = 0.5 * (A + A.T)
    e, it, hist = pcg.solve(lam, mu, Eb, tol=1e-13)
    ref = fe.homogenize(m.E, m.nu, [Eb])
    np.testing.assert_allclose(pcg.flat_fields(e), ref["eps"][0], atol=1e-14)
    np.testing.assert_allclose(pcg.average_stress(lam, mu, e), ref["sig_mean"][0], atol=1e-15)


def test_iteration_count_size_independent():
    """Sec. "Linear finite elements": the FE projection has a condition number
    independent of system size, so the iteration count stays flat under mesh
    refinement of the same geometry."""
    its = []
    for n in (16, 32, 64):
        m = ms.circle(n, n / 4.0)
        lam, mu = fe.lame(m.E, m.nu)
        _, it, _ = pcg.solve(lam, mu, np.array([[0.01, 0], [0, 0]]), tol=1e-10)
        its.append(it)
    assert max(its) - min(its) <= 4, its
    assert max(its) < 60


def test_c_cg_matches_direct():
    m = ms.circle(16, 5.0)
    Eb = ms.unit_loads(2)
    d = fe.homogenize(m.E, m.nu, Eb)
    c = fe.homogenize(m.E, m.nu, Eb, method="ccg", tol=1e-14)
    np.testing.assert_allclose(c["C_eff"], d["C_eff"], rtol=0, atol=1e-12)
    for l in range(3):
        np.testing.assert_allclose(c["u"][l], d["u"][l], atol=1e-11)


@pytest.mark.parametrize("shape", [(7, 6), (5, 4, 6)])
def test_local_evaluation_matches_assembly(shape):
    dim = len(shape)
    rng = np.random.default_rng(12)
    lam, mu = fe.lame(rng.uniform(0.5, 3, shape), rng.uniform(0.1, 0.4, shape))
    K = fe.assemble(lam, mu)
    p = rng.standard_normal(int(np.prod(shape)) * dim)
    q = (K @ p).reshape(-1, dim)
    nodes = rng.choice(int(np.prod(shape)), 10, replace=False)
    np.testing.assert_allclose(fe.apply_K_at_nodes(lam, mu, p, nodes), q[nodes], atol=1e-13)
    Eb = np.eye(dim) * 0.01
    Eb[0, 1] = Eb[1, 0] = 0.004
    f = fe.load_vector(lam, mu, Eb).reshape(-1, dim)
    np.testing.assert_allclose(fe.load_at_nodes(lam, mu, Eb, nodes), f[nodes], atol=1e-15)


@pytest.mark.parametrize("shape,h", [((5, 4), (1.0, 1.0)), ((6, 3), (0.7, 1.9)), ((3, 4, 5), (1.0, 1.0, 1.0)),
                                     ((4, 3, 5), (1.3, 0.6, 2.1))])
def test_element_strains_at_matches_fields(shape, h):
    """Local strain evaluation at selected voxels equals the full-field
    post-processing there (ragged and non-unit grids; first and last voxels)."""
    dim = len(shape)
    N = int(np.prod(shape))
    rng = np.random.default_rng(11)
    u = rng.standard_normal((N, dim))
    Eb = rng.standard_normal((dim, dim))
    Eb = 0.5 * (Eb + Eb.T)
    lam = np.ones(shape)
    eps, _ = fe.fields(u, lam, lam, Eb, h)
    vox = np.array([0, N - 1, N // 2, 1, N - 2])
    loc = fe.element_strains_at(u, shape, vox, Eb, h)
    np.testing.assert_allclose(loc, eps[vox], rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape,h", [((5, 4), (1.0, 1.0)), ((6, 3), (0.7, 1.9)), ((3, 4, 5), (1.0, 1.0, 1.0)),
                                     ((4, 4, 4), (1.3, 0.6, 2.1)), ((2, 3, 2), (1.0, 1.0, 1.0))])
def test_structured_assembly_equals_triplet_assembly(shape, h):
    """The node-neighbour assembly used for large grids gives the triplet
    assembly's matrix entry by entry (axes of length 2 included, where two
    neighbour offsets reach the same node)."""
    rng = np.random.default_rng(13)
    lam = rng.uniform(0.5, 3.0, shape)
    mu = rng.uniform(0.5, 3.0, shape)
    K = fe.assemble(lam, mu, h).toarray()
    Ks = fe.assemble_structured(lam, mu, h).toarray()
    np.testing.assert_allclose(Ks, K, rtol=0, atol=1e-13 * np.abs(K).max())
