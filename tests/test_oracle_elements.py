"""Pins of the oracle's element definitions and derivative symbols against what
the paper states (stencils, shape functions, symbols, Nyquist conditions)."""
import itertools
import os

import numpy as np
import pytest

from oracle import fe, projection as pj

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_stencils.txt")


def _paper_stencils():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, ax, ox, oy, c = line.split()
        out.setdefault((name, ax), []).append(((int(ox), int(oy)), float(c)))
    return out


@pytest.mark.parametrize("h", [(1.0, 1.0), (0.7, 1.9)])
def test_element1_shape_functions_match_paper(h):
    # Sec. "Linear finite elements": N00 = 1 - x/dx - y/dy, N10 = x/dx, N01 = y/dy
    verts, g, vol = fe.elements(2, np.array(h))[0]
    assert [tuple(v) for v in verts] == [(0, 0), (1, 0), (0, 1)]
    dx, dy = h
    np.testing.assert_allclose(g[0], [-1 / dx, -1 / dy], rtol=0, atol=1e-15)
    np.testing.assert_allclose(g[1], [1 / dx, 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(g[2], [0.0, 1 / dy], rtol=0, atol=1e-15)
    assert vol == pytest.approx(dx * dy / 2)
    # the shape functions interpolate: value 1 at own vertex, 0 at the others
    rng = np.random.default_rng(0)
    X = verts * np.array(h)
    for _ in range(5):
        lam = rng.dirichlet([1, 1, 1])
        x = lam @ X
        N = np.array([1 - x[0] / dx - x[1] / dy, x[0] / dx, x[1] / dy])
        np.testing.assert_allclose(N, lam, atol=1e-14)


def test_stencils_match_paper_fixture():
    """Every stencil the paper states (fixture) equals the oracle's symbol."""
    st = _paper_stencils()
    shape = (6, 5)
    h = np.array([1.3, 0.8])
    sym = {"fd": pj.symbols("fd", shape, h)[0], "cd": pj.symbols("cd", shape, h)[0],
           "ls": pj.symbols("ls", shape, h)[0], "fe1": pj.symbols("fe", shape, h)[0],
           "fe2": pj.symbols("fe", shape, h)[1]}
    for (name, ax), terms in st.items():
        a = "xy".index(ax)
        offs = [np.array(o) for o, _ in terms]
        coef = [c / h[a] for _, c in terms]
        ref = pj.stencil_symbol(offs, coef, shape, h)
        np.testing.assert_allclose(sym[name][a], ref, atol=1e-14, err_msg=f"{name} {ax}")


def test_fd_equals_fe_element1_and_closed_form():
    # Sec. "Linear finite elements": the element (1) stencil is the forward
    # difference; forward-difference symbol (exp(i k d) - 1)/d.
    shape = (8, 7)
    h = np.array([1.0, 2.0])
    fe_ = pj.symbols("fe", shape, h)
    fd = pj.symbols("fd", shape, h)
    np.testing.assert_allclose(fe_[0], fd[0], atol=1e-15)
    K = np.meshgrid(*[pj.wave_numbers(n, hh) for n, hh in zip(shape, h)], indexing="ij")
    for a in range(2):
        np.testing.assert_allclose(fd[0, a], (np.exp(1j * K[a] * h[a]) - 1) / h[a], atol=1e-14)
        # element (2) is the backward difference on the upper-right nodes:
        # exp(i k.(1,1)) (1 - exp(-i k_a d_a)) / d_a
        ph = np.exp(1j * (K[0] * h[0] + K[1] * h[1]))
        np.testing.assert_allclose(fe_[1, a], ph * (1 - np.exp(-1j * K[a] * h[a])) / h[a], atol=1e-14)


def test_central_difference_closed_form_and_lanczos():
    # central-difference symbol i sin(k d)/d = i k sigma(k), sigma = sin(kd)/(kd)
    shape = (9, 8)
    h = np.array([0.5, 1.5])
    cd = pj.symbols("cd", shape, h)[0]
    K = np.meshgrid(*[pj.wave_numbers(n, hh) for n, hh in zip(shape, h)], indexing="ij")
    for a in range(2):
        np.testing.assert_allclose(cd[a], 1j * np.sin(K[a] * h[a]) / h[a], atol=1e-14)
        sig = np.sinc(K[a] * h[a] / np.pi)
        np.testing.assert_allclose(cd[a], 1j * K[a] * sig, atol=1e-14)


def test_least_squares_is_mean_of_triangles():
    """Sec. "Least squares": minimising the corner residual gives the closed
    form, and (Sec. "Linear finite elements") it is the mean of the two
    triangle gradients."""
    rng = np.random.default_rng(3)
    dx, dy = 1.7, 0.6
    corners = {(0, 0): None, (1, 0): None, (0, 1): None, (1, 1): None}
    chi = {c: rng.standard_normal(2) for c in corners}
    # brute-force least squares over (F, psi00) of sum |psi_kl - chi_kl|^2
    A, b = [], []
    for (k, l), x in chi.items():
        dr = np.array([k * dx, l * dy])
        for i in range(2):
            row = np.zeros(6)
            row[i * 2:(i + 1) * 2] = dr      # F[i, :] . dr
            row[4 + i] = 1.0                  # psi00[i]
            A.append(row)
            b.append(x[i])
    sol = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0]
    F_ls = sol[:4].reshape(2, 2)
    F_closed = 0.5 * np.stack([(chi[1, 0] - chi[0, 0] + chi[1, 1] - chi[0, 1]) / dx,
                               (chi[0, 1] - chi[0, 0] + chi[1, 1] - chi[1, 0]) / dy], axis=1)
    np.testing.assert_allclose(F_ls, F_closed, atol=1e-13)
    # the two FE triangle gradients on a 1x1 periodic grid cannot hold four
    # distinct corners, so evaluate them directly from the element stencils
    grads = []
    for verts, g, _ in fe.elements(2, np.array([dx, dy])):
        G = sum(np.outer(chi[tuple(v)], g[c]) for c, v in enumerate(verts))
        grads.append(G)
    np.testing.assert_allclose(0.5 * (grads[0] + grads[1]), F_closed, atol=1e-13)
    # and the symbol of the LS stencil is the mean of the two FE symbols
    shape = (6, 6)
    np.testing.assert_allclose(pj.symbols("ls", shape)[0], pj.symbols("fe", shape).mean(axis=0), atol=1e-15)


@pytest.mark.parametrize("kind", ["fe", "fd", "cd", "ls"])
def test_stencils_sum_to_zero(kind):
    # Sec. "Discrete projection": sum_ij s_ij = 0, so Dhat(k = 0) = 0
    D = pj.symbols(kind, (6, 5))
    assert np.abs(D[..., 0, 0]).max() < 1e-15


def _symbol_at(kind, k, h):
    """Symbol of a 1D stencil at an arbitrary wavenumber k."""
    if kind == "fd":
        return (np.exp(1j * k * h) - 1) / h
    if kind == "cd":
        return (np.exp(1j * k * h) - np.exp(-1j * k * h)) / (2 * h)
    if kind == "fourier":
        return 1j * k


def test_nyquist_conditions():
    """Sec. "Even vs. odd number of grid points": a projection is unambiguous
    on even grids iff D(k_Ny) = D(-k_Ny) and D(k_Ny) D*(k_Ny) != 0.  Forward
    differences (= FE element 1) satisfy both, central differences violate the
    second, the Fourier derivative violates the first."""
    h = 1.0
    kny = np.pi / h
    fd = _symbol_at("fd", kny, h), _symbol_at("fd", -kny, h)
    cd = _symbol_at("cd", kny, h), _symbol_at("cd", -kny, h)
    fo = _symbol_at("fourier", kny, h), _symbol_at("fourier", -kny, h)
    assert abs(fd[0] - fd[1]) < 1e-15 and abs(fd[0]) ** 2 > 1.0
    assert abs(cd[0] - cd[1]) < 1e-15 and abs(cd[0]) ** 2 < 1e-30
    assert abs(fo[0] - fo[1]) > 1.0
    # on an 8-point grid the FE operator has S(k) > 0 for every k != 0
    S = np.sum(np.abs(pj.symbols("fe", (8, 8))) ** 2, axis=(0, 1))
    assert S[0, 0] == 0 and S.ravel()[1:].min() > 0.1
    # while central differences vanish on the Nyquist lines of even grids
    Scd = np.sum(np.abs(pj.symbols("cd", (8, 8))) ** 2, axis=(0, 1))
    assert Scd[4, 4] < 1e-28


def test_kuhn_tetrahedra_tile_the_voxel():
    h = np.array([1.0, 1.3, 0.7])
    els = fe.elements(3, h)
    assert len(els) == 6
    vols = [v for _, _, v in els]
    np.testing.assert_allclose(vols, np.prod(h) / 6, rtol=1e-14)
    # every tetrahedron contains the 000-111 diagonal; the six paths are distinct
    paths = set()
    for verts, _, _ in els:
        assert tuple(verts[0]) == (0, 0, 0) and tuple(verts[-1]) == (1, 1, 1)
        paths.add(tuple(map(tuple, verts)))
    assert len(paths) == 6
    # a random point of the unit cube lies in exactly one tetrahedron
    rng = np.random.default_rng(1)
    for _ in range(50):
        x = rng.random(3)
        inside = 0
        for verts, g, _ in els:
            X = verts * 1.0
            J = (X[1:] - X[0]).T
            lam = np.linalg.solve(J, x - X[0])
            bary = np.concatenate([[1 - lam.sum()], lam])
            inside += bool(np.all(bary > 0))
        assert inside == 1


@pytest.mark.parametrize("shape", [(9, 8), (7, 6, 8)])
def test_patch_test_affine_displacement(shape):
    """FE patch test: in a uniform material an affine displacement produces no
    nodal force at nodes whose elements do not straddle the periodic seam
    (conforming elements, correct assembly signs)."""
    dim = len(shape)
    rng = np.random.default_rng(5)
    lam, mu = fe.lame(np.full(shape, 2.0), np.full(shape, 0.3))
    h = np.array([1.0, 1.4, 0.8])[:dim]
    K = fe.assemble(lam, mu, h)
    A = rng.standard_normal((dim, dim))
    pos = np.stack(np.indices(shape), axis=-1).reshape(-1, dim) * h
    u = pos @ A.T
    q = (K @ u.ravel()).reshape(-1, dim)
    idx = np.stack(np.indices(shape), axis=-1).reshape(-1, dim)
    interior = np.all((idx >= 1) & (idx <= np.array(shape) - 2), axis=1)
    assert interior.sum() > 0
    assert np.abs(q[interior]).max() < 1e-12 * np.abs(A).max() * np.abs(K).max() * 10
    # and a seam node does feel the jump (the check is not vacuous)
    assert np.abs(q[~interior]).max() > 1e-3
