"""Pins of the oracle's projection operators: brute force, invariants, the
single-element closed form and Milton's Fourier projection."""
import numpy as np
import pytest

from oracle import fe, projection as pj


def _rand_sym(rng, shape):
    e = rng.standard_normal(shape)
    return 0.5 * (e + np.swapaxes(e, -1, -2))


@pytest.mark.parametrize("shape", [(4, 4), (5, 4), (3, 4, 5), (4, 4, 4)])
def test_small_strain_operator_equals_dense_brute_force(shape):
    """Small-strain appendix: the per-wavevector operator equals the orthogonal
    projection B (B^T B)^+ B^T onto compatible element strain fields, assembled
    densely in real space (includes odd sizes and Nyquist planes)."""
    dim = len(shape)
    Gd = pj.dense_projection(shape)
    Dh = pj.symbols("fe", shape)
    G = pj.small_strain_operator(Dh)
    rng = np.random.default_rng(11)
    for _ in range(2):
        e = _rand_sym(rng, shape + (Dh.shape[0], dim, dim))
        np.testing.assert_allclose(pj.apply_small_strain(G, e).ravel(), Gd @ e.ravel(), atol=1e-13)


@pytest.mark.parametrize("shape", [(4, 4), (5, 3), (3, 4, 2)])
def test_projection_invariants(shape):
    """G is idempotent and self-adjoint with eigenvalues in {0, 1}; its rank is
    the number of non-rigid displacement modes; G(Bu) = Bu; G(uniform) = 0; the
    complement I - G yields divergence-free (equilibrated) fields."""
    dim = len(shape)
    N = int(np.prod(shape))
    Gd = pj.dense_projection(shape)
    B = pj.dense_B(shape)
    np.testing.assert_allclose(Gd @ Gd, Gd, atol=1e-13)
    np.testing.assert_allclose(Gd, Gd.T, atol=1e-13)
    ev = np.linalg.eigvalsh(0.5 * (Gd + Gd.T))
    assert np.all(np.minimum(np.abs(ev), np.abs(ev - 1)) < 1e-10)
    assert int(np.round(ev.sum())) == N * dim - dim
    rng = np.random.default_rng(2)
    u = rng.standard_normal(N * dim)
    np.testing.assert_allclose(Gd @ (B @ u), B @ u, atol=1e-12)
    Eb = _rand_sym(rng, (dim, dim))
    ne = 2 if dim == 2 else 6
    uni = np.broadcast_to(Eb, (N, ne, dim, dim)).ravel()
    assert np.abs(Gd @ uni).max() < 1e-13
    e = rng.standard_normal(Gd.shape[0])
    assert np.abs(B.T @ (e - Gd @ e)).max() < 1e-12


def test_projection_of_random_field_is_compatible():
    """Sec. "Linear finite elements" (randomly perturbed triangles): G maps a
    random element field onto one that is the symmetric gradient of a nodal
    displacement."""
    shape = (5, 6)
    rng = np.random.default_rng(4)
    Dh = pj.symbols("fe", shape)
    G = pj.small_strain_operator(Dh)
    e = _rand_sym(rng, shape + (2, 2, 2))
    Ge = pj.apply_small_strain(G, e).ravel()
    B = pj.dense_B(shape)
    u, *_ = np.linalg.lstsq(B, Ge, rcond=None)
    assert np.abs(B @ u - Ge).max() < 1e-12
    assert np.abs(B @ u - e.ravel()).max() > 0.1


def test_fourier_small_strain_matches_milton():
    """Small-strain appendix, single element with the Fourier derivative: the
    operator reduces to the classical small-strain projection (Milton):
    G_ijlm = 1/2 (n_i d_jl n_m + n_i d_jm n_l + n_j d_il n_m + n_j d_im n_l)
             - n_i n_j n_l n_m,  n = k/|k|."""
    shape = (6, 5, 4)
    Dh = pj.symbols("fourier", shape)
    G = pj.small_strain_operator(Dh)[0, 0]
    K = np.meshgrid(*[pj.wave_numbers(n) for n in shape], indexing="ij")
    k = np.stack(K)
    kn = np.linalg.norm(k, axis=0)
    n = k / np.where(kn > 0, kn, 1)
    d = np.eye(3)
    ref = 0.5 * (np.einsum("i...,jl,m...->ijlm...", n, d, n) + np.einsum("i...,jm,l...->ijlm...", n, d, n)
                 + np.einsum("j...,il,m...->ijlm...", n, d, n) + np.einsum("j...,im,l...->ijlm...", n, d, n)) \
        - np.einsum("i...,j...,l...,m...->ijlm...", n, n, n, n)
    ref[..., 0, 0, 0] = 0
    np.testing.assert_allclose(G.real, ref, atol=1e-13)
    assert np.abs(G.imag).max() < 1e-13


def test_single_element_h_closed_form():
    """Small-strain appendix: with one element, h = (1 + g_11)^-1 = 1 - g_11/2
    (g_11 is a rank-one projector); checked for FD and Fourier symbols."""
    for kind in ("fd", "fourier"):
        Dh = pj.symbols(kind, (5, 6))[0]
        D = Dh.shape[0]
        S = np.sum(np.abs(Dh) ** 2, axis=0)
        ok = S > 0
        g = Dh[:, None] * np.conj(Dh)[None, :] / np.where(ok, S, 1)
        A = np.moveaxis(np.eye(D)[:, :, None, None] + g, (0, 1), (-2, -1))
        hinv = np.moveaxis(np.linalg.inv(A), (-2, -1), (0, 1))
        hcl = pj.single_element_h(Dh)
        np.testing.assert_allclose(hinv[:, :, ok], hcl[:, :, ok], atol=1e-14)


def test_gradient_projection_original_fourier():
    """Eq. original-G: with D = i k, g = k k / k^2, and g(0) = 0; idempotent."""
    shape = (5, 4)
    g = pj.gradient_projection(pj.symbols("fourier", shape))
    K = np.meshgrid(*[pj.wave_numbers(n) for n in shape], indexing="ij")
    k2 = K[0] ** 2 + K[1] ** 2
    ref = np.array([[K[a] * K[b] / np.where(k2 > 0, k2, 1) for b in range(2)] for a in range(2)])
    np.testing.assert_allclose(g, ref, atol=1e-15)
    assert np.abs(g[..., 0, 0]).max() == 0
    gg = np.einsum("ab...,bc...->ac...", g, g)
    np.testing.assert_allclose(gg, g, atol=1e-14)


def test_gradient_projection_fe_idempotent_hermitian():
    """Eq. discrete_projection_op with the FE stencil: d = n_e D derivatives,
    g is a Hermitian rank-one projector for k != 0."""
    g = pj.gradient_projection(pj.symbols("fe", (4, 6)))
    gg = np.einsum("ab...,bc...->ac...", g, g)
    np.testing.assert_allclose(gg, g, atol=1e-14)
    np.testing.assert_allclose(g, np.conj(np.swapaxes(g, 0, 1)), atol=1e-15)
    tr = np.einsum("aa...->...", g).real
    assert np.allclose(tr.ravel()[1:], 1.0) and tr[0, 0] == 0


def test_difference_symbols_vanish_exactly_at_nyquist():
    """The central difference i sin(k h) / h (Sec. "Finite differences") is
    exactly zero at the Nyquist wavevector of an even axis, and the
    least-squares x-derivative carries the factor (1 + exp(i k_y)), exactly
    zero at the y-Nyquist wavevector (Sec. "Least squares").  Elsewhere the
    symbols equal their closed forms to rounding."""
    shape, h = (4, 6), (1.0, 0.7)
    cd = pj.symbols("cd", shape, h)[0]
    assert np.all(cd[0][2, :] == 0) and np.all(cd[1][:, 3] == 0)
    K = np.meshgrid(*[pj.wave_numbers(n, hh) for n, hh in zip(shape, h)], indexing="ij")
    for a in range(2):
        np.testing.assert_allclose(cd[a], 1j * np.sin(K[a] * h[a]) / h[a], rtol=0, atol=1e-15)
    ls = pj.symbols("ls", shape, h)[0]
    assert np.all(ls[0][:, 3] == 0) and np.all(ls[1][2, :] == 0)
    ex = (np.exp(1j * K[0] * h[0]) - 1) * (1 + np.exp(1j * K[1] * h[1])) / (2 * h[0])
    np.testing.assert_allclose(ls[0], ex, rtol=0, atol=1e-15)


def test_modes_without_derivative_are_projected_out():
    """On a 2 x 3 grid the central difference along the 2-point axis vanishes
    at every wavevector (sin(0) = sin(pi) = 0): the projection then maps every
    field onto gradients along the other axis only, and the wavevectors whose
    whole symbol vanishes (m_y = 0) are projected to zero."""
    D = pj.symbols("cd", (2, 3))
    assert np.all(D[0, 0] == 0)
    G = pj.small_strain_operator(D)
    assert np.all(G[..., :, 0] == 0)
    # the xx strain component never survives: no x-derivative exists
    assert np.all(G[0, 0, 0, 0] == 0)
