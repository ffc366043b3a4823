"""Discrete derivative symbols and the small-strain projection operator, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper's Sec. "Discrete projection" (Eqs. discrderiv, genfourderiv,
discrete_projection_op), Secs. "Finite differences" / "Least squares" /
"Linear finite elements" for the stencils, the discrete Fourier transform
appendix for the wavevector grid, the small-strain appendix for the operator
G_{Theta Lambda, ijlm}, and the two-point Fourier appendix.

Conventions
  * Symbols are evaluated on the FFT grid of numpy: entry m along an axis of
    length n stands for k = 2 pi m / (n h) with m taken in the paper's range
    [-n/2, n/2 - 1] (even n) or [-(n-1)/2, (n-1)/2] (odd n).  Periodic (stencil)
    symbols do not depend on that choice; the Fourier derivative i k does, and
    follows the paper's range (Nyquist at -pi/h).
  * Dhat has shape (n_e, D, *grid): Dhat[T, a] is the symbol of the derivative
    in direction a at evaluation point (element) T.
  * The forward transform is sum_r f(r) exp(-i k.r) (numpy.fft.fftn) and the
    inverse carries 1/N (numpy.fft.ifftn), as in the appendix.
"""
from __future__ import annotations

import numpy as np

from . import fe


def wave_numbers(n, h=1.0):
    """k = 2 pi m / (n h) with m in the paper's range (Fourier_wave_vectors),
    arranged in numpy FFT order."""
    m = np.fft.fftfreq(n, d=1.0 / n)  # 0..ceil(n/2)-1, then negative
    m = np.round(m).astype(np.int64)
    if n % 2 == 0:
        m[n // 2] = -n // 2  # numpy already uses -n/2 for the Nyquist entry
    return 2.0 * np.pi * m / (n * h)


def _kgrid(shape, h):
    ks = [wave_numbers(n, hh) for n, hh in zip(shape, h)]
    return np.meshgrid(*ks, indexing="ij")


def _axis_phase(m, r, n):
    """exp(2 pi i m r / n) for the integer wave indices m of an axis of n
    points and an integer node offset r, exact (1, i, -1, -i) where m r / n
    is a whole number of quarter turns."""
    t = np.mod(m * r, n)
    quarter = (4 * t) % n == 0
    exact = np.array([1.0 + 0j, 1j, -1.0 + 0j, -1j])
    return np.where(quarter, exact[((4 * t) // n) % 4], np.exp(2j * np.pi * (t / n)))


def stencil_symbol(offsets, coeffs, shape, h):
    """Eq. genfourderiv: (1/h_a) sum_j s_j exp(i k . r_j) for a stencil with
    node offsets r_j (voxel units) and coefficients s_j (already divided by
    h_a here).

    exp(i k . r_j) is the product over the axes of exp(i k_a r_a h_a) =
    exp(2 pi i m_a r_a / n_a), each factor exact at whole quarter turns.  A
    symbol that vanishes mathematically is then exactly zero instead of a
    rounding residue that the projection would treat as a derivative
    direction: a central difference at the Nyquist wavevector
    (i sin(pi) / h), or the least-squares x-derivative, whose factor
    (1 + exp(i k_y)) vanishes at the y-Nyquist wavevector."""
    ms = [np.round(np.fft.fftfreq(n, d=1.0 / n)).astype(np.int64) for n in shape]
    M = np.meshgrid(*ms, indexing="ij")
    out = np.zeros(shape, dtype=np.complex128)
    for off, c in zip(offsets, coeffs):
        e = np.ones(shape, dtype=np.complex128)
        for a in range(len(shape)):
            if int(off[a]) != 0:
                e = e * _axis_phase(M[a], int(off[a]), shape[a])
        out = out + c * e
    return out


def symbols(kind, shape, h=None):
    """Derivative symbols Dhat (n_e, D, *shape) for a discretisation kind:

    'fe'        linear finite elements, one evaluation point per element
                (2 triangles / 6 Kuhn tetrahedra per voxel); the stencil of an
                element is its shape-function gradients on its vertices
    'fd'        forward differences (Eq. forward-difference-derivative-fourier)
    'cd'        central differences (Eq. central-difference-derivative-fourier)
    'ls'        least-squares voxel gradient (Sec. "Least squares")
    'fourier'   Fourier derivative i k (Eq. original-G)
    'fourier2'  Fourier derivative at the two triangle centroids (2D appendix)
    """
    shape = tuple(shape)
    dim = len(shape)
    h = np.ones(dim) if h is None else np.asarray(h, float)[:dim]
    if kind == "fe":
        out = []
        for verts, g, _vol in fe.elements(dim, h):
            out.append([stencil_symbol(verts, g[:, a], shape, h) for a in range(dim)])
        return np.array(out)
    if kind == "fd":
        out = []
        for a in range(dim):
            e = np.zeros(dim, int)
            e[a] = 1
            out.append(stencil_symbol([np.zeros(dim, int), e], [-1.0 / h[a], 1.0 / h[a]], shape, h))
        return np.array([out])
    if kind == "cd":
        out = []
        for a in range(dim):
            e = np.zeros(dim, int)
            e[a] = 1
            out.append(stencil_symbol([-e, e], [-0.5 / h[a], 0.5 / h[a]], shape, h))
        return np.array([out])
    if kind == "ls":
        if dim != 2:
            raise NotImplementedError("least-squares stencil is given for 2D")
        c00, c10, c01, c11 = (0, 0), (1, 0), (0, 1), (1, 1)
        dx = stencil_symbol([c00, c10, c01, c11], np.array([-1, 1, -1, 1]) * 0.5 / h[0], shape, h)
        dy = stencil_symbol([c00, c10, c01, c11], np.array([-1, -1, 1, 1]) * 0.5 / h[1], shape, h)
        return np.array([[dx, dy]])
    if kind == "fourier":
        K = _kgrid(shape, h)
        return np.array([[1j * K[a] for a in range(dim)]])
    if kind == "fourier2":
        if dim != 2:
            raise NotImplementedError("two-point Fourier derivative is given for 2D")
        K = _kgrid(shape, h)
        s = (K[0] * h[0] + K[1] * h[1]) / 6.0
        d1 = [1j * K[a] * np.exp(-1j * s) for a in range(2)]
        d2 = [1j * K[a] * np.exp(+1j * s) for a in range(2)]
        return np.array([d1, d2])
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# finite-strain (gradient) projection, Eq. discrete_projection_op
# ---------------------------------------------------------------------------
def gradient_projection(Dhat):
    """g_ab(k) = D_a D_b^* / (D_c D_c^*) over the d = n_e D derivative indices;
    zero where the denominator vanishes (k = 0).  Shape (d, d, *grid)."""
    ne, D = Dhat.shape[:2]
    Dv = Dhat.reshape((ne * D,) + Dhat.shape[2:])
    S = np.sum(np.abs(Dv) ** 2, axis=0)
    safe = np.where(S > 0, S, 1.0)
    g = Dv[:, None] * np.conj(Dv)[None, :] / safe
    return np.where(S > 0, g, 0.0)


# ---------------------------------------------------------------------------
# small-strain projection, small-strain appendix
# ---------------------------------------------------------------------------
def small_strain_operator(Dhat, tiny=0.0):
    """G[T, L, i, j, l, m, *grid] of the small-strain appendix:

        Dinv_T = Dhat_T^* / sum_L Dhat_L . Dhat_L^*
        g_TL   = Dhat_T (x) Dinv_L
        h      = (1 + sum_T g_TT)^-1
        G_TL,ijlm = 1/2 (g_TL,il h_jm + g_TL,im h_jl + g_TL,jl h_im + g_TL,jm h_il)

    and G = 0 where sum |Dhat|^2 <= tiny (k = 0, which carries the mean)."""
    ne, D = Dhat.shape[:2]
    grid = Dhat.shape[2:]
    S = np.sum(np.abs(Dhat) ** 2, axis=(0, 1))
    ok = S > tiny
    safe = np.where(ok, S, 1.0)
    Dinv = np.conj(Dhat) / safe
    g = Dhat[:, None, :, None] * Dinv[None, :, None, :]          # [T, L, i, l, grid]
    gTT = sum(g[t, t] for t in range(ne))                        # [i, l, grid]
    eye = np.eye(D).reshape((D, D) + (1,) * len(grid))
    Amat = np.moveaxis(eye + gTT, (0, 1), (-2, -1))              # [grid, D, D]
    hmat = np.moveaxis(np.linalg.inv(Amat), (-2, -1), (0, 1))    # [j, m, grid]
    G = 0.5 * (np.einsum("TLil...,jm...->TLijlm...", g, hmat)
               + np.einsum("TLim...,jl...->TLijlm...", g, hmat)
               + np.einsum("TLjl...,im...->TLijlm...", g, hmat)
               + np.einsum("TLjm...,il...->TLijlm...", g, hmat))
    return np.where(ok, G, 0.0)


def apply_small_strain(G, e):
    """Projected strain: e'_T,ij = sum_L G_TL,ijlm e_L,ml on a real element
    field e[N-grid..., n_e, D, D] (grid axes first).  Uses numpy FFTs for the
    convolution (the appendix's forward/inverse transforms)."""
    grid = G.shape[6:]
    nd = len(grid)
    ehat = np.fft.fftn(e, axes=tuple(range(nd)))
    eh = np.moveaxis(ehat, tuple(range(nd)), tuple(range(-nd, 0)))   # [L, m, l, grid]
    out = np.einsum("TLijlm...,Lml...->Tij...", G, eh)
    out = np.moveaxis(out, tuple(range(-nd, 0)), tuple(range(nd)))
    return np.fft.ifftn(out, axes=tuple(range(nd))).real


def single_element_h(Dhat1):
    """Closed form of the small-strain appendix for one element:
    h = 1 - g_11 / 2."""
    D = Dhat1.shape[0]
    S = np.sum(np.abs(Dhat1) ** 2, axis=0)
    safe = np.where(S > 0, S, 1.0)
    g = Dhat1[:, None] * np.conj(Dhat1)[None, :] / safe
    eye = np.eye(D).reshape((D, D) + (1,) * (Dhat1.ndim - 1))
    return eye - 0.5 * g


# ---------------------------------------------------------------------------
# dense brute force
# ---------------------------------------------------------------------------
def dense_B(shape, h=None):
    """Dense matrix of u (N*D, node-major) -> element strain field
    (N, n_e, D, D) flattened, e = sym(grad u) per element."""
    shape = tuple(shape)
    dim = len(shape)
    N = int(np.prod(shape))
    cols = []
    for j in range(N * dim):
        u = np.zeros(N * dim)
        u[j] = 1.0
        G = fe.element_gradients(u, shape, h)
        cols.append((0.5 * (G + np.swapaxes(G, -1, -2))).ravel())
    return np.array(cols).T


def dense_projection(shape, h=None):
    """G = B (B^T B)^+ B^T: the orthogonal projection (Frobenius inner product
    over all elements) onto compatible element strain fields."""
    B = dense_B(shape, h)
    return B @ np.linalg.pinv(B.T @ B) @ B.T
