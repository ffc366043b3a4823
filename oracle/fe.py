"""Canonical periodic linear-FE small-strain homogenization, FP64, CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring): the plain definition the
GPU path must reproduce.

The paper states that the finite-element projection scheme is equivalent to a
canonical finite-element formulation on a fully structured grid (abstract; Sec.
"Linear finite elements").  This module is that formulation written out:

* Grid (discrete Fourier transform appendix): a periodic grid of N_x x N_y
  (x N_z) voxels of size h_a; node (i, j[, k]) sits at the lower-left corner of
  voxel (i, j[, k]); under periodicity there is one node per voxel.
* Elements (Sec. "Linear finite elements"): in 2D each pixel splits into
  element (1) with nodes 00, 10, 01 and element (2) with nodes 11, 01, 10.  In
  3D (the paper only says the generalisation is straightforward) each voxel
  splits into the six Kuhn tetrahedra around its 000-111 diagonal, tetrahedron
  pi having vertices 0, e_pi0, e_pi0 + e_pi1, 111, for the permutations pi in
  the order (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x).
* Small strain (small-strain appendix): e = sym(grad u) per element;
  isotropic law sigma = lambda tr(e) I + 2 mu e (plane strain in 2D).
* Weak form (Sec. "Compatibility projection", the weighted-residual equation):
  sum_e |e| B_e^T C_e (Ebar + B_e u~) = 0, i.e. K u~ = f with
  K = sum_e |e| B_e^T C_e B_e and f = -sum_e |e| B_e^T C_e Ebar; the mean
  strain Ebar is the macroscopic boundary condition carried by k = 0.

Array conventions: fields are C-ordered (Nx, Ny[, Nz]); nodal vectors are
(N, D) with node index the C-order flat voxel index; element fields are
(N, n_e, D, D).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

KUHN_ORDER = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


# ---------------------------------------------------------------------------
# elements
# ---------------------------------------------------------------------------
def element_vertices(dim):
    """Vertex offsets (voxel units) of the n_e elements of one voxel."""
    if dim == 2:
        return [np.array([[0, 0], [1, 0], [0, 1]]),
                np.array([[1, 1], [0, 1], [1, 0]])]
    if dim == 3:
        out = []
        for perm in KUHN_ORDER:
            v = [np.zeros(3, dtype=int)]
            for a in perm:
                w = v[-1].copy()
                w[a] += 1
                v.append(w)
            out.append(np.array(v))
        return out
    raise ValueError("dim must be 2 or 3")


def shape_gradients(verts, h):
    """Gradients of the linear (barycentric) shape functions of a simplex.

    With vertices X_0..X_D and J = [X_1 - X_0, ..., X_D - X_0] (columns), the
    shape function of vertex a >= 1 is N_a(x) = (J^-1 (x - X_0))_{a-1}, and
    N_0 = 1 - sum_{a>=1} N_a.  Returns (grad[n_vert, D], volume)."""
    verts = np.asarray(verts, dtype=np.float64)
    dim = verts.shape[1]
    X = verts * np.asarray(h, dtype=np.float64)[:dim]
    J = (X[1:] - X[0]).T
    Jinv = np.linalg.inv(J)
    g = np.zeros((dim + 1, dim))
    g[1:] = Jinv
    g[0] = -Jinv.sum(axis=0)
    vol = abs(np.linalg.det(J)) / math.factorial(dim)
    return g, vol


def elements(dim, h):
    """List of (vertex offsets, shape gradients, volume) per element."""
    return [(v,) + shape_gradients(v, h) for v in element_vertices(dim)]


def lame(E, nu, plane_stress=False):
    """Lame constants of isotropic elasticity (plane strain in 2D unless
    plane_stress)."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    mu = E / (2.0 * (1.0 + nu))
    if plane_stress:
        lam = E * nu / (1.0 - nu * nu)
    else:
        lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return lam, mu


# ---------------------------------------------------------------------------
# grid helpers
# ---------------------------------------------------------------------------
def _node_index(shape, offset):
    """Flat index of node (voxel + offset) for every voxel (periodic)."""
    idx = np.indices(shape)
    parts = [(idx[a] + offset[a]) % shape[a] for a in range(len(shape))]
    return np.ravel_multi_index(parts, shape).ravel()


def _default_h(dim, h):
    if h is None:
        return np.ones(dim)
    return np.asarray(h, dtype=np.float64)[:dim]


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------
def element_block(g, vol, c, d):
    """Coefficient blocks of the element stiffness between vertices c and d:
    K_e[c i, d j] = |e| (lambda A_ij + mu B_ij) with
    A_ij = g_c,i g_d,j and B_ij = delta_ij (g_c . g_d) + g_c,j g_d,i,
    the isotropic tensor C_iajb = lambda d_ia d_jb + mu (d_ij d_ab + d_ib d_aj)
    contracted with the two shape-function gradients."""
    gc, gd = g[c], g[d]
    A = vol * np.outer(gc, gd)
    B = vol * (np.eye(len(gc)) * np.dot(gc, gd) + np.outer(gd, gc))
    return A, B


def assemble(lam, mu, h=None):
    """Sparse periodic stiffness K (ndof x ndof, CSR), dof = node*D + i."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    shape = lam.shape
    dim = len(shape)
    h = _default_h(dim, h)
    N = lam.size
    lamf = lam.ravel()
    muf = mu.ravel()
    rows, cols, vals = [], [], []
    for verts, g, vol in elements(dim, h):
        nodes = [_node_index(shape, v) for v in verts]
        for c in range(dim + 1):
            for d in range(dim + 1):
                A, B = element_block(g, vol, c, d)
                for i in range(dim):
                    for j in range(dim):
                        v = lamf * A[i, j] + muf * B[i, j]
                        rows.append(nodes[c] * dim + i)
                        cols.append(nodes[d] * dim + j)
                        vals.append(v)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    K = sp.coo_matrix((vals, (rows, cols)), shape=(N * dim, N * dim)).tocsr()
    K.sum_duplicates()
    return K


def assemble_structured(lam, mu, h=None):
    """The same periodic stiffness as `assemble`, built per node from
    node-neighbour coefficient blocks instead of a per-element triplet list
    (far less memory and time, for grids such as 128^3).

    Node n couples to node n + o for the vertex offsets o = v_d - v_c of every
    element; the block of K[n, n + o] sums, over the elements and vertex pairs
    (c, d) with that offset, lambda A_cd + mu B_cd of the element's voxel
    n - v_c (element_block).  Terms with the same offset and the same vertex
    v_c share the voxel, so their coefficient blocks are added here; the C
    routine of the oracle (csr_cg.c) evaluates them per node.  On grids with
    an axis of length 1 or 2, two offsets can reach the same neighbour; their
    entries stay separate (duplicate column indices, which a product with K
    sums)."""
    from . import cg as ccg
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    shape = lam.shape
    dim = len(shape)
    h = _default_h(dim, h)
    N = lam.size
    coef = {}
    for verts, g, vol in elements(dim, h):
        for c in range(dim + 1):
            for d in range(dim + 1):
                key = (tuple(int(x) for x in verts[d] - verts[c]), tuple(int(x) for x in verts[c]))
                A, B = element_block(g, vol, c, d)
                a0, b0 = coef.get(key, (0.0, 0.0))
                coef[key] = (a0 + A, b0 + B)
    offs = sorted({o for o, _ in coef})
    slot = {o: k for k, o in enumerate(offs)}
    terms = sorted(coef)
    pad = lambda v: list(v) + [0] * (3 - len(v))
    slot_off = np.array([pad(o) for o in offs], dtype=np.int32)
    t_slot = np.array([slot[o] for o, _ in terms], dtype=np.int32)
    t_vc = np.array([pad(vc) for _, vc in terms], dtype=np.int32)
    t_A = np.ascontiguousarray([coef[t][0] for t in terms], dtype=np.float64)
    t_B = np.ascontiguousarray([coef[t][1] for t in terms], dtype=np.float64)
    nb = len(offs)
    indices, data = ccg.structured_csr(shape, slot_off, t_slot, t_vc, t_A, t_B, lam, mu)
    idx_t = np.int32 if N * dim * nb * dim < 2 ** 31 else np.int64
    indptr = np.arange(0, N * dim * nb * dim + 1, nb * dim, dtype=idx_t)
    return sp.csr_matrix((data, indices, indptr), shape=(N * dim, N * dim))


def stress_of(lam, mu, eps):
    """sigma = lambda tr(eps) I + 2 mu eps for eps[..., D, D]."""
    D = eps.shape[-1]
    tr = np.trace(eps, axis1=-2, axis2=-1)
    return lam[..., None, None] * tr[..., None, None] * np.eye(D) + 2.0 * mu[..., None, None] * eps


def load_vector(lam, mu, Ebar, h=None):
    """f = -sum_e |e| B_e^T C_e Ebar  (nodal force of the uniform strain)."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    shape = lam.shape
    dim = len(shape)
    h = _default_h(dim, h)
    N = lam.size
    sig = stress_of(lam.ravel(), mu.ravel(), np.broadcast_to(np.asarray(Ebar, float), (N, dim, dim)))
    f = np.zeros((N, dim))
    for verts, g, vol in elements(dim, h):
        for c in range(dim + 1):
            node = _node_index(shape, verts[c])
            # force on vertex c: -|e| sigma . grad N_c
            np.add.at(f, node, -vol * sig @ g[c])
    return f.ravel()


# ---------------------------------------------------------------------------
# solvers
# ---------------------------------------------------------------------------
def remove_mean(u, dim):
    u = np.asarray(u, dtype=np.float64).reshape(-1, dim)
    return (u - u.mean(axis=0)).ravel()


def solve_direct(K, f, dim):
    """Sparse LU with the D dofs of node 0 pinned; returns the zero-mean
    fluctuation.  K is singular only through rigid translations and f sums to
    zero, so the pinned system is regular and its residual at node 0 vanishes."""
    n = K.shape[0]
    free = np.arange(dim, n)
    Kf = K[free][:, free].tocsc()
    lu = spla.splu(Kf)
    u = np.zeros(n)
    u[free] = lu.solve(f[free])
    return remove_mean(u, dim)


def solve_cg(K, f, dim, tol=1e-13, maxit=200000):
    """Plain (unpreconditioned) conjugate gradients from the zero field, stop
    at ||f - K u|| <= tol ||f||.  Returns (u, iterations)."""
    u = np.zeros_like(f)
    r = f.copy()
    nf = np.linalg.norm(f)
    if nf == 0.0:
        return u, 0
    p = r.copy()
    rr = r @ r
    it = 0
    while it < maxit:
        q = K @ p
        a = rr / (p @ q)
        u += a * p
        r -= a * q
        it += 1
        rr_new = r @ r
        if math.sqrt(rr_new) <= tol * nf:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return remove_mean(u, dim), it


# ---------------------------------------------------------------------------
# post-processing
# ---------------------------------------------------------------------------
def element_gradients(u, shape, h=None):
    """grad u per element: G[N, n_e, D, D] with G[..., i, a] = d u_i / d x_a."""
    dim = len(shape)
    h = _default_h(dim, h)
    N = int(np.prod(shape))
    u = np.asarray(u, dtype=np.float64).reshape(N, dim)
    els = elements(dim, h)
    G = np.zeros((N, len(els), dim, dim))
    for e, (verts, g, vol) in enumerate(els):
        for c in range(dim + 1):
            node = _node_index(shape, verts[c])
            G[:, e] += u[node][:, :, None] * g[c][None, None, :]
    return G


def fields(u, lam, mu, Ebar, h=None):
    """Element strain eps = Ebar + sym(grad u) and stress sigma = C eps."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    shape = lam.shape
    G = element_gradients(u, shape, h)
    eps = np.asarray(Ebar, float)[None, None] + 0.5 * (G + np.swapaxes(G, -1, -2))
    ne = G.shape[1]
    lamv = np.repeat(lam.ravel()[:, None], ne, axis=1)
    muv = np.repeat(mu.ravel()[:, None], ne, axis=1)
    sig = stress_of(lamv, muv, eps)
    return eps, sig


def element_volumes(dim, h=None):
    h = _default_h(dim, h)
    return np.array([vol for _, _, vol in elements(dim, h)])


def average(field_e, dim, h=None):
    """Volume average over all elements of an element field (N, n_e, ...)."""
    w = element_volumes(dim, h)
    return np.tensordot(w, field_e.sum(axis=0), axes=(0, 0)) / (w.sum() * field_e.shape[0])


def energy_matrix(eps_list, lam, mu, h=None):
    """W_lm = < eps_l : C : eps_m > (volume average) for a list of strain
    fields (one per load case)."""
    dim = eps_list[0].shape[-1]
    ne = eps_list[0].shape[1]
    lamv = np.repeat(np.asarray(lam, float).ravel()[:, None], ne, axis=1)
    muv = np.repeat(np.asarray(mu, float).ravel()[:, None], ne, axis=1)
    L = len(eps_list)
    W = np.zeros((L, L))
    for l in range(L):
        s = stress_of(lamv, muv, eps_list[l])
        for m in range(L):
            W[l, m] = average(np.einsum("neij,neij->ne", s, eps_list[m]), dim, h)
    return W


VOIGT_PAIRS = {2: [(0, 0), (1, 1), (0, 1)],
               3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]}


def voigt_strain(E):
    """Engineering Voigt vector of a symmetric strain (shear doubled)."""
    dim = E.shape[-1]
    return np.array([E[a, b] * (1.0 if a == b else 2.0) for a, b in VOIGT_PAIRS[dim]])


def voigt_stress(S):
    dim = S.shape[-1]
    return np.array([S[a, b] for a, b in VOIGT_PAIRS[dim]])


def c_eff_energy(W, Ebars):
    """Effective Voigt stiffness from the energy matrix: W = E^T C E where the
    columns of E are the engineering Voigt strains of the load cases."""
    Ev = np.stack([voigt_strain(E) for E in Ebars], axis=1)
    Einv = np.linalg.inv(Ev)
    return Einv.T @ W @ Einv


def c_eff_stress(sig_means, Ebars):
    """Effective Voigt stiffness from the average stresses: S = C E."""
    Ev = np.stack([voigt_strain(E) for E in Ebars], axis=1)
    Sv = np.stack([voigt_stress(S) for S in sig_means], axis=1)
    return Sv @ np.linalg.inv(Ev)


# ---------------------------------------------------------------------------
# one-call solve
# ---------------------------------------------------------------------------
def homogenize(E, nu, Ebars, h=None, method="direct", tol=1e-13, lam_mu=None):
    """Solve every load case; returns a dict with u, eps, sig, sig_mean, W and
    (when the load cases form a Voigt basis) C_eff (energy and stress form)."""
    if lam_mu is None:
        lam, mu = lame(E, nu)
    else:
        lam, mu = (np.asarray(a, float) for a in lam_mu)
    shape = lam.shape
    dim = len(shape)
    K = assemble(lam, mu, h)
    out = {"u": [], "eps": [], "sig": [], "sig_mean": [], "iters": []}
    for Ebar in Ebars:
        f = load_vector(lam, mu, Ebar, h)
        if method == "direct":
            u = solve_direct(K, f, dim)
            it = 0
        elif method == "cg":
            u, it = solve_cg(K, f, dim, tol)
        elif method == "ccg":
            from . import cg as ccg
            u, it, _ = ccg.solve(K, f, tol)
            u = remove_mean(u, dim)
        else:
            raise ValueError(method)
        eps, sig = fields(u, lam, mu, Ebar, h)
        out["u"].append(u.reshape(-1, dim))
        out["eps"].append(eps)
        out["sig"].append(sig)
        out["sig_mean"].append(average(sig, dim, h))
        out["iters"].append(it)
    out["W"] = energy_matrix(out["eps"], lam, mu, h)
    nv = len(VOIGT_PAIRS[dim])
    if len(Ebars) == nv:
        out["C_eff"] = c_eff_energy(out["W"], Ebars)
        out["C_eff_stress"] = c_eff_stress(out["sig_mean"], Ebars)
    out["K"] = K
    return out


# ---------------------------------------------------------------------------
# local evaluation at sampled nodes (for grids too large to assemble)
# ---------------------------------------------------------------------------
def apply_K_at_nodes(lam, mu, p, nodes, h=None):
    """(K p) at selected nodes, summing the element contributions of the
    elements that have the node as a vertex (no global assembly).

    p: nodal field (N, D); nodes: flat node indices.  Returns (len(nodes), D)."""
    lam = np.asarray(lam)
    mu = np.asarray(mu)
    shape = lam.shape
    dim = len(shape)
    h = _default_h(dim, h)
    p = np.asarray(p, dtype=np.float64).reshape(-1, dim)
    nodes = np.asarray(nodes, dtype=np.int64)
    pos = np.stack(np.unravel_index(nodes, shape), axis=1)
    out = np.zeros((len(nodes), dim))
    lamf = np.asarray(lam, np.float64).ravel()
    muf = np.asarray(mu, np.float64).ravel()
    for verts, g, vol in elements(dim, h):
        for c in range(dim + 1):
            vox = (pos - verts[c]) % np.asarray(shape)
            vflat = np.ravel_multi_index(vox.T, shape)
            for d in range(dim + 1):
                nd = np.ravel_multi_index(((vox + verts[d]) % np.asarray(shape)).T, shape)
                A, B = element_block(g, vol, c, d)
                pd = p[nd]
                out += lamf[vflat, None] * (pd @ A.T) + muf[vflat, None] * (pd @ B.T)
    return out


def element_strains_at(u, shape, voxels, Ebar, h=None):
    """Element strains eps = Ebar + sym(grad u) of selected voxels only (local
    evaluation of `fields` for grids too large to post-process whole).

    u: nodal field (N, D); voxels: flat voxel indices.  Returns
    (len(voxels), n_e, D, D); element e of voxel v uses the nodes v + verts[c]
    with the shape-function gradients g[c], as in `element_gradients`."""
    dim = len(shape)
    h = _default_h(dim, h)
    u = np.asarray(u, dtype=np.float64).reshape(-1, dim)
    voxels = np.asarray(voxels, dtype=np.int64)
    pos = np.stack(np.unravel_index(voxels, shape), axis=1)
    els = elements(dim, h)
    G = np.zeros((len(voxels), len(els), dim, dim))
    for e, (verts, g, vol) in enumerate(els):
        for c in range(dim + 1):
            node = np.ravel_multi_index(((pos + verts[c]) % np.asarray(shape)).T, shape)
            G[:, e] += u[node][:, :, None] * g[c][None, None, :]
    return np.asarray(Ebar, float)[None, None] + 0.5 * (G + np.swapaxes(G, -1, -2))


def load_at_nodes(lam, mu, Ebar, nodes, h=None):
    """f at selected nodes (local evaluation of load_vector)."""
    lam = np.asarray(lam)
    mu = np.asarray(mu)
    shape = lam.shape
    dim = len(shape)
    h = _default_h(dim, h)
    nodes = np.asarray(nodes, dtype=np.int64)
    pos = np.stack(np.unravel_index(nodes, shape), axis=1)
    out = np.zeros((len(nodes), dim))
    Ebar = np.asarray(Ebar, float)
    for verts, g, vol in elements(dim, h):
        for c in range(dim + 1):
            vox = (pos - verts[c]) % np.asarray(shape)
            vflat = np.ravel_multi_index(vox.T, shape)
            sig = stress_of(lam.ravel()[vflat], mu.ravel()[vflat],
                            np.broadcast_to(Ebar, (len(nodes), dim, dim)))
            out += -vol * sig @ g[c]
    return out
