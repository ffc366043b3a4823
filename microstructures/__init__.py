"""Seeded synthetic microstructures (material fields) for tests and benchmarks.

This module only produces inputs: per-voxel Young's modulus and Poisson ratio
arrays on a periodic voxel grid.  It holds none of the homogenization
arithmetic, and both the CPU oracle and the GPU library consume its output.

Conventions (the paper's discrete Fourier transform appendix places voxel
(i, j[, k]) with its lower-left corner at (i*dx, j*dy[, k*dz])):
  * arrays are C-ordered with shape (Nx, Ny) or (Nx, Ny, Nz), last index fastest;
  * the voxel spacing is 1, so voxel centres sit at (i + 1/2, j + 1/2[, k + 1/2]);
  * membership tests use periodic minimum-image distances from voxel centres.

Every generator returns a ``Micro`` with float64 arrays ``E`` and ``nu`` of the
grid shape, the integer ``phase`` map where the structure has phases, and a
``recipe`` string describing how it was drawn.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Micro:
    E: np.ndarray
    nu: np.ndarray
    phase: np.ndarray | None
    recipe: str

    @property
    def shape(self):
        return self.E.shape

    @property
    def dim(self):
        return self.E.ndim


def _centres(shape):
    axes = [np.arange(n, dtype=np.float64) + 0.5 for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def _periodic_delta(x, c, L):
    d = x - c
    return d - L * np.round(d / L)


def from_phases(phase, table, recipe):
    """Expand an integer phase map with a table [(E, nu), ...] into fields."""
    phase = np.asarray(phase, dtype=np.int32)
    table = np.asarray(table, dtype=np.float64)
    return Micro(E=table[phase, 0].copy(), nu=table[phase, 1].copy(),
                 phase=phase, recipe=recipe)


def homogeneous(shape, E=1.0, nu=0.3):
    ph = np.zeros(shape, dtype=np.int32)
    return from_phases(ph, [(E, nu)], f"homogeneous {shape} E={E} nu={nu}")


def circle(n=32, radius=8.0, centre=None, E=(1.0, 10.0), nu=(0.3, 0.3)):
    """Centred circular inclusion on an n x n grid (voxel-centre test).

    With n=32, R=8 and centre (16, 16) the inclusion holds 208 voxels and no
    voxel centre lies on the circle.
    """
    if centre is None:
        centre = (n / 2.0, n / 2.0)
    X, Y = _centres((n, n))
    dx = X - centre[0]
    dy = Y - centre[1]
    ph = (dx * dx + dy * dy <= radius * radius).astype(np.int32)
    return from_phases(ph, [(E[0], nu[0]), (E[1], nu[1])],
                       f"circle n={n} R={radius} centre={centre}")


def eshelby(n=151, frac=0.1, E_hard=1.0, contrast=10.0, nu=0.33):
    """Circular soft inhomogeneity (phase 1, E_hard / contrast) in a hard
    matrix (phase 0), radius frac * n voxels, centred on the middle voxel of
    an odd n x n grid so the discretised disc keeps the square's symmetries
    (the paper's 2D Eshelby-inhomogeneity setup: 151 x 151, half axes 10 % of
    the edge, stiffness ratio 10, equal Poisson ratios)."""
    m = circle(n, frac * n, (n / 2.0, n / 2.0), E=(E_hard, E_hard / contrast), nu=(nu, nu))
    m.recipe = f"eshelby n={n} R={frac * n} contrast={contrast} nu={nu}"
    return m


def single_voxel(n=17, E_hard=1.0, contrast=10.0, nu=0.33):
    """One soft voxel (phase 1, E_hard / contrast) at the centre of an odd n x n
    hard matrix (phase 0), equal Poisson ratios (the paper's single-voxel
    inhomogeneity, 17 x 17)."""
    ph = np.zeros((n, n), dtype=np.int32)
    ph[n // 2, n // 2] = 1
    return from_phases(ph, [(E_hard, nu), (E_hard / contrast, nu)],
                       f"single voxel n={n} contrast={contrast} nu={nu}")


def two_pillars(n=17, left=7, E_hard=1.0, contrast=10.0, nu=0.33):
    """Two pillars along y separated in x by zero-stiffness columns (phase 2,
    E = 0): x-columns [vacuum][left pillar: `left` columns][vacuum][right
    pillar: the rest]; the left pillar holds a soft line of three voxels
    (phase 1, E_hard / contrast) along y at its centre (the paper's two-pillar
    setup on 17 x 17: pillars of 7 and 8 columns)."""
    ph = np.zeros((n, n), dtype=np.int32)
    ph[0, :] = 2
    ph[1 + left, :] = 2
    cx = 1 + left // 2
    ph[cx, n // 2 - 1:n // 2 + 2] = 1
    return from_phases(ph, [(E_hard, nu), (E_hard / contrast, nu), (0.0, nu)],
                       f"two pillars n={n} left={left} contrast={contrast} nu={nu} vacuum columns 0 and {1 + left}")


def sphere(n=16, radius=4.0, E=(1.0, 10.0), nu=(0.3, 0.3)):
    X, Y, Z = _centres((n, n, n))
    c = n / 2.0
    ph = ((X - c) ** 2 + (Y - c) ** 2 + (Z - c) ** 2 <= radius * radius).astype(np.int32)
    return from_phases(ph, [(E[0], nu[0]), (E[1], nu[1])], f"sphere n={n} R={radius}")


def laminate(shape, axis, n_layer=None, E=(1.0, 10.0), nu=(0.3, 0.3)):
    """Two-phase laminate: phase 1 occupies the first n_layer voxel layers
    normal to ``axis`` (interfaces on voxel faces)."""
    shape = tuple(shape)
    if n_layer is None:
        n_layer = shape[axis] // 2
    idx = np.arange(shape[axis])
    sel = (idx < n_layer).astype(np.int32)
    bshape = [1] * len(shape)
    bshape[axis] = shape[axis]
    ph = np.broadcast_to(sel.reshape(bshape), shape).copy()
    return from_phases(ph, [(E[0], nu[0]), (E[1], nu[1])],
                       f"laminate {shape} axis={axis} layers={n_layer}")


def voronoi(shape, n_seeds, seed, E=(1.0, 100.0), nu=(0.3, 0.2), p=0.5):
    """Periodic Voronoi grains from uniform seed points; each grain draws its
    phase Bernoulli(p).  Voxels go to the nearest seed by periodic
    minimum-image distance; ties go to the lower seed index."""
    shape = tuple(shape)
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(n_seeds, len(shape))) * np.asarray(shape, np.float64)
    grain_phase = (rng.random(n_seeds) < p).astype(np.int32)
    cen = [np.arange(n, dtype=np.float64) + 0.5 for n in shape]
    best = np.full(shape, np.inf)
    owner = np.zeros(shape, dtype=np.int32)
    for s in range(n_seeds):
        d2 = np.zeros(shape)
        for a, n in enumerate(shape):
            d = _periodic_delta(cen[a], pts[s, a], n)
            bs = [1] * len(shape)
            bs[a] = n
            d2 = d2 + (d * d).reshape(bs)
        closer = d2 < best  # strict: ties keep the lower index
        best = np.where(closer, d2, best)
        owner = np.where(closer, s, owner)
    ph = grain_phase[owner]
    return from_phases(ph, [(E[0], nu[0]), (E[1], nu[1])],
                       f"voronoi {shape} seeds={n_seeds} seed={seed} p={p}")


def rsa_spheres(n=128, seed=1003, r_range=(4.0, 10.0), target_fraction=0.20,
                max_attempts=1_000_000, E=(1.0, 10.0), nu=(0.3, 0.25)):
    """Random sequential addition of non-overlapping spheres in a periodic n^3
    cell: radius ~ U[r_range], centre ~ U[0, n)^3, accepted if the periodic
    centre distance to every accepted sphere is >= r_i + r_j; stops once the
    voxel volume fraction reaches ``target_fraction``."""
    rng = np.random.default_rng(seed)
    ph = np.zeros((n, n, n), dtype=np.int32)
    cen = np.arange(n, dtype=np.float64) + 0.5
    centres = np.zeros((0, 3))
    radii = np.zeros(0)
    count = 0
    target = target_fraction * n ** 3
    attempts = 0
    while count < target and attempts < max_attempts:
        attempts += 1
        r = rng.uniform(*r_range)
        c = rng.uniform(0.0, n, size=3)
        if len(radii):
            d = c[None, :] - centres
            d -= n * np.round(d / n)
            if np.any(np.sqrt((d * d).sum(1)) < r + radii):
                continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        lo = [int(math.floor(c[a] - r - 1)) for a in range(3)]
        hi = [int(math.ceil(c[a] + r + 1)) for a in range(3)]
        ii = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
        dd = [_periodic_delta(cen[ii[a] % n], c[a], n) for a in range(3)]
        inside = (dd[0][:, None, None] ** 2 + dd[1][None, :, None] ** 2
                  + dd[2][None, None, :] ** 2) <= r * r
        sub = np.ix_(ii[0] % n, ii[1] % n, ii[2] % n)
        newly = inside & (ph[sub] == 0)
        block = ph[sub]
        block[newly] = 1
        ph[sub] = block
        count += int(newly.sum())
    m = from_phases(ph, [(E[0], nu[0]), (E[1], nu[1])],
                    f"rsa_spheres n={n} seed={seed} r={r_range} vf>={target_fraction}")
    m.extra = {"centres": centres, "radii": radii, "attempts": attempts}
    return m


def gaussian_random_field(shape, ell=16.0, seed=1004):
    """Gaussian random field with a Gaussian spectrum: white noise N(0, 1),
    filtered in Fourier space by sqrt(P(k)), P(k) = exp(-|k|^2 ell^2 / 2),
    k = 2 pi m / n, real part, then normalised to sample mean 0 and std 1."""
    shape = tuple(shape)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    W = np.fft.fftn(w)
    k2 = np.zeros(shape)
    for a, n in enumerate(shape):
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=1.0)
        bs = [1] * len(shape)
        bs[a] = n
        k2 = k2 + (k * k).reshape(bs)
    g = np.fft.ifftn(W * np.sqrt(np.exp(-k2 * ell * ell / 2.0))).real
    g = (g - g.mean()) / g.std()
    return g


def grf_modulus(shape, ell=16.0, seed=1004, nu=0.3):
    """E(x) = exp(g(x)) with g a normalised Gaussian random field; uniform nu."""
    g = gaussian_random_field(shape, ell, seed)
    E = np.exp(g)
    return Micro(E=E, nu=np.full(shape, float(nu)), phase=None,
                 recipe=f"grf {tuple(shape)} ell={ell} seed={seed} E=exp(g) nu={nu}")


def uneven_batch(seed=1005, n_maps=48, sizes=(64, 128, 256, 512)):
    """Uneven batch of 2D two-phase maps; map i uses the sub-stream
    default_rng([seed, i]): size n from ``sizes``, type laminate or circle,
    contrast c = exp(U[ln 2, ln 1000]); matrix E=1, nu=0.3, phase 2 E=c, nu=0.3.
    Laminates put phase 2 in the first n/2 layers normal to x or y; circles are
    centred at (n/2, n/2) with R = n/4."""
    maps = []
    for i in range(n_maps):
        rng = np.random.default_rng([seed, i])
        n = int(rng.choice(sizes))
        kind = ("laminate", "circle")[int(rng.integers(2))]
        c = float(np.exp(rng.uniform(np.log(2.0), np.log(1000.0))))
        if kind == "laminate":
            axis = int(rng.integers(2))
            m = laminate((n, n), axis, n // 2, E=(1.0, c), nu=(0.3, 0.3))
            # phase ids: 1 = the first n/2 layers (stiffness c), 0 = matrix
            m.recipe = f"map {i}: laminate n={n} axis={axis} contrast={c:.6g}"
            m.extra = {"kind": kind, "axis": axis, "contrast": c}
        else:
            m = circle(n, n / 4.0, (n / 2.0, n / 2.0), E=(1.0, c), nu=(0.3, 0.3))
            m.recipe = f"map {i}: circle n={n} R={n/4} contrast={c:.6g}"
            m.extra = {"kind": kind, "contrast": c}
        maps.append(m)
    return maps


# Named workloads with the shapes, distributions and load sets of the
# benchmark configurations.
UNIT_STRAIN = 0.01


def unit_loads(dim, amp=UNIT_STRAIN):
    """The Voigt unit load set: one symmetric macroscopic strain per Voigt
    component, tensor shear eps_ab = eps_ba = amp (engineering 2*amp)."""
    if dim == 2:
        pairs = [(0, 0), (1, 1), (0, 1)]
    else:
        pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    out = np.zeros((len(pairs), dim, dim))
    for l, (a, b) in enumerate(pairs):
        out[l, a, b] = amp
        out[l, b, a] = amp
    return out


def workload(name):
    """Return (Micro, Ebar[n_load, D, D], tol, precision-name) for a named
    configuration."""
    if name == "circle32":
        m = circle(32, 8.0, (16.0, 16.0), E=(1.0, 10.0), nu=(0.3, 0.3))
        Eb = np.zeros((1, 2, 2))
        Eb[0, 0, 0] = UNIT_STRAIN
        return m, Eb, 1e-10, "fp64"
    if name.startswith("eshelby"):
        # biaxial macroscopic strain exx = eyy = 1 %
        n = int(name[7:] or 151)
        Eb = np.zeros((1, 2, 2))
        Eb[0, 0, 0] = Eb[0, 1, 1] = UNIT_STRAIN
        return eshelby(n), Eb, 1e-10, "fp64"
    if name == "voronoi1024":
        m = voronoi((1024, 1024), 64, 1002)
        return m, unit_loads(2), 1e-10, "fp64"
    if name == "spheres128":
        m = rsa_spheres(128, 1003)
        return m, unit_loads(3), 1e-5, "fp32"
    if name == "grf256":
        m = grf_modulus((256, 256, 256), 16.0, 1004)
        return m, unit_loads(3), 1e-5, "fp32"
    if name.startswith("grf"):
        n = int(name[3:])
        m = grf_modulus((n, n, n), 16.0, 1004)
        return m, unit_loads(3), 1e-5, "fp32"
    raise KeyError(name)
