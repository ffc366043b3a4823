"""Helpers shared by the GPU parity tests (inputs and oracle references)."""
import sys

import numpy as np

from oracle import fe


def say(*a):
    """Name the case on stdout before the GPU runs it (flushed)."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def random_material(shape, seed, prec="fp64", emin=1.0, emax=10.0):
    """Random per-voxel (E, nu) -> (lam, mu) in the plan precision; the
    oracle receives exactly the same (rounded) values in FP64."""
    rng = np.random.default_rng(seed)
    E = rng.uniform(emin, emax, shape)
    nu = rng.uniform(0.1, 0.4, shape)
    lam, mu = fe.lame(E, nu)
    dt = np.float64 if prec == "fp64" else np.float32
    return lam.astype(dt).astype(np.float64), mu.astype(dt).astype(np.float64)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64) if not np.iscomplexobj(t.cpu().numpy()) else t.cpu().numpy()
