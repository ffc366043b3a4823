"""Writes tests/golden/grf64_oracle.json: the oracle's effective stiffness of
the benchmark recipe (E = exp(Gaussian random field), nu = 0.3, 6 Kuhn
tetrahedra per voxel, the 6 unit load cases) at 64^3 voxels, with the
correlation length scaled with the cell (16 voxels at 256^3 -> 4 at 64^3).

Calls only oracle/ (sparse assembly of the canonical periodic FE stiffness
and the plain C CSR conjugate gradients to ||f - K u|| <= 1e-13 ||f||) and the
seeded input generator.  The GPU parity test reads the stored values instead
of re-solving (the solve takes tens of CPU minutes).

    python tests/golden/make_grf64.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import microstructures as ms  # noqa: E402
from oracle import cg as ocg  # noqa: E402
from oracle import fe  # noqa: E402

N_EDGE = 64
ELL = 16.0 * N_EDGE / 256.0
SEED = 1004
NU = 0.3
TOL = 1e-13


def main():
    t0 = time.time()
    m = ms.grf_modulus((N_EDGE,) * 3, ELL, SEED, NU)
    lam, mu = fe.lame(m.E, m.nu)
    Eb = ms.unit_loads(3)
    K = fe.assemble(lam, mu)
    print(f"assembled nnz={K.nnz} in {time.time() - t0:.1f} s", flush=True)
    eps, sig_mean, iters, relres = [], [], [], []
    for l in range(6):
        f = fe.load_vector(lam, mu, Eb[l])
        t1 = time.time()
        u, it, rr = ocg.solve(K, f, TOL, 2_000_000)
        u = fe.remove_mean(u, 3)
        e, s = fe.fields(u, lam, mu, Eb[l])
        eps.append(e)
        sig_mean.append(fe.average(s, 3))
        iters.append(int(it))
        relres.append(float(rr))
        print(f"load case {l}: {it} CG iterations, ||r||/||f|| = {rr:.3e}, {time.time() - t1:.1f} s", flush=True)
    W = fe.energy_matrix(eps, lam, mu)
    out = {
        "what": "oracle C_eff of the E=exp(GRF) benchmark recipe at 64^3 (canonical periodic linear FE, "
                "6 Kuhn tetrahedra per voxel, plain CG on the assembled stiffness)",
        "recipe": m.recipe,
        "n": N_EDGE, "ell": ELL, "seed": SEED, "nu": NU,
        "load_cases": Eb.tolist(),
        "cg_tol": TOL, "cg_iterations": iters, "cg_rel_residual": relres,
        "C_eff": fe.c_eff_energy(W, Eb).tolist(),
        "C_eff_stress": fe.c_eff_stress(sig_mean, Eb).tolist(),
        "W": W.tolist(),
        "stress_mean": [s.tolist() for s in sig_mean],
        "seconds": round(time.time() - t0, 1),
        "command": "python tests/golden/make_grf64.py",
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grf64_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
