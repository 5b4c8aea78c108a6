"""Write oracle reference solutions of the full-size workloads (sampled cells).

Calls only the oracle and the seeded input generators.  Output:
tests/golden/<name>_reference.npz with the converged T_L, T and q at a seeded
sample of cells plus the global error scales (max |T_L - T_ref|, max |T - T_ref|,
max ||q||) and the oracle's iteration count, residual and energy defect.

Usage: python tests/golden/make_reference.py config2 [config3] [porous_10k]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs as C  # noqa: E402

MAKERS = {
    "config2": C.config2,
    "config3": C.config3,
    # porous film above the one-workgroup PCG limit of the GPU path (all cells stored)
    "porous_10k": lambda: C.porous_problem(4242, n_lo=9000, n_hi=11000),
}
SAMPLE = {"porous_10k": 1 << 30}


def make(name, n_sample=4096, tol=1e-12, defect_tol=1e-10, time_limit=None):
    p = MAKERS[name]()
    n_sample = SAMPLE.get(name, n_sample)
    t0 = time.time()
    r = oracle.solve(p, tol=tol, defect_tol=defect_tol, max_iter=100000, verbose=True, time_limit=time_limit)
    idx = np.sort(np.random.default_rng(12345).choice(p.n_cells, size=min(n_sample, p.n_cells), replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_reference.npz")
    np.savez_compressed(
        out, cells=idx, T_lattice=r.T_lattice[idx], T=r.T[idx], q=r.q[idx],
        scale_TL=np.max(np.abs(r.T_lattice - p.T_ref)), scale_T=np.max(np.abs(r.T - p.T_ref)),
        scale_q=np.max(np.linalg.norm(r.q, axis=1)), iterations=r.iterations, residual=r.residual,
        energy_defect=r.energy_defect, seconds=time.time() - t0, name=p.name)
    print(f"{name}: {r.iterations} iterations, residual {r.residual:.2e}, defect {r.energy_defect:.2e}, "
          f"{time.time() - t0:.0f} s -> {out}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["config2"]:
        make(n)
