"""Write the oracle's converged solutions of the parity workloads.

Calls only the oracle and the seeded input generators (nothing of the GPU
library).  Output: tests/golden/<name>_reference.npz holding the converged
T_L, T and q -- on every cell, or on a seeded sample of cells when the case
says so (then `cells` lists them) -- plus the global error scales
(max |T_L - T_ref|, max |T - T_ref|, max ||q||) and the oracle's iteration
count, residual and energy defect.  The porous-film batch (config 4) is one
file with the members' arrays under "<j>/<field>".

Every reference runs the oracle to a residual of 1e-12 and an energy defect
of 1e-10 (the oracle's stopping rule, Methods: convergence criterion), so the
stored fields sit on the discrete fixed point to about 1e-11 of the
deviation scale.  The largest cases (the FinFET-like device, the 64-film
batch) iterate with the oracle's Anderson acceleration, which changes the
path of the outer iteration and not its fixed point.

Usage: python tests/golden/make_reference.py config2 [config3] [serving_5008] [config4] ...
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs as C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name -> (problem maker, cells stored: None = every cell, k = a seeded sample of k)
MAKERS = {
    "config2": (C.config2, None),
    "config3": (C.config3, None),
    # porous film above the one-workgroup PCG limit of the GPU path
    "porous_10k": (lambda: C.porous_problem(4242, n_lo=9000, n_hi=11000), None),
    # full-size 3D requests of the serving stream (a FinFET-like tet mesh and a box)
    "serving_5008": (lambda: C.serving_request(5008), None),
    "serving_5027": (lambda: C.serving_request(5027), None),
}
CONFIG4_SAMPLE = 1024   # cells stored per porous film of the 64-film batch


# cases whose plain oracle iteration takes hours: the oracle's Anderson
# acceleration of the outer iteration (same fixed point; tests/test_oracle_accel.py)
ACCEL = {"config3", "config4"}


def _solve(p, tol, defect_tol, verbose, accel=None):
    return oracle.solve(p, tol=tol, defect_tol=defect_tol, max_iter=100000, verbose=verbose, accel=accel)


def _fields(p, r, n_sample, seed=12345):
    d = {"scale_TL": np.max(np.abs(r.T_lattice - p.T_ref)), "scale_T": np.max(np.abs(r.T - p.T_ref)),
         "scale_q": np.max(np.linalg.norm(r.q, axis=1)), "iterations": r.iterations, "residual": r.residual,
         "energy_defect": r.energy_defect, "seconds": r.seconds, "name": p.name}
    if n_sample is None or n_sample >= p.n_cells:
        d.update(T_lattice=r.T_lattice, T=r.T, q=r.q)
    else:
        idx = np.sort(np.random.default_rng(seed).choice(p.n_cells, size=n_sample, replace=False))
        d.update(cells=idx.astype(np.int32), T_lattice=r.T_lattice[idx], T=r.T[idx], q=r.q[idx])
    return d


def make(name, tol=1e-12, defect_tol=1e-10, verbose=True):
    t0 = time.time()
    out = os.path.join(HERE, f"{name}_reference.npz")
    if name == "config4":
        d = {}
        for j, p in enumerate(C.config4()):
            r = _solve(p, tol, defect_tol, False, accel="anderson")
            for k, x in _fields(p, r, CONFIG4_SAMPLE, seed=12345 + j).items():
                d[f"{j}/{k}"] = x
            print(f"config4[{j}] {p.name}: {r.iterations} iterations, residual {r.residual:.2e}, "
                  f"defect {r.energy_defect:.2e}, {r.seconds:.0f} s", flush=True)
        d["members"] = j + 1
    else:
        maker, n_sample = MAKERS[name]
        p = maker()
        r = _solve(p, tol, defect_tol, verbose, accel="anderson" if name in ACCEL else None)
        d = _fields(p, r, n_sample)
        print(f"{name}: {r.iterations} iterations, residual {r.residual:.2e}, defect {r.energy_defect:.2e}",
              flush=True)
    np.savez_compressed(out, **d)
    print(f"{name}: {time.time() - t0:.0f} s -> {out}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["config2"]:
        make(n)
