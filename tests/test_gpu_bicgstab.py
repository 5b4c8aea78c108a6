"""GPU Jacobi-BiCGSTAB inner solver (the paper's optional iterative solve of
each (band, direction) transport system) through the C ABI.

  * per iteration it solves the same systems as the exact level-order sweep:
    after a few outer iterations from the same start the distributions agree
    to the inner tolerance;
  * converged fields equal the oracle's (FP64 1e-9, mixed 1e-6), including a
    mesh whose upwind graph is cyclic (every interior face implicit, no
    lagging);
  * it refuses the second-order scheme.
"""
import json

import numpy as np
import pytest

import oracle
from workloads import configs as C

from test_oracle_pins import tiny_dart

pytestmark = pytest.mark.gpu

BICG = {"inner_solver": 1, "inner_max_iter": 2000, "inner_rtol": 1e-13}


def _N():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_03226_amd import nbte
    return nbte


@pytest.mark.parametrize("maker", [C.config2_small, C.config3_small])
def test_bicgstab_iterates_equal_sweep_iterates(maker):
    N = _N()
    p = maker()
    got = []
    for tuning in ({}, BICG):
        mesh, h = N.build_problem(p)
        N.nbte_set_tuning(h, **tuning)
        N.nbte_prepare(h, p.Q, N.make_opts(scheme="synthetic", precision="fp64", T_ref=p.T_ref))
        N.nbte_iterate(h, 4)
        got.append([N.nbte_get_distribution(h, b, i) for b, i in [(0, 0), (p.n_bands - 1, p.n_dirs - 1), (1, 5)]])
    err = max(np.max(np.abs(a - b)) / np.max(np.abs(a)) for a, b in zip(*got))
    print(p.name, json.dumps({"bicgstab_vs_sweep": err}), flush=True)
    assert err < 1e-9


def _dart():
    return tiny_dart(np.random.default_rng(17), B=3, D=16)


CASES = [("config1", C.config1, "sequential"), ("config2_small", C.config2_small, "synthetic"),
         ("config3_small", C.config3_small, "synthetic"), ("dart", _dart, "synthetic")]
_REF = {}


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("mixed", 1e-6)])
@pytest.mark.parametrize("name,maker,scheme", CASES)
def test_bicgstab_converged_parity(name, maker, scheme, precision, bar):
    N = _N()
    p = maker()
    if name not in _REF:
        _REF[name] = oracle.solve(p, scheme=scheme, tol=1e-13, max_iter=20000, defect_tol=1e-11)
    r = _REF[name]
    out = N.solve(p, precision=precision, scheme=scheme, tol=1e-12 if precision == "fp64" else 1e-8,
                  max_iter=20000, allow_not_converged=True, tuning=BICG)
    err = {"err_TL": float(np.max(np.abs(out["T_lattice"] - r.T_lattice)) / np.max(np.abs(r.T_lattice - p.T_ref))),
           "err_T": float(np.max(np.abs(out["T"] - r.T)) / np.max(np.abs(r.T - p.T_ref))),
           "err_q": float(np.max(np.linalg.norm(out["q"] - r.q, axis=1)) / np.max(np.linalg.norm(r.q, axis=1)))}
    print(name, precision, json.dumps(dict(err, iterations=out["iterations"])), flush=True)
    assert max(err.values()) < bar, err


def test_bicgstab_refuses_second_order():
    N = _N()
    p = C.config1()
    with pytest.raises(N.NbteError) as e:
        N.solve(p, precision="fp64", scheme="sequential", tol=1e-10, max_iter=10, order=2, tuning=BICG)
    assert e.value.status == N.ERR_INVALID_ARG
