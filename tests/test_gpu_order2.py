"""GPU second-order upwind (deferred correction) against the oracle's
second-order scheme, through the C ABI.

  * one iteration from a rough start: every sampled (band, direction)
    distribution equals the oracle's transport solve with the correction of
    the initial distribution and the reconstructed boundary values (FP64;
    also on the FinFET recipe's tetrahedra, where the iteration does not
    converge);
  * converged fields equal the oracle's second-order fixed point (FP64 1e-9,
    mixed 1e-6), on quadrilaterals, hexahedra and a tetrahedral mesh whose
    cells partly have no gradient;
  * where the deferred correction does not contract (ballistic bands on the
    FinFET recipe's tetrahedra) the solve reports NBTE_ERR_DIVERGED;
  * a second-order batch member equals its stand-alone solve bitwise.
"""
import json

import numpy as np
import pytest

import oracle
from workloads import configs as C

from test_oracle_pins import tiny_hex, tiny_tet

pytestmark = pytest.mark.gpu


def _N():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_03226_amd import nbte
    return nbte


def _tiny_hex():
    return tiny_hex(np.random.default_rng(5))


def _tiny_tet():
    return tiny_tet(np.random.default_rng(5))


CASES = [("config1", C.config1, "sequential"), ("config2_small", C.config2_small, "synthetic"),
         ("tiny_hex", _tiny_hex, "synthetic"), ("tiny_tet", _tiny_tet, "synthetic")]


@pytest.mark.parametrize("name,maker,scheme", CASES + [("config3_small", C.config3_small, "synthetic")])
def test_one_second_order_iteration_matches_the_oracle(name, maker, scheme):
    N = _N()
    p = maker()
    su = oracle.prepare(p)
    xc = su.g.xc
    span = np.ptp(xc, axis=0) + 1e-30
    rng = np.random.default_rng(42)
    theta0 = np.sin(2.1 * xc[:, 0] / span[0]) + 0.5 * np.cos(3.3 * xc[:, 1] / span[1]) + 0.2 * rng.standard_normal(su.g.N)
    mesh, h = N.build_problem(p)
    opts = N.make_opts(scheme="sequential", precision="fp64", T_ref=p.T_ref, T_init=p.T_ref + theta0, order=2)
    N.nbte_prepare(h, p.Q, opts)
    N.nbte_iterate(h, 1)
    B, D = p.n_bands, p.n_dirs
    e0 = np.ascontiguousarray(np.broadcast_to(oracle.equilibrium(su, theta0)[:, None, :], (B, D, su.g.N)))
    div0, bd0 = oracle.reconstruct(su, e0)
    inflow = oracle.boundary_inflow(su, e0, bd0)
    e, _ = oracle.transport(su, theta0, inflow, -su.v[:, None, None] * div0)
    systems = [(0, 0), (B - 1, D - 1)] + [(int(rng.integers(B)), int(rng.integers(D))) for _ in range(10)]
    worst = 0.0
    for b, i in systems:
        eg = N.nbte_get_distribution(h, b, i)
        worst = max(worst, np.max(np.abs(eg - e[b, i])) / np.max(np.abs(e[b, i])))
    print(name, json.dumps({"err_e": worst}), flush=True)
    assert worst < 1e-12


_REF = {}


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("mixed", 1e-6)])
@pytest.mark.parametrize("name,maker,scheme", CASES)
def test_second_order_converged_parity(name, maker, scheme, precision, bar):
    N = _N()
    p = maker()
    if name not in _REF:
        _REF[name] = oracle.solve(p, scheme=scheme, tol=1e-13, max_iter=20000, defect_tol=1e-11, order=2)
    r = _REF[name]
    tol = 1e-12 if precision == "fp64" else 1e-8
    out = N.solve(p, precision=precision, scheme=scheme, tol=tol, max_iter=20000, allow_not_converged=True, order=2)
    err = {"err_TL": float(np.max(np.abs(out["T_lattice"] - r.T_lattice)) / np.max(np.abs(r.T_lattice - p.T_ref))),
           "err_T": float(np.max(np.abs(out["T"] - r.T)) / np.max(np.abs(r.T - p.T_ref))),
           "err_q": float(np.max(np.linalg.norm(out["q"] - r.q, axis=1)) / np.max(np.linalg.norm(r.q, axis=1)))}
    rec = dict(err, iterations=out["iterations"], oracle_iterations=r.iterations,
               energy_defect=out["energy_defect"])
    print(f"{name}/{precision}", json.dumps(rec), flush=True)
    assert max(err.values()) < bar, rec
    if precision == "fp64":
        assert out["energy_defect"] < 1e-9


def test_non_contracting_correction_is_reported_as_divergence():
    N = _N()
    p = C.config3_small()
    with pytest.raises(N.NbteError) as e:
        N.solve(p, precision="fp64", scheme="synthetic", tol=1e-10, max_iter=2000, order=2)
    assert e.value.status == N.ERR_DIVERGED


def test_second_order_refuses_acceleration():
    N = _N()
    p = C.config1()
    with pytest.raises(N.NbteError) as e:
        N.solve(p, precision="fp64", scheme="sequential", tol=1e-10, max_iter=10, order=2, accel=3)
    assert e.value.status == N.ERR_INVALID_ARG


def test_second_order_batch_member_equals_standalone():
    N = _N()
    probs = [C.config1(), C.config2_small(), C.config4_small()[0]]
    orders = [2, 2, 1]
    alone = [N.solve(p, precision="fp64", scheme=p.scheme, tol=1e-10, max_iter=4000, order=o)
             for p, o in zip(probs, orders)]
    batch = N.nbte_batch_create()
    handles, keep = [], []
    for p, o in zip(probs, orders):
        mesh, h = N.build_problem(p)
        keep.append(mesh)
        N.nbte_batch_admit(batch, h, p.Q, N.make_opts(scheme=p.scheme, precision="fp64", T_ref=p.T_ref, tol=1e-10,
                                                       max_iter=4000, order=o))
        handles.append(h)
    res = {}
    while len(res) < len(handles):
        N.nbte_batch_step(batch, 8)
        done, _ = N.nbte_batch_poll(batch)
        for h in done:
            if h.handle.value not in res:
                res[h.handle.value] = N.nbte_read_result(h)
                N.nbte_batch_remove(batch, h)
    for h, a in zip(handles, alone):
        b = res[h.handle.value]
        assert a["iterations"] == b["iterations"]
        for k in ("T_lattice", "T", "q"):
            assert np.array_equal(a[k], b[k]), k
