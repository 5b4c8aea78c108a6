"""Pins of the oracle's outer acceleration (Anderson acceleration of the
fixed-point iteration).  The acceleration is not part of the paper's method:
it changes the path of the outer iteration, never its fixed point.

  A1  on a linear fixed-point map x = M x + b in R^n with a history of at
      least n + 1 entries, Anderson acceleration is equivalent to GMRES
      (Walker & Ni 2011) and reaches the fixed point in at most n + 1 steps
      up to rounding, where the plain iteration is still far from it;
  A2  a history of one entry (depth 0) is the plain iteration, bitwise;
  A3  the accelerated iteration reaches ONE dense solve of the fully coupled
      system (the P2 reference, written independently of the oracle), for
      the sequential and the synthetic scheme;
  A4  the state packing is exact: unpack(pack(theta, inflow)) = (theta, inflow)
      on the entries it carries, and it carries the reflective walls'
      incoming entries only.
"""
import numpy as np
import pytest

import oracle
from workloads import configs as C

from test_oracle_pins import TINY, _rel, dense_coupled


def _linear_map(n, rho, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rho * np.linspace(-1.0, 1.0, n)            # spectral radius rho, real spectrum
    M = Q @ np.diag(lam) @ Q.T
    b = rng.standard_normal(n)
    x_star = np.linalg.solve(np.eye(n) - M, b)
    return (lambda x: M @ x + b), x_star


def test_A1_anderson_on_a_linear_map_terminates_like_gmres():
    n = 12
    G, x_star = _linear_map(n, 0.95, 3)
    x = np.zeros(n)
    X, Gs = [], []
    for k in range(n + 2):
        X.append(x)
        Gs.append(G(x))
        x = oracle.anderson_next(X, Gs)       # full history
    assert np.linalg.norm(x - x_star) / np.linalg.norm(x_star) < 1e-9
    y = np.zeros(n)
    for _ in range(n + 2):
        y = G(y)
    assert np.linalg.norm(y - x_star) / np.linalg.norm(x_star) > 1e-2


def test_A1_short_history_still_contracts_faster_than_plain():
    G, x_star = _linear_map(40, 0.97, 4)
    x, y = np.zeros(40), np.zeros(40)
    X, Gs = [], []
    for _ in range(60):
        X.append(x)
        Gs.append(G(x))
        del X[:-6], Gs[:-6]
        x = oracle.anderson_next(X, Gs)
        y = G(y)
    assert np.linalg.norm(x - x_star) < 0.05 * np.linalg.norm(y - x_star)


def test_A2_depth_zero_is_the_plain_iteration():
    p = C.config1()
    a = oracle.solve(p, tol=1e-10, max_iter=500)
    b = oracle.solve(p, tol=1e-10, max_iter=500, accel="anderson", depth=0)
    assert a.iterations == b.iterations
    assert np.array_equal(a.T_lattice, b.T_lattice) and np.array_equal(a.q, b.q)


@pytest.mark.parametrize("name,maker", TINY[:3])
@pytest.mark.parametrize("scheme", ["sequential", "synthetic"])
def test_A3_accelerated_iteration_equals_dense_coupled_solve(name, maker, scheme):
    rng = np.random.default_rng(5)
    p = maker(rng)
    thL, th, q = dense_coupled(p)
    r = oracle.solve(p, scheme=scheme, tol=1e-14, max_iter=20000, accel="anderson", depth=5)
    assert _rel(r.theta_L, thL) < 1e-11
    assert _rel(r.T - p.T_ref, th) < 1e-11
    assert np.max(np.linalg.norm(r.q - q, axis=1)) / np.max(np.linalg.norm(q, axis=1)) < 1e-11


def test_A4_state_packing_round_trip():
    rng = np.random.default_rng(9)
    p = TINY[1][1](rng)                      # hex: thermalizing, partial, diffuse, specular walls
    su = oracle.prepare(p)
    B, D, NBF = len(su.C), len(su.w), len(su.g.bf_owner)
    theta = rng.standard_normal(su.g.N)
    inflow = rng.standard_normal((B, D, NBF))
    x = oracle.accel_state(su, theta, inflow)
    n_refl_in = int(np.sum((su.sdotS < 0) & (su.bc_kind != 0)[:, None]))
    assert len(x) == su.g.N + B * n_refl_in
    th2, in2 = oracle.accel_unpack(su, x, np.zeros_like(inflow))
    assert np.array_equal(th2, theta)
    keep = ((su.sdotS < 0) & (su.bc_kind != 0)[:, None]).T[None]
    keep = np.broadcast_to(keep, inflow.shape)
    assert np.allclose(in2[keep], inflow[keep], rtol=1e-15, atol=0)
    assert np.all(in2[~keep] == 0)


def test_accelerated_reflective_device_needs_fewer_iterations():
    """Not a pin (a property of this workload): with partially specular walls
    the lagged wall inflow is the slow mode; accelerating it with the
    temperature halves the outer iterations."""
    p = C.config3_small()
    a = oracle.solve(p, tol=1e-9, max_iter=3000)
    b = oracle.solve(p, tol=1e-9, max_iter=3000, accel="anderson", depth=5)
    assert b.iterations < 0.6 * a.iterations
    dev = np.max(np.abs(a.T_lattice - p.T_ref))
    assert np.max(np.abs(a.T_lattice - b.T_lattice)) / dev < 1e-7
