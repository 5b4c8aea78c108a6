"""Pins of the oracle against facts that do not come from the oracle itself.

  P1  every (band, direction) sweep equals numpy.linalg.solve of the assembled
      upwind system (tiny meshes of every cell type);
  P2  the converged iteration equals ONE dense solve of the fully coupled
      system (all e and T_L unknowns, boundary conditions implicit);
  P3  diffusive limit: exact interior identities of first-order upwind on a
      uniform 1D mesh (linear T, cell flux -kappa_d dT/dx, face flux
      -(kappa_d + kappa_num) dT/dx), and O(Kn) agreement with Fourier's law;
  P4  ballistic limit: closed-form slab flux, error ~ 1/Kn; exact uniform
      transport of a uniform inflow;
  P5  global energy balance at convergence;
  P6  linearity / superposition and T_ref invariance;
  P7  weight scaling, cell renumbering and mirror symmetry;
  P8  zero net flux through specular/diffuse/partial walls for any e;
  P9  sequential and both synthetic readings reach the same fixed point;
  plus the collision-divergence identity Q - D_h q = beta (theta_seq - theta).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import geometry as geo
from workloads import Boundary, Problem
from workloads import configs as C
from workloads import meshes as M
from workloads.tables import gl_azimuth_quadrature, inplane_quadrature

NM = 1e-9
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# tiny problems of every cell type
# ----------------------------------------------------------------------------

def _bands(B, rng, lam_nm=(20, 300)):
    C_ = rng.uniform(0.5e6, 2e6, B)
    v = rng.uniform(2000, 8000, B)
    lam = np.exp(rng.uniform(np.log(lam_nm[0]), np.log(lam_nm[1]), B)) * NM
    return C_, v, lam / v


def tiny_quad(rng, B=2, D=8, n=3, Q=True):
    xs = np.linspace(0, 60 * NM, n + 1)
    xyz, cells, bf, tags = M.structured_quad(xs, xs)
    s, w = inplane_quadrature(D)
    C_, v, tau = _bands(B, rng)
    return Problem("tq", 2, xyz, "quad4", cells, bf, tags,
                   [Boundary(1, "thermalizing", 301.0), Boundary(2, "thermalizing", 299.5),
                    Boundary(3, "specular"), Boundary(4, "diffuse")],
                   C_, v, tau, s, w, rng.uniform(0, 1e17, len(cells)) if Q else np.zeros(len(cells)))


def tiny_hex(rng, B=2, n=2):
    xs = np.linspace(0, 50 * NM, n + 1)
    xyz, cells = M.structured_hex(xs, xs, xs)
    bf = M.hex_boundary(cells)
    tags = M.box_tags(xyz, bf, (0, 0, 0), (50 * NM,) * 3, 1e-6 * NM)
    s, w = gl_azimuth_quadrature(2, 8)
    C_, v, tau = _bands(B, rng)
    return Problem("th", 3, xyz, "hex8", cells, bf, tags,
                   [Boundary(1, "thermalizing", 302.0), Boundary(2, "thermalizing", 300.0),
                    Boundary(3, "partial", specularity=0.3), Boundary(4, "partial", specularity=0.7),
                    Boundary(5, "diffuse"), Boundary(6, "specular")],
                   C_, v, tau, s, w, rng.uniform(0, 1e17, len(cells)))


def tiny_tet(rng, B=2):
    xs = np.linspace(0, 40 * NM, 2)
    xyz, hexes = M.structured_hex(xs, xs, xs)
    cells = M.hex_to_tets(hexes)
    bf = M.tet_boundary(cells)
    tags = M.box_tags(xyz, bf, (0, 0, 0), (40 * NM,) * 3, 1e-6 * NM)
    s, w = gl_azimuth_quadrature(2, 4)
    C_, v, tau = _bands(B, rng)
    return Problem("tt", 3, xyz, "tet4", cells, bf, tags,
                   [Boundary(1, "thermalizing", 301.0)] +
                   [Boundary(t, "partial", specularity=0.5) for t in (2, 3, 4, 5, 6)],
                   C_, v, tau, s, w, rng.uniform(0, 1e17, len(cells)))


def tiny_tri(rng, B=2, D=8):
    p = C.config4_small()[2]
    C_, v, tau = _bands(B, rng)
    s, w = inplane_quadrature(D)
    return Problem("tr", 2, p.xyz, "tri3", p.cells, p.bfaces, p.bface_tag, p.boundaries,
                   C_, v, tau, s, w, np.zeros(p.n_cells))


TINY = [("quad", tiny_quad), ("hex", tiny_hex), ("tet", tiny_tet), ("tri", tiny_tri)]


# ----------------------------------------------------------------------------
# dense assembly, written independently of the oracle's solver
# ----------------------------------------------------------------------------

def _mirror_and_win(g, s, w, p):
    """Per boundary face: mirror direction indices and sum_in w |s.S|."""
    Sb = g.S[g.bf_owner, g.bf_local]
    nhat = Sb / np.linalg.norm(Sb, axis=1)[:, None]
    mir = np.zeros((len(Sb), len(w)), int)
    for j in range(len(Sb)):
        for i in range(len(w)):
            r = s[i] - 2 * np.dot(s[i], nhat[j]) * nhat[j]
            mir[j, i] = int(np.argmin(np.linalg.norm(s - r, axis=1)))
    sS = Sb @ s.T
    win = np.array([sum(w[k] * -sS[j, k] for k in range(len(w)) if sS[j, k] < 0) for j in range(len(Sb))])
    return sS, mir, win


def dense_coupled(p):
    """Unknowns: e[b,i,c] and theta_L[c]; boundary inflow expressed implicitly
    through the owner's outgoing values; energy conservation of the collision
    term closes each cell."""
    g = geo.build(p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    B, D, N = len(p.C), len(p.w), g.N
    W = p.w.sum()
    Ctot = p.C.sum()
    nE = B * D * N
    n = nE + N
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    idx = lambda b, i, c: (b * D + i) * N + c
    bcs = {bb.tag: bb for bb in p.boundaries}
    sS, mir, win = _mirror_and_win(g, p.s, p.w, p)
    for b in range(B):
        for i in range(D):
            for c in range(N):
                r = idx(b, i, c)
                a = g.S[c] @ p.s[i] / g.V[c]
                A[r, r] += 1 / p.tau[b] + p.v[b] * a[a > 0].sum()
                A[r, nE + c] -= p.C[b] / (W * p.tau[b])
                rhs[r] += p.Q[c] * p.C[b] / (Ctot * W)
                for f in range(g.F):
                    if a[f] >= 0:
                        continue
                    coef = p.v[b] * -a[f]
                    nb = g.nbr[c, f]
                    if nb >= 0:
                        A[r, idx(b, i, nb)] -= coef
                        continue
                    j = -(nb + 1)
                    bc = bcs[int(g.bf_tag[j])]
                    if bc.kind == "thermalizing":
                        rhs[r] += coef * p.C[b] * (bc.T_wall - p.T_ref) / W
                        continue
                    ps = {"specular": 1.0, "diffuse": 0.0, "partial": bc.specularity}[bc.kind]
                    if ps > 0:
                        A[r, idx(b, mir[j, i], c)] -= coef * ps
                    if ps < 1:
                        for k in range(D):
                            if sS[j, k] > 0:
                                A[r, idx(b, k, c)] -= coef * (1 - ps) * p.w[k] * sS[j, k] / win[j]
    for c in range(N):
        r = nE + c
        for b in range(B):
            for i in range(D):
                A[r, idx(b, i, c)] += p.w[i] / p.tau[b]
            A[r, r] -= p.C[b] / p.tau[b]
    x = np.linalg.solve(A, rhs)
    e = x[:nE].reshape(B, D, N)
    theta_L = x[nE:]
    theta = np.einsum("i,bic->c", p.w, e) / Ctot
    q = np.einsum("b,i,ik,bic->ck", p.v, p.w, p.s, e)
    return theta_L, theta, q


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# ----------------------------------------------------------------------------
# P1
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("name,maker", TINY)
def test_P1_sweep_equals_dense_system_solve(name, maker):
    rng = np.random.default_rng(11)
    p = maker(rng)
    su = oracle.prepare(p)
    g = su.g
    B, D, N = len(p.C), len(p.w), g.N
    theta = rng.uniform(-1, 1, N)
    inflow = rng.uniform(-1, 1, (B, D, len(g.bf_owner))) * 1e4
    e, outflux = oracle.transport(su, theta, inflow)
    for b in range(B):
        for i in range(D):
            A = np.zeros((N, N))
            r = p.C[b] * theta / (su.W * p.tau[b]) + p.Q * p.C[b] / (su.C_tot * su.W)
            for c in range(N):
                a = g.S[c] @ p.s[i] / g.V[c]
                A[c, c] = 1 / p.tau[b] + p.v[b] * a[a > 0].sum()
                for f in range(g.F):
                    if a[f] < 0:
                        nb = g.nbr[c, f]
                        if nb >= 0:
                            A[c, nb] -= p.v[b] * -a[f]
                        else:
                            r[c] += p.v[b] * -a[f] * inflow[b, i, -(nb + 1)]
            ref = np.linalg.solve(A, r)
            assert _rel(e[b, i], ref) < 1e-13


# ----------------------------------------------------------------------------
# P2 and P9
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("name,maker", TINY[:3])
@pytest.mark.parametrize("scheme", ["sequential", "synthetic", "synthetic_literal"])
def test_P2_P9_iteration_equals_dense_coupled_solve(name, maker, scheme):
    rng = np.random.default_rng(5)
    p = maker(rng)
    thL, th, q = dense_coupled(p)
    r = oracle.solve(p, scheme=scheme, tol=1e-14, max_iter=20000)
    assert _rel(r.theta_L, thL) < 1e-11
    assert _rel(r.T - p.T_ref, th) < 1e-11
    assert np.max(np.linalg.norm(r.q - q, axis=1)) / np.max(np.linalg.norm(q, axis=1)) < 1e-11


# ----------------------------------------------------------------------------
# P4: ballistic limit
# ----------------------------------------------------------------------------

def _golden_flux_factor():
    out = {}
    for line in open(os.path.join(GOLDEN, "ballistic_flux_factor.txt")):
        if line.strip() and not line.startswith("#"):
            D, F = line.split()
            out[int(D)] = float(F)
    return out


def test_P4_flux_factor_fixture_matches_quadrature():
    for D, F in _golden_flux_factor().items():
        s, w = inplane_quadrature(D)
        assert np.sum(w[s[:, 0] > 0] * s[s[:, 0] > 0, 0]) / w.sum() == pytest.approx(F, rel=1e-14)


@pytest.mark.parametrize("name,maker", TINY)
def test_P4_uniform_inflow_is_transported_exactly(name, maker):
    """With no collisions a uniform inflow E stays E in every cell, because
    sum_{out} a = sum_{in} |a| for a closed cell."""
    rng = np.random.default_rng(2)
    p = maker(rng)
    p.tau = np.full(len(p.C), 1e200)
    p.Q = np.zeros(p.n_cells)
    su = oracle.prepare(p)
    E = 3.7e4
    inflow = np.full((len(p.C), len(p.w), len(su.g.bf_owner)), E)
    e, outflux = oracle.transport(su, np.zeros(su.g.N), inflow)
    assert np.max(np.abs(e / E - 1)) < 1e-13


def test_P4_ballistic_slab_flux():
    """Thermalizing walls 301/299 K, specular sides, Kn >> 1: the flux tends to
    sum C v (T_h - T_c) F(D) and T to the wall mean, with error ~ 1/Kn."""
    F = _golden_flux_factor()[16]
    errs = []
    for kn in (1e2, 1e3, 1e4):
        tau = kn * 100 * NM / 6000.0
        p = C.config1(n=8, tau=tau)
        r = oracle.solve(p, scheme="sequential", tol=1e-14, max_iter=2000)
        q_ball = p.C[0] * p.v[0] * 2.0 * F
        errs.append(np.max(np.abs(r.q[:, 0] / q_ball - 1)))
        assert np.max(np.abs(r.T - 300.0)) < 10.0 / kn
    errs = np.array(errs)
    assert errs[0] < 0.05
    ratios = errs[:-1] / errs[1:]
    assert np.all((ratios > 7) & (ratios < 13)), ratios


# ----------------------------------------------------------------------------
# P3: diffusive limit
# ----------------------------------------------------------------------------

def _slab(kn, h_over_lam=1 / 20, D=16, L=1000 * NM):
    lam = kn * L
    n = int(round(L / (lam * h_over_lam)))
    xyz, cells, bf, tags = M.structured_quad(np.linspace(0, L, n + 1), np.array([0, 50 * NM]))
    s, w = inplane_quadrature(D)
    v = 6000.0
    return Problem("slab", 2, xyz, "quad4", cells, bf, tags,
                   [Boundary(1, "thermalizing", 301.0), Boundary(2, "thermalizing", 299.0),
                    Boundary(3, "specular"), Boundary(4, "specular")],
                   np.array([1.66e6]), np.array([v]), np.array([lam / v]), s, w, np.zeros(n)), n, lam


def test_P3_interior_identities_on_uniform_mesh():
    p, n, lam = _slab(0.01)
    r = oracle.solve(p, scheme="synthetic", tol=1e-14, max_iter=500)
    x = (np.arange(n) + 0.5) / n * 1000 * NM
    inner = (x > 30 * lam) & (x < 1000 * NM - 30 * lam)
    th = r.theta_L[inner]
    # linear interior: second differences vanish
    d2 = th[2:] - 2 * th[1:-1] + th[:-2]
    assert np.max(np.abs(d2)) < 1e-11
    slope = (th[-1] - th[0]) / (x[inner][-1] - x[inner][0])
    s, w = inplane_quadrature(16)
    W = w.sum()
    Cv, v, tau = 1.66e6, 6000.0, lam / 6000.0
    h = 1000 * NM / n
    kappa_d = Cv * v * v * tau * np.sum(w * s[:, 0] ** 2) / W
    kappa_num = Cv * v * h * np.sum(w * np.abs(s[:, 0])) / (2 * W)
    # conserved face flux = heat leaving through the cold wall (per unit depth / height)
    face_flux = r.flows_by_tag[2] / (50 * NM)
    assert face_flux == pytest.approx(-(kappa_d + kappa_num) * slope, rel=1e-9)
    # cell-centred moment q = -kappa_d dT/dx
    assert np.max(np.abs(r.q[inner, 0] / (-kappa_d * slope) - 1)) < 1e-9


def test_P3_fourier_limit_error_is_first_order_in_Kn():
    dev = []
    for kn in (0.02, 0.01):
        p, n, lam = _slab(kn)
        r = oracle.solve(p, scheme="synthetic", tol=1e-12, max_iter=500)
        x = (np.arange(n) + 0.5) / n
        T_F = 301.0 - 2.0 * x
        inner = (x > 0.25) & (x < 0.75)
        dev.append(np.max(np.abs(r.T_lattice[inner] - T_F[inner])) / 2.0)
    assert dev[0] < 0.05 and dev[1] < 0.025
    assert 1.6 < dev[0] / dev[1] < 2.4


# ----------------------------------------------------------------------------
# P5, P6, P7, P8 and the collision-divergence identity
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [C.config2_small, C.config3_small, lambda: C.config4_small()[2]])
def test_P5_energy_balance(maker):
    p = maker()
    r = oracle.solve(p, tol=1e-13, max_iter=3000, defect_tol=1e-10)
    assert r.energy_defect < 1e-10


def test_collision_divergence_identity():
    """Multiplying the discrete per-mode balance by w V and summing over modes:
    Qdot - D_h q = beta (theta_seq - theta) exactly, with the face values of
    the sweep."""
    rng = np.random.default_rng(3)
    for maker in (tiny_hex, tiny_tet, tiny_quad):
        p = maker(rng)
        su = oracle.prepare(p)
        theta = rng.uniform(-1, 1, su.g.N)
        e0 = np.broadcast_to(oracle.equilibrium(su, rng.uniform(-1, 1, su.g.N))[:, None, :],
                             (len(p.C), len(p.w), su.g.N))
        inflow = oracle.boundary_inflow(su, e0)
        e, outflux = oracle.transport(su, theta, inflow)
        ts, _, _ = oracle.moments(su, e)
        lhs = su.Q - oracle.divergence(su, outflux)
        rhs = su.beta * (ts - theta)
        assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


def test_P8_reflective_walls_carry_no_net_flux():
    rng = np.random.default_rng(8)
    for maker in (tiny_hex, tiny_tet, tiny_quad):
        p = maker(rng)
        su = oracle.prepare(p)
        e = rng.uniform(-1, 1, (len(p.C), len(p.w), su.g.N)) * 1e3
        inflow = oracle.boundary_inflow(su, e)
        flows = oracle.boundary_flows(su, e, inflow)
        refl = su.bc_kind != 0
        scale = np.einsum("b,i,fi->f", p.v, p.w, np.abs(su.sdotS)) * 1e3
        assert np.max(np.abs(flows[refl]) / scale[refl]) < 1e-15


def test_P6_superposition_and_reference_shift():
    rng = np.random.default_rng(6)
    p = tiny_hex(rng)
    full = oracle.solve(p, tol=1e-14, max_iter=5000)
    # walls only
    pw = tiny_hex(np.random.default_rng(6)); pw.Q = np.zeros(p.n_cells)
    walls = oracle.solve(pw, tol=1e-14, max_iter=5000)
    # source only (walls at T_ref)
    pq = tiny_hex(np.random.default_rng(6))
    pq.boundaries = [Boundary(b.tag, b.kind, 300.0 if b.kind == "thermalizing" else 0.0, b.specularity)
                     for b in pq.boundaries]
    src = oracle.solve(pq, tol=1e-14, max_iter=5000)
    assert _rel(full.theta_L, walls.theta_L + src.theta_L) < 1e-11
    assert _rel(full.q, walls.q + src.q) < 1e-11
    # T_ref shift
    ps = tiny_hex(np.random.default_rng(6)); ps.T_ref = 250.0
    sh = oracle.solve(ps, tol=1e-14, max_iter=5000)
    assert np.max(np.abs(sh.T_lattice - full.T_lattice)) / np.max(np.abs(full.theta_L)) < 1e-11
    assert _rel(sh.q, full.q) < 1e-11


def test_P7_weight_scaling_renumbering_and_symmetry():
    rng = np.random.default_rng(7)
    p = tiny_tet(rng)
    ref = oracle.solve(p, tol=1e-14, max_iter=5000)
    ps = tiny_tet(np.random.default_rng(7)); ps.w = ps.w * 2.5
    sc = oracle.solve(ps, tol=1e-14, max_iter=5000)
    assert _rel(sc.theta_L, ref.theta_L) < 1e-11 and _rel(sc.q, ref.q) < 1e-11
    perm = np.random.default_rng(1).permutation(p.n_cells)
    pp = tiny_tet(np.random.default_rng(7)); pp.cells = p.cells[perm]; pp.Q = p.Q[perm]
    rp = oracle.solve(pp, tol=1e-14, max_iter=5000)
    assert _rel(rp.theta_L, ref.theta_L[perm]) < 1e-11
    # config 1: antisymmetric about x = L/2 and independent of y
    r1 = oracle.solve(C.config1(), tol=1e-14, max_iter=5000)
    th = (r1.T_lattice - 300.0).reshape(16, 16)
    assert np.max(np.abs(th + th[:, ::-1])) < 1e-12
    assert np.max(np.abs(th - th[:1])) < 1e-12


# ----------------------------------------------------------------------------
# cyclic upwind graphs: a non-convex (dart) quad makes the upwind graph of
# some directions cyclic; the oracle then solves that system with a sparse
# direct solve, which must still equal the dense solve (P1) and give the
# coupled fixed point (P2)
# ----------------------------------------------------------------------------

def dart_mesh(R=50 * NM):
    """Three quads around the point P = 0: two convex sectors between the rays
    at 10, 60 and 110 degrees, and a dart that closes the fan through the
    lower half-plane (reflex angle at P).  The three interior edges are rays
    from P inside one half-plane, so for every in-plane direction at an
    angle in (110, 190) degrees (and its opposite) each cell is upwind of the
    next one counter-clockwise: the cycle 0 -> 1 -> 2 -> 0.  The dart is
    numbered last so that every interior edge takes its orientation from a
    convex cell."""
    ang = np.radians([10.0, 60.0, 110.0])
    V = R * np.c_[np.cos(ang), np.sin(ang)]
    Wo = 1.5 * R * np.c_[np.cos(np.radians([35.0, 85.0])), np.sin(np.radians([35.0, 85.0]))]
    xyz = np.vstack([[0.0, 0.0], V, Wo, [0.0, -2.0 * R]])          # P=0, V1..V3 = 1..3, W1 = 4, W2 = 5, W3 = 6
    cells = np.array([[0, 1, 4, 2], [0, 2, 5, 3], [0, 3, 6, 1]], np.int64)
    bf = np.array([[1, 4], [4, 2], [2, 5], [5, 3], [3, 6], [6, 1]], np.int64)
    tags = np.array([2, 2, 2, 2, 1, 2], np.int32)
    return xyz, cells, bf, tags


def tiny_dart(rng, B=2, D=8):
    xyz, cells, bf, tags = dart_mesh()
    s, w = inplane_quadrature(D)
    C_, v, tau = _bands(B, rng)
    return Problem("dart", 2, xyz, "quad4", cells, bf, tags,
                   [Boundary(1, "thermalizing", 301.0), Boundary(2, "diffuse")],
                   C_, v, tau, s, w, rng.uniform(0, 1e17, len(cells)))


def test_dart_mesh_has_cyclic_directions_and_the_oracle_solves_them_exactly():
    from oracle.solver import _lib, _p
    import ctypes
    rng = np.random.default_rng(17)
    p = tiny_dart(rng)
    su = oracle.prepare(p)
    g = su.g
    assert np.all(g.V > 0)
    assert np.max(np.abs(g.S.sum(axis=1))) < 1e-12 * np.max(np.abs(g.S))   # every cell closes
    phi = np.degrees(np.arctan2(p.s[:, 1], p.s[:, 0])) % 360
    cyclic = (phi > 110) & (phi < 190) | (phi > 290) & (phi < 370)
    assert cyclic.any() and not cyclic.all()
    nbr = np.ascontiguousarray(g.nbr, np.int64)
    S = np.ascontiguousarray(g.S)
    for i in range(len(p.w)):
        e = np.empty(g.N)
        fl = np.empty(g.N)
        st = _lib().oracle_sweep_system(g.N, g.F, _p(nbr, ctypes.c_int64), _p(S), _p(g.V),
                                        _p(np.ascontiguousarray(p.s[i])), 1.0, 1.0, _p(np.ones(g.N)),
                                        _p(np.zeros(len(g.bf_owner))), _p(e), _p(fl))
        assert st == (1 if cyclic[i] else 0), (i, phi[i])
    # P1 on the cyclic systems: the direct fallback equals the dense solve
    theta = rng.uniform(-1, 1, g.N)
    inflow = rng.uniform(-1, 1, (len(p.C), len(p.w), len(g.bf_owner))) * 1e4
    e, _ = oracle.transport(su, theta, inflow)
    for b in range(len(p.C)):
        for i in np.flatnonzero(cyclic):
            A = np.zeros((g.N, g.N))
            r = p.C[b] * theta / (su.W * p.tau[b]) + p.Q * p.C[b] / (su.C_tot * su.W)
            for c in range(g.N):
                a = g.S[c] @ p.s[i] / g.V[c]
                A[c, c] = 1 / p.tau[b] + p.v[b] * a[a > 0].sum()
                for f in range(g.F):
                    if a[f] < 0:
                        nb = g.nbr[c, f]
                        if nb >= 0:
                            A[c, nb] -= p.v[b] * -a[f]
                        else:
                            r[c] += p.v[b] * -a[f] * inflow[b, i, -(nb + 1)]
            assert _rel(e[b, i], np.linalg.solve(A, r)) < 1e-13
    # P2 on the cyclic mesh
    thL, th, q = dense_coupled(p)
    res = oracle.solve(p, scheme="synthetic", tol=1e-14, max_iter=20000)
    assert _rel(res.theta_L, thL) < 1e-11
    assert np.max(np.linalg.norm(res.q - q, axis=1)) / np.max(np.linalg.norm(q, axis=1)) < 1e-11


# ----------------------------------------------------------------------------
# energy temperature T (the macroscopic temperature of the outputs): exact
# special cases that fix its normalisation
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("name,maker", TINY)
def test_energy_temperature_of_local_equilibrium_is_the_lattice_temperature(name, maker):
    """e = C theta / W in every direction (local equilibrium at an arbitrary
    field theta) carries the energy C theta per volume, so T - T_ref = theta
    exactly; it also has no net flux (q = 0 for a quadrature with
    sum_i w_i s_i = 0) and the collision-weighted temperature is theta too."""
    rng = np.random.default_rng(23)
    p = maker(rng)
    su = oracle.prepare(p)
    theta = rng.uniform(-3, 3, su.g.N)
    e = np.broadcast_to(oracle.equilibrium(su, theta)[:, None, :], (len(p.C), len(p.w), su.g.N))
    ts, th, q = oracle.moments(su, e)
    assert np.max(np.abs(th - theta)) <= 1e-14 * np.max(np.abs(theta))
    assert np.max(np.abs(ts - theta)) <= 1e-14 * np.max(np.abs(theta))
    assert np.max(np.abs(p.w @ p.s)) < 1e-14
    assert np.max(np.abs(q)) <= 1e-12 * np.max(p.C * p.v) * np.max(np.abs(theta))


def test_gray_medium_energy_and_lattice_temperatures_coincide():
    """With one band the collision weight 1/tau is common to every mode, so
    the lattice temperature of Eq. (5) and the energy temperature are the
    same moment of ANY distribution; the converged gray solve (config 1,
    sequential) therefore has T = T_L on every cell, and the iteration's
    sequential update equals the energy temperature of each iterate."""
    rng = np.random.default_rng(29)
    p = C.config1(n=6, D=8)
    su = oracle.prepare(p)
    e = rng.standard_normal((1, len(p.w), su.g.N))
    ts, th, _ = oracle.moments(su, e)
    assert np.max(np.abs(ts - th)) <= 1e-14 * np.max(np.abs(th))
    r = oracle.solve(p, scheme="sequential", tol=1e-13)
    assert np.max(np.abs(r.T - r.T_lattice)) <= 1e-12 * np.max(np.abs(r.T_lattice - p.T_ref))
