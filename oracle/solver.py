"""ORACLE (test infrastructure only): plain FP64 steady non-gray BTE-RTA solve.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does.  It shares no code with the GPU
library: geometry, boundary handling, sweeps, moments and the diffusion
correction are all written here (numpy/scipy) or in oracle/sweep.c.

Deviational variables are used throughout: theta = T - T_ref.  Because every
equation is linear in (e, theta), the temperatures it returns do not depend on
T_ref.

The steps follow the Methods section:
  * per-mode steady BTE, Eq. (4), first-order upwind finite volume, solved
    exactly per (band, direction) system (oracle/sweep.c);
  * equilibrium e0 = C theta_L / W_Omega, Eq. (11);
  * heat source split over bands by heat capacity and uniformly over
    directions (Numerical results, FinFET: "equilibrium phonon source"),
    S = Qdot C / (C_tot W);
  * sequential update of the lattice temperature, Eq. (5);
  * heat flux, Eq. (7), and the energy temperature T = T_ref + sum w e / C_tot;
  * synthetic scheme, Eqs. (9)-(10): the face-based divergence of the kinetic
    flux and a diffusion solve with kappa_bulk;
  * Fourier initial guess (Discussions): a Dirichlet diffusion solve.

Readings where the paper leaves the discrete form open are listed in the
module-level constants and the docstrings below (boundary formulas, the
lagged boundary treatment, the DSA reading of the synthetic update).
"""
from __future__ import annotations

import ctypes
import os
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import geometry as geo

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "_oracle_sweep.so")
        if not os.path.exists(path):
            from .build import build
            build()
        lib = ctypes.CDLL(path)
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.POINTER(ctypes.c_int64)
        i32 = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_sweep_all.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int64, i64, d, d, d, d, d, d, d, d, d, i32]
        lib.oracle_sweep_all.restype = None
        lib.oracle_sweep_system.argtypes = [ctypes.c_int64, ctypes.c_int32, i64, d, d, d,
                                            ctypes.c_double, ctypes.c_double, d, d, d, d]
        lib.oracle_sweep_system.restype = ctypes.c_int
        lib.oracle_sweep_all_sys.argtypes = lib.oracle_sweep_all.argtypes
        lib.oracle_sweep_all_sys.restype = None
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def threads(n=0):
    """OpenMP threads of the per-system loop (n > 0 sets them); returns the
    number the next transport() uses."""
    return int(_lib().oracle_threads(int(n)))


class OracleError(RuntimeError):
    pass


@dataclass
class Setup:
    g: geo.Geometry
    C: np.ndarray
    v: np.ndarray
    tau: np.ndarray
    s: np.ndarray
    w: np.ndarray
    W: float
    beta: float
    C_tot: float
    kappa: float
    Q: np.ndarray
    bc_kind: np.ndarray      # (NBF,) 0 thermalizing, 1 specular, 2 diffuse, 3 partial
    bc_theta: np.ndarray     # (NBF,) wall theta (thermalizing)
    bc_p: np.ndarray         # (NBF,) specularity (partial)
    sdotS: np.ndarray        # (NBF, D) s_i . S_f (outward)
    mirror: np.ndarray       # (NBF, D) mirror direction index, -1 where not needed
    T_ref: float
    L_c: float               # smallest extent of the domain
    L_cache: dict = field(default_factory=dict)


KIND = {"thermalizing": 0, "specular": 1, "diffuse": 2, "partial": 3}


def prepare(problem) -> Setup:
    """Geometry, band and quadrature tables and the boundary plan."""
    g = geo.build(problem.xyz, problem.cell_type, problem.cells, problem.bfaces, problem.bface_tag)
    C = np.asarray(problem.C, float); v = np.asarray(problem.v, float); tau = np.asarray(problem.tau, float)
    s = np.asarray(problem.s, float); w = np.asarray(problem.w, float)
    if np.any(~np.isfinite(C)) or np.any(C <= 0) or np.any(v <= 0) or np.any(tau <= 0):
        raise OracleError("invalid band table")
    if np.any(w <= 0) or np.any(np.abs(np.linalg.norm(s, axis=1) - 1) > 1e-12):
        raise OracleError("invalid quadrature")
    W = float(np.sum(w))
    beta = float(np.sum(C / tau))
    C_tot = float(np.sum(C))
    # bulk conductivity of the discrete quadrature (x-x component)
    kappa = float(np.sum(C * v * v * tau) * np.sum(w * s[:, 0] ** 2) / W)
    NBF = len(g.bf_owner)
    D = len(w)
    kinds = {b.tag: b for b in problem.boundaries}
    bc_kind = np.zeros(NBF, np.int32)
    bc_theta = np.zeros(NBF)
    bc_p = np.zeros(NBF)
    for j in range(NBF):
        b = kinds.get(int(g.bf_tag[j]))
        if b is None:
            raise OracleError(f"no boundary condition for tag {g.bf_tag[j]}")
        bc_kind[j] = KIND[b.kind]
        bc_theta[j] = b.T_wall - problem.T_ref
        bc_p[j] = b.specularity if b.kind == "partial" else (1.0 if b.kind == "specular" else 0.0)
    if not np.any(bc_kind == 0):
        raise OracleError("ill-posed: no thermalizing wall")
    Sbf = g.S[g.bf_owner, g.bf_local]                     # (NBF,3)
    sdotS = Sbf @ s.T                                    # (NBF,D)
    nhat = Sbf / np.linalg.norm(Sbf, axis=1)[:, None]
    mirror = -np.ones((NBF, D), np.int64)
    need = (bc_kind == 1) | (bc_kind == 3)
    for j in np.flatnonzero(need):
        sn = s @ nhat[j]
        refl = s - 2.0 * sn[:, None] * nhat[j][None, :]
        dist = np.linalg.norm(refl[:, None, :] - s[None, :, :], axis=2)
        m = np.argmin(dist, axis=1)
        if np.any(dist[np.arange(D), m] > 1e-9):
            raise OracleError("quadrature not closed under specular reflection")
        mirror[j] = m
    su = Setup(g=g, C=C, v=v, tau=tau, s=s, w=w, W=W, beta=beta, C_tot=C_tot, kappa=kappa,
               Q=np.asarray(problem.Q, float), bc_kind=bc_kind, bc_theta=bc_theta, bc_p=bc_p,
               sdotS=sdotS, mirror=mirror, T_ref=problem.T_ref,
               L_c=float(np.min(np.ptp(np.asarray(problem.xyz, float), axis=0))))
    return su


# ----------------------------------------------------------------------------
# diffusion operator (synthetic correction and Fourier guess)
# ----------------------------------------------------------------------------

def _face_conductivity(su: Setup, dist, nhat, mode):
    """Conductivity used on a face of the diffusion operator.

    mode "bulk": kappa_bulk, as printed in Eq. (10).
    mode "consistent" (default): the conductivity the discrete transport
      operator actually shows for smooth temperature fields, so that the
      correction neither stalls nor overshoots:
        kappa_f = sum_l C_l v_l Lambda_eff,l * sum_i w_i (s_i.n)^2 / W
                + sum_l C_l v_l * dist * sum_i w_i |s_i.n| / (2 W)
      with Lambda_eff = Lambda / (1 + 2 Lambda / L_c), L_c the smallest extent
      of the domain.  The second term is the numerical conductivity of the
      first-order upwind scheme (exact for a linear profile on a uniform 1D
      mesh); the first limits ballistic bands by the domain size.
    The choice only changes the iteration path: at the fixed point the
    correction vanishes whatever operator is used."""
    if mode == "bulk":
        return np.full(len(dist), su.kappa)
    if mode != "consistent":
        raise OracleError(f"unknown diffusion-correction conductivity {mode}")
    lam = su.v * su.tau
    leff = lam / (1.0 + 2.0 * lam / su.L_c)
    mu = nhat @ su.s.T                                   # (M, D)
    k_lim = np.sum(su.C * su.v * leff) * ((mu * mu) @ su.w) / su.W
    k_num = np.sum(su.C * su.v) * dist * (np.abs(mu) @ su.w) / (2.0 * su.W)
    return k_lim + k_num


def diffusion_operator(su: Setup, mode="consistent"):
    """Two-point-flux form of -div(kappa grad theta), multiplied by V:
       (L x)_c = sum_{interior f} T_f (x_c - x_n) + sum_{thermalizing f} T_f x_c,
       T_f = kappa_f A_f / |(x_n - x_c) . n_f|   (interior),
             kappa_f A_f / |(x_f - x_c) . n_f|   (wall),
    Neumann on every other boundary.  Returns (L, splu(L), dir_rhs) where
    dir_rhs = sum T_f theta_wall is the Dirichlet data of the Fourier problem.
    Cached per mode on the setup."""
    if mode in su.L_cache:
        return su.L_cache[mode]
    g = su.g
    N, F = g.N, g.F
    A = np.linalg.norm(g.S, axis=2)
    nh = g.S / A[:, :, None]
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    dir_rhs = np.zeros(N)
    for f in range(F):
        nb = g.nbr[:, f]
        inter = nb >= 0
        c = np.flatnonzero(inter)
        n = nb[inter]
        d = np.abs(np.einsum("ij,ij->i", g.xc[n] - g.xc[c], nh[c, f]))
        T = _face_conductivity(su, d, nh[c, f], mode) * A[c, f] / d
        diag[c] += T
        rows.append(c); cols.append(n); vals.append(-T)
        bnd = np.flatnonzero(~inter)
        j = -(nb[bnd] + 1)
        wall = su.bc_kind[j] == 0
        cb = bnd[wall]
        db = np.abs(np.einsum("ij,ij->i", g.xf[cb, f] - g.xc[cb], nh[cb, f]))
        Tb = _face_conductivity(su, 2.0 * db, nh[cb, f], mode) * A[cb, f] / db
        diag[cb] += Tb
        dir_rhs[cb] += Tb * su.bc_theta[j[wall]]
    rows.append(np.arange(N)); cols.append(np.arange(N)); vals.append(diag)
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    out = (L, spla.splu(L.tocsc()), dir_rhs)
    su.L_cache[mode] = out
    return out


def fourier_guess(su: Setup):
    """theta solving the Fourier problem -div(kappa_bulk grad theta) = Qdot
    with the wall temperatures (Discussions: Fourier initial guess)."""
    _, lu, dir_rhs = diffusion_operator(su, "bulk")
    return lu.solve(su.g.V * su.Q + dir_rhs)


# ----------------------------------------------------------------------------
# one iteration's pieces
# ----------------------------------------------------------------------------

def equilibrium(su: Setup, theta):
    """e0_lambda(c) = C_lambda theta(c) / W, Eq. (11).  Shape (B, N)."""
    return su.C[:, None] * theta[None, :] / su.W


def source(su: Setup):
    """S_lambda(c) = Qdot_c C_lambda / (C_tot W): equilibrium phonon source."""
    return su.Q[None, :] * su.C[:, None] / (su.C_tot * su.W)


def boundary_inflow(su: Setup, e, bdelta=None):
    """Inflow values on every boundary face for every (band, direction), from
    the previous iterate e (lagged), shape (B, D, NBF).  Only the entries with
    s_i . S_f < 0 are used.
      thermalizing: C theta_w / W
      specular:     e of the mirror direction at the owner cell
      diffuse:      sum_{out j} w_j (s_j.S) e_j / sum_{in k} w_k |s_k.S|
      partial(p):   p * specular + (1 - p) * diffuse
    bdelta (B, D, NBF), optional: second-order increments of the outgoing
    face values (the owner's value plus its reconstruction on the face)."""
    g = su.g
    B, D = len(su.C), len(su.w)
    NBF = len(g.bf_owner)
    eo = e[:, :, g.bf_owner]                     # (B, D, NBF) values at the owners
    if bdelta is not None:
        eo = eo + bdelta
    out = su.sdotS > 0                           # (NBF, D)
    inn = su.sdotS < 0
    wout = np.where(out, su.w[None, :] * su.sdotS, 0.0)          # (NBF, D)
    win = np.where(inn, su.w[None, :] * (-su.sdotS), 0.0)
    diff = np.einsum("fd,bdf->bf", wout, eo) / win.sum(axis=1)[None, :]   # (B, NBF)
    inflow = np.zeros((B, D, NBF))
    th = su.bc_kind == 0
    inflow[:, :, th] = (su.C[:, None] * su.bc_theta[th][None, :] / su.W)[:, None, :]
    for kind in (1, 2, 3):
        m = np.flatnonzero(su.bc_kind == kind)
        if len(m) == 0:
            continue
        dif = np.broadcast_to(diff[:, None, m], (B, D, len(m)))
        if kind == 2:
            inflow[:, :, m] = dif
            continue
        mir = su.mirror[m]                                   # (len m, D)
        spec = np.take_along_axis(eo[:, :, m], mir.T[None, :, :], axis=1)
        p = su.bc_p[m][None, None, :]
        inflow[:, :, m] = p * spec + (1.0 - p) * dif
    return inflow


def transport(su: Setup, theta, inflow, corr=None):
    """Solve every (band, direction) system for the given lattice temperature
    and boundary inflow.  Returns e and per-volume outflow, shape (B, D, N).
    corr (B, D, N), optional: an extra right-hand side per system (the
    second-order scheme's deferred correction)."""
    g = su.g
    B, D, N = len(su.C), len(su.w), g.N
    rhs = np.ascontiguousarray(equilibrium(su, theta) / su.tau[:, None] + source(su))
    e = np.empty((B, D, N))
    outflux = np.empty((B, D, N))
    status = np.zeros(B * D, np.int32)
    nbr = np.ascontiguousarray(g.nbr, np.int64)
    S = np.ascontiguousarray(g.S)
    inflow = np.ascontiguousarray(inflow)
    s = np.ascontiguousarray(su.s)
    inv_tau = 1.0 / su.tau
    args = (N, g.F, B, D, len(g.bf_owner), _p(nbr, ctypes.c_int64), _p(S), _p(g.V), _p(s), _p(su.v), _p(inv_tau))
    if corr is None:
        _lib().oracle_sweep_all(*args, _p(rhs), _p(inflow), _p(e), _p(outflux), _p(status, ctypes.c_int32))
    else:
        rhs = np.ascontiguousarray(rhs[:, None, :] + corr)
        _lib().oracle_sweep_all_sys(*args, _p(rhs), _p(inflow), _p(e), _p(outflux), _p(status, ctypes.c_int32))
    if np.any(status == 2):
        raise MemoryError("oracle sweep allocation failed")
    for k in np.flatnonzero(status == 1):    # cyclic upwind graph: sparse direct solve
        b, i = divmod(int(k), D)
        r = rhs[b] if corr is None else rhs[b, i]
        e[b, i], outflux[b, i] = _direct_system(su, b, i, r, inflow[b, i])
    return e, outflux


def transport_systems(su: Setup, theta, inflow, systems):
    """Solve only the listed (band, direction) systems (same arithmetic as
    transport()); returns {(b, i): e}.  inflow may be given for those systems
    only, as a dict {(b, i): (NBF,) array}, or as the full (B, D, NBF) array."""
    g = su.g
    N = g.N
    nbr = np.ascontiguousarray(g.nbr, np.int64)
    S = np.ascontiguousarray(g.S)
    out = {}
    for (b, i) in systems:
        rhs = np.ascontiguousarray(su.C[b] * theta / (su.W * su.tau[b]) + su.Q * su.C[b] / (su.C_tot * su.W))
        inf = np.ascontiguousarray(inflow[(b, i)] if isinstance(inflow, dict) else inflow[b, i])
        e = np.empty(N)
        flux = np.empty(N)
        s = np.ascontiguousarray(su.s[i])
        st = _lib().oracle_sweep_system(N, g.F, _p(nbr, ctypes.c_int64), _p(S), _p(g.V), _p(s), float(su.v[b]),
                                        float(1.0 / su.tau[b]), _p(rhs), _p(inf), _p(e), _p(flux))
        if st == 1:
            e, flux = _direct_system(su, b, i, rhs, inf)
        elif st != 0:
            raise MemoryError("oracle sweep allocation failed")
        out[(b, i)] = e
    return out


def _direct_system(su: Setup, b, i, rhs, inflow_bi):
    g = su.g
    N, F = g.N, g.F
    a = np.einsum("cfk,k->cf", g.S, su.s[i]) / g.V[:, None]
    v = su.v[b]
    diag = 1.0 / su.tau[b] + v * np.where(a > 0, a, 0.0).sum(axis=1)
    rows, cols, vals = [np.arange(N)], [np.arange(N)], [diag]
    r = rhs.copy()
    for f in range(F):
        nb = g.nbr[:, f]
        m = (a[:, f] < 0) & (nb >= 0)
        rows.append(np.flatnonzero(m)); cols.append(nb[m]); vals.append(-v * (-a[m, f]))
        mb = (a[:, f] < 0) & (nb < 0)
        r[mb] += v * (-a[mb, f]) * inflow_bi[-(nb[mb] + 1)]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    e = spla.spsolve(A.tocsc(), r)
    out = np.zeros(N)
    for f in range(F):
        nb = g.nbr[:, f]
        up = np.where(nb >= 0, e[np.maximum(nb, 0)], inflow_bi[np.maximum(-(nb + 1), 0)])
        out += np.where(a[:, f] > 0, a[:, f] * e, np.where(a[:, f] < 0, a[:, f] * up, 0.0))
    return e, out


def moments(su: Setup, e):
    """theta_seq (Eq. (5)), energy temperature theta and heat flux q (Eq. (7))."""
    we = np.einsum("i,bic->bc", su.w, e)                       # sum_i w_i e_bi(c)
    theta_seq = np.einsum("b,bc->c", 1.0 / su.tau, we) / su.beta
    theta = we.sum(axis=0) / su.C_tot
    q = np.einsum("b,i,ik,bic->ck", su.v, su.w, su.s, e)
    return theta_seq, theta, q


def divergence(su: Setup, outflux):
    """Face-based divergence of the kinetic heat flux (per volume), using the
    same upwind face values as the transport solve:
      (D_h q)_c = sum_lambda sum_i w_i v_lambda sum_f a_cfi e_up."""
    return np.einsum("b,i,bic->c", su.v, su.w, outflux)


def boundary_flows(su: Setup, e, inflow, bdelta=None):
    """Heat leaving through every boundary face (positive outward):
       sum_lambda sum_i w_i v_lambda (s_i . S_f) e_up
    (bdelta: second-order increments of the outgoing face values)."""
    g = su.g
    eo = e[:, :, g.bf_owner]
    if bdelta is not None:
        eo = eo + bdelta
    up = np.where((su.sdotS > 0).T[None, :, :], eo, inflow)    # (B, D, NBF)
    return np.einsum("b,i,fi,bif->f", su.v, su.w, su.sdotS, up)


# ----------------------------------------------------------------------------
# second-order upwind by deferred correction (an extension of the method's
# first-order face values; the implicit sweep stays first order)
# ----------------------------------------------------------------------------

def lsq_weights(su: Setup):
    """Least-squares cell gradients over the interior face neighbours:
    G_c = sum_f w_cf (e_n(f) - e_c), with d_f = x_n(f) - x_c (cell centres),
    M_c = sum_f d_f d_f^T and w_cf = M_c^-1 d_f in the mesh's dimension.  A
    cell whose neighbour offsets do not span the dimension (smallest to largest
    eigenvalue of M_c below 1e-8) has no gradient: w = 0, its faces stay first
    order.  Returns (N, F, 3); cached on the setup."""
    if "lsq" in su.L_cache:
        return su.L_cache["lsq"]
    g = su.g
    dim = g.dim
    inter = g.nbr >= 0
    nbc = np.where(inter, g.nbr, 0)
    d = np.where(inter[:, :, None], g.xc[nbc] - g.xc[:, None, :], 0.0)[:, :, :dim]
    M = np.einsum("cfi,cfj->cij", d, d)
    ev = np.linalg.eigvalsh(M)
    ok = ev[:, 0] > 1e-8 * ev[:, -1]
    Wt = np.zeros((g.N, g.F, 3))
    Mi = np.linalg.inv(np.where(ok[:, None, None], M, np.eye(dim)[None]))
    Wt[:, :, :dim] = np.einsum("cij,cfj->cfi", Mi, d) * ok[:, None, None]
    su.L_cache["lsq"] = Wt
    return Wt


def reconstruct_fields(su: Setup, E, dirs):
    """Second-order increments of the fields E (K, N) of the directions dirs
    (K,): with the gradient G_c of each field, the face value seen from cell
    c on its face f is e_c + G_c . (x_f - x_c).  Returns
      div (K, N):     sum_f a_cf delta_f, the per-volume net outflow carried by
                      the increments of the upwind side: outgoing faces
                      (a_cf > 0) take the cell's own, incoming interior faces
                      the neighbour's G_n . (x_f - x_n), boundary inflow none;
      bdelta (K, NBF): G_owner . (x_f - x_owner) on every boundary face (the
                      increment of its outgoing values)."""
    g = su.g
    Wt = lsq_weights(su)
    inter = g.nbr >= 0
    nbc = np.where(inter, g.nbr, 0)
    de = np.where(inter[None], E[:, nbc] - E[:, :, None], 0.0)          # (K, N, F)
    G = np.einsum("kcf,cfx->kcx", de, Wt)                                 # (K, N, 3)
    d_own = np.einsum("kcx,cfx->kcf", G, g.xf - g.xc[:, None, :])        # own side of every face
    d_nbr = np.einsum("kcfx,cfx->kcf", G[:, nbc], g.xf - g.xc[nbc])       # neighbour's side
    a = np.einsum("cfx,kx->kcf", g.S, su.s[dirs]) / g.V[None, :, None]
    div = np.where(a > 0, a * d_own, np.where((a < 0) & inter[None], a * d_nbr, 0.0)).sum(axis=2)
    bdelta = d_own[:, g.bf_owner, g.bf_local]
    return div, bdelta


def reconstruct(su: Setup, e):
    """reconstruct_fields for every (band, direction) system of e (B, D, N):
    div (B, D, N) and bdelta (B, D, NBF)."""
    B, D = e.shape[0], e.shape[1]
    div = np.empty(e.shape)
    bdelta = np.empty((B, D, len(su.g.bf_owner)))
    for b in range(B):
        div[b], bdelta[b] = reconstruct_fields(su, e[b], np.arange(D))
    return div, bdelta


def solve_system_order2(su: Setup, b, i, rhs, inflow_bi, tol=1e-13, max_iter=10000):
    """One (band, direction) system with second-order face values, by
    deferred correction: e^{k+1} = A1^-1 (rhs - v div(e^k)), A1 the
    first-order upwind matrix (exact sweep).  Returns (e, iterations)."""
    g = su.g
    N = g.N
    nbr = np.ascontiguousarray(g.nbr, np.int64)
    S = np.ascontiguousarray(g.S)
    s = np.ascontiguousarray(su.s[i])
    inf = np.ascontiguousarray(inflow_bi, float)
    e = np.zeros(N)
    flux = np.empty(N)
    for k in range(1, max_iter + 1):
        div, _ = reconstruct_fields(su, e[None, :], np.array([i]))
        r = np.ascontiguousarray(rhs - su.v[b] * div[0])
        new = np.empty(N)
        st = _lib().oracle_sweep_system(N, g.F, _p(nbr, ctypes.c_int64), _p(S), _p(g.V), _p(s), float(su.v[b]),
                                        float(1.0 / su.tau[b]), _p(r), _p(inf), _p(new), _p(flux))
        if st == 1:
            new, _ = _direct_system(su, b, i, r, inf)
        elif st != 0:
            raise MemoryError("oracle sweep allocation failed")
        ch = np.max(np.abs(new - e)) / max(np.max(np.abs(new)), 1e-300)
        e = new
        if ch <= tol:
            return e, k
    raise OracleError("deferred correction did not converge")


# ----------------------------------------------------------------------------
# outer acceleration (an addition to the method; the fixed point is unchanged)
# ----------------------------------------------------------------------------

def anderson_next(X_hist, G_hist):
    """Anderson acceleration of a fixed-point iteration x = G(x) (D. G.
    Anderson, J. ACM 12 (1965); the unconstrained least-squares form of
    H. F. Walker and P. Ni, SIAM J. Numer. Anal. 49 (2011)).

    X_hist, G_hist: the last m+1 iterates x_j and their images G(x_j), oldest
    first.  With the residuals f_j = G(x_j) - x_j and the columns
    dF_j = f_{j+1} - f_j, dG_j = G(x_{j+1}) - G(x_j) (j over the history),
    the next iterate is
        x_new = G(x_k) - dG gamma,   gamma = argmin_gamma || f_k - dF gamma ||_2
    (least squares by a library routine).  One entry of history (m = 0)
    gives the plain iteration x_new = G(x_k)."""
    g = G_hist[-1]
    if len(X_hist) < 2:
        return g.copy()
    F = [gj - xj for xj, gj in zip(X_hist, G_hist)]
    dF = np.stack([F[j + 1] - F[j] for j in range(len(F) - 1)], axis=1)
    dG = np.stack([G_hist[j + 1] - G_hist[j] for j in range(len(G_hist) - 1)], axis=1)
    gamma = np.linalg.lstsq(dF, F[-1], rcond=None)[0]
    return g - dG @ gamma


def _accel_mask(su: Setup):
    """(B, D, NBF) mask of the inflow entries that change between iterations:
    incoming directions of the specular, diffuse and partial walls."""
    B = len(su.C)
    m = ((su.sdotS < 0) & (su.bc_kind != 0)[:, None]).T        # (D, NBF)
    return np.broadcast_to(m[None, :, :], (B,) + m.shape)


def accel_state(su: Setup, theta, inflow):
    """The state of the outer iteration as one vector: the lattice
    temperature theta (N) followed by the reflective walls' incoming values
    in temperature units, inflow * W / C_lambda, band-major over the masked
    (band, direction, face) entries."""
    return np.concatenate([theta, (inflow * (su.W / su.C)[:, None, None])[_accel_mask(su)]])


def accel_unpack(su: Setup, x, inflow_like):
    """Inverse of accel_state: (theta, inflow); entries outside the mask
    (thermalizing walls, outgoing directions) are taken from inflow_like."""
    N = su.g.N
    inflow = np.array(inflow_like, copy=True)
    m = _accel_mask(su)
    inflow[m] = x[N:] * np.broadcast_to((su.C / su.W)[:, None, None], inflow.shape)[m]
    return x[:N].copy(), inflow


# ----------------------------------------------------------------------------
# the iteration
# ----------------------------------------------------------------------------

@dataclass
class Result:
    T_lattice: np.ndarray
    T: np.ndarray
    q: np.ndarray
    theta_L: np.ndarray
    iterations: int
    residual: float
    energy_defect: float
    flows_by_tag: dict
    history: list = field(default_factory=list)
    seconds: float = 0.0
    e: np.ndarray = None


def energy_defect(su: Setup, flows):
    heat_in = float(np.sum(su.g.V * su.Q))
    net_out = float(np.sum(flows))
    scale = max(abs(heat_in), 0.5 * float(np.sum(np.abs(flows))))
    return abs(net_out - heat_in) / scale if scale > 0 else 0.0


def solve(problem, scheme=None, tol=1e-13, max_iter=100000, T_init=None, defect_tol=None,
          setup: Setup = None, keep_e=False, verbose=False, time_limit=None, dsa_kappa="consistent",
          accel=None, depth=5, order=1):
    """Iterate to the steady state.

    scheme: "sequential" (Eq. (5)), "synthetic" (default; the DSA reading of
    Eqs. (9)-(10): theta^{n+1} = theta_seq + delta), or "synthetic_literal"
    (theta^{n+1} = theta^n + delta, q_nonF built with theta^n as printed).
    Both synthetic forms solve  L delta = V (Qdot - D_h' q), where D_h' is the
    face-based divergence of Eq. (14) without the faces of reflective
    (specular, diffuse, partial) walls: their net flux is zero at the fixed
    point, and with lagged wall inflow its transient value would otherwise be
    amplified by the correction.  dsa_kappa selects the conductivity of L
    (see _face_conductivity).

    accel="anderson": Anderson acceleration of depth `depth` (anderson_next)
    of the outer iteration, whose state is the lattice temperature and the
    lagged inflow of the reflective walls (accel_state); the converged fields
    are those of the plain iteration.

    order=2: second-order upwind face values (reconstruct_fields) by deferred
    correction: each sweep keeps the first-order implicit operator and moves
    the reconstruction increments of the previous distribution to its
    right-hand side; the boundary conditions, the divergence of the synthetic
    correction and the boundary flows use the same second-order face values.
    At the fixed point the discrete equations are the second-order ones.

    Stops when max|theta^{n+1} - theta^n| / max|theta^{n+1}| <= tol and, if
    defect_tol is given, the energy defect is <= defect_tol; theta^{n+1} is
    the image of theta^n under one iteration (before any acceleration)."""
    t0 = time.perf_counter()
    su = setup if setup is not None else prepare(problem)
    scheme = scheme or problem.scheme
    if scheme not in ("sequential", "synthetic", "synthetic_literal"):
        raise OracleError(f"unknown scheme {scheme}")
    if T_init is None:
        theta = fourier_guess(su)
    else:
        theta = np.asarray(T_init, float) - su.T_ref
    e = np.broadcast_to(equilibrium(su, theta)[:, None, :], (len(su.C), len(su.w), su.g.N))
    if accel not in (None, "anderson"):
        raise OracleError(f"unknown outer acceleration {accel}")
    if order not in (1, 2):
        raise OracleError(f"unknown spatial order {order}")
    if order == 2 and accel is not None:
        raise OracleError("outer acceleration of the second-order scheme is not provided")
    hist = []
    res = np.inf
    it = 0
    div_o = bd_o = None
    if order == 2:
        e = np.ascontiguousarray(e)
        div_o, bd_o = reconstruct(su, e)
    inflow = boundary_inflow(su, e, bd_o)
    inflow_used, theta_new, bd_used = inflow, theta, bd_o
    X_hist, G_hist = [], []
    while it < max_iter:
        corr = None if order == 1 else -su.v[:, None, None] * div_o
        e, outflux = transport(su, theta, inflow, corr)
        if order == 2:
            outflux = outflux + div_o
        bd_used = bd_o
        theta_seq, th_energy, q = moments(su, e)
        if scheme == "sequential":
            theta_new = theta_seq
        else:
            r = su.Q - divergence(su, outflux)
            flows = boundary_flows(su, e, inflow, bd_used)
            refl = su.bc_kind != 0
            np.add.at(r, su.g.bf_owner[refl], flows[refl] / su.g.V[su.g.bf_owner[refl]])
            delta = diffusion_operator(su, dsa_kappa)[1].solve(su.g.V * r)
            theta_new = (theta_seq if scheme == "synthetic" else theta) + delta
        denom = np.max(np.abs(theta_new))
        if not np.all(np.isfinite(theta_new)):
            raise OracleError("iteration diverged (non-finite temperature)")
        res = float(np.max(np.abs(theta_new - theta)) / denom) if denom > 0 else 0.0
        theta_prev, inflow_used = theta, inflow
        theta = theta_new
        it += 1
        flows = boundary_flows(su, e, inflow_used, bd_used)
        dfc = energy_defect(su, flows)
        hist.append((res, dfc))
        if verbose:
            print(f"oracle it {it} res {res:.3e} defect {dfc:.3e}", flush=True)
        if res <= tol and (defect_tol is None or dfc <= defect_tol):
            break
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
        if order == 2:
            div_o, bd_o = reconstruct(su, e)
        inflow = boundary_inflow(su, e, bd_o)
        if accel == "anderson" and depth > 0:
            # x_n = (theta^n, inflow^n) -> G(x_n) = (theta^{n+1}, inflow from e^{n+1})
            X_hist.append(accel_state(su, theta_prev, inflow_used))
            G_hist.append(accel_state(su, theta, inflow))
            del X_hist[:-(depth + 1)], G_hist[:-(depth + 1)]
            theta, inflow = accel_unpack(su, anderson_next(X_hist, G_hist), inflow)
    inflow = inflow_used
    theta = theta_new
    flows = boundary_flows(su, e, inflow, bd_used)
    by_tag = {int(t): float(np.sum(flows[su.g.bf_tag == t])) for t in np.unique(su.g.bf_tag)}
    return Result(T_lattice=su.T_ref + theta, T=su.T_ref + th_energy, q=q, theta_L=theta,
                  iterations=it, residual=res, energy_defect=energy_defect(su, flows),
                  flows_by_tag=by_tag, history=hist, seconds=time.perf_counter() - t0,
                  e=e if keep_e else None)
