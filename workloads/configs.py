"""The five synthetic workloads (and reduced-size variants for parity tests).

Seeds: workload k draws from numpy.random.default_rng(k); the j-th solve of a
multi-solve workload draws from default_rng(1000 k + j).
Units: SI (lengths in metres).
"""
from __future__ import annotations

import numpy as np

from . import meshes as M
from .problem import Boundary, Problem
from .tables import bose_einstein_bands, gl_azimuth_quadrature, inplane_quadrature, mean_free_path

NM = 1e-9


# ----------------------------------------------------------------------------
# 1: 2D gray square, plain FP64, sequential
# ----------------------------------------------------------------------------

def config1(n=16, L=100 * NM, D=16, tau=16.7e-12):
    xs = np.linspace(0, L, n + 1)
    xyz, cells, bf, tags = M.structured_quad(xs, xs)
    s, w = inplane_quadrature(D)
    return Problem(
        name=f"gray2d_{n}x{n}_D{D}", dim=2, xyz=xyz, cell_type="quad4", cells=cells,
        bfaces=bf, bface_tag=tags,
        boundaries=[Boundary(M.TAG_X0, "thermalizing", 301.0), Boundary(M.TAG_X1, "thermalizing", 299.0),
                    Boundary(M.TAG_Y0, "specular"), Boundary(M.TAG_Y1, "specular")],
        C=np.array([1.66e6]), v=np.array([6000.0]), tau=np.array([tau]),
        s=s, w=w, Q=np.zeros(len(cells)), T_ref=300.0, scheme="sequential", precision="fp64",
        meta={"config": 1})


# ----------------------------------------------------------------------------
# 2: 3D non-gray box
# ----------------------------------------------------------------------------

def config2(n=24, L=1000 * NM, B=16, n_polar=8, n_azim=16, seed=2):
    rng = np.random.default_rng(seed)
    xs = np.linspace(0, L, n + 1)
    xyz, cells = M.structured_hex(xs, xs, xs)
    bf = M.hex_boundary(cells)
    tags = M.box_tags(xyz, bf, (0, 0, 0), (L, L, L), 1e-6 * L)
    C, v, tau = bose_einstein_bands(rng, B)
    s, w = gl_azimuth_quadrature(n_polar, n_azim)
    return Problem(
        name=f"box3d_{n}^3_B{B}_D{len(w)}", dim=3, xyz=xyz, cell_type="hex8", cells=cells,
        bfaces=bf, bface_tag=tags,
        boundaries=[Boundary(M.TAG_X0, "thermalizing", 301.0), Boundary(M.TAG_X1, "thermalizing", 299.0)]
        + [Boundary(t, "diffuse") for t in (M.TAG_Y0, M.TAG_Y1, M.TAG_Z0, M.TAG_Z1)],
        C=C, v=v, tau=tau, s=s, w=w, Q=np.zeros(len(cells)), T_ref=300.0,
        scheme="synthetic", precision="mixed", meta={"config": 2})


# ----------------------------------------------------------------------------
# 3: FinFET-like tets
# ----------------------------------------------------------------------------

def finfet_grid(scale=1.0):
    """Coordinate lines of the structured grid that conforms to the fin.
    scale < 1 coarsens every segment (parity-test sizes)."""
    def cnt(n):
        return max(1, int(round(n * scale)))
    xs = np.concatenate([M.graded(0, 95, cnt(12), 5.0, "b")[:-1], np.linspace(95, 105, cnt(4) + 1)[:-1],
                         M.graded(105, 200, cnt(12), 5.0, "a")])
    ys = np.concatenate([M.graded(0, 50, cnt(7), 3.0, "b")[:-1], np.linspace(50, 150, cnt(14) + 1)[:-1],
                         M.graded(150, 200, cnt(7), 3.0, "a")])
    zs = np.concatenate([M.graded(0, 100, cnt(30), 4.0, "b")[:-1], np.linspace(100, 140, cnt(10) + 1)])
    return xs * NM, ys * NM, zs * NM


def config3(scale=1.0, B=32, n_polar=6, n_azim=16, seed=3, Q0=1e18, sigma=5 * NM, p=0.5):
    rng = np.random.default_rng(seed)
    xs, ys, zs = finfet_grid(scale)

    def keep(cx, cy, cz):
        sub = cz < 100 * NM
        fin = (cx > 95 * NM) & (cx < 105 * NM) & (cy > 50 * NM) & (cy < 150 * NM) & (cz < 140 * NM)
        return sub | fin

    xyz, hexes = M.structured_hex(xs, ys, zs, keep=keep)
    cells = M.hex_to_tets(hexes)
    bf = M.tet_boundary(cells)
    tags = M.tag_by_plane(xyz, bf, [(lambda c: np.abs(c[:, 2]) < 1e-3 * NM, 1)], default=2)
    C, v, tau = bose_einstein_bands(rng, B)
    s, w = gl_azimuth_quadrature(n_polar, n_azim)
    cen = xyz[cells].mean(axis=1)
    r2 = np.sum((cen - np.array([100, 100, 140]) * NM) ** 2, axis=1)
    Q = Q0 * np.exp(-r2 / (2 * sigma ** 2))
    return Problem(
        name=f"finfet_tet{len(cells)}_B{B}_D{len(w)}", dim=3, xyz=xyz, cell_type="tet4", cells=cells,
        bfaces=bf, bface_tag=tags,
        boundaries=[Boundary(1, "thermalizing", 300.0), Boundary(2, "partial", specularity=p)],
        C=C, v=v, tau=tau, s=s, w=w, Q=Q, T_ref=300.0, scheme="synthetic", precision="mixed",
        meta={"config": 3})


# ----------------------------------------------------------------------------
# 4: batch of porous films
# ----------------------------------------------------------------------------

def _draw_pores(rng, Lx, Ly, h_est):
    n = int(rng.integers(0, 9))
    pores = []
    tries = 0
    while len(pores) < n and tries < 500:
        tries += 1
        r = rng.uniform(0.05, 0.15) * min(Lx, Ly)
        lo_x, hi_x = r + 3 * h_est, Lx - r - 3 * h_est
        lo_y, hi_y = r + 3 * h_est, Ly - r - 3 * h_est
        if hi_x <= lo_x or hi_y <= lo_y:
            continue
        cx = rng.uniform(lo_x, hi_x)
        cy = rng.uniform(lo_y, hi_y)
        if all(np.hypot(cx - px, cy - py) > r + pr + 3 * h_est for (px, py, pr) in pores):
            pores.append((cx, cy, r))
    return pores


def porous_problem(seed, n_lo=2000, n_hi=40000, B=8, D=32, kn_lo=0.1, kn_hi=10.0):
    rng = np.random.default_rng(seed)
    Lx = np.exp(rng.uniform(np.log(200), np.log(2000))) * NM
    Ly = np.exp(rng.uniform(np.log(200), np.log(2000))) * NM
    n_target = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
    h_est = np.sqrt(2 * Lx * Ly / n_target)
    pores = _draw_pores(rng, Lx, Ly, h_est)
    for attempt in range(20):
        try:
            xyz, tri, bf, tags = M.porous_film(rng, Lx, Ly, pores, n_target)
            break
        except RuntimeError:
            continue
    else:
        raise RuntimeError("porous mesh generation failed")
    C, v, tau = bose_einstein_bands(rng, B)
    kn = np.exp(rng.uniform(np.log(kn_lo), np.log(kn_hi)))
    tau = tau * (kn * Lx / mean_free_path(C, v, tau))
    s, w = inplane_quadrature(D)
    return Problem(
        name=f"porous_{len(tri)}_p{len(pores)}_Kn{kn:.3g}", dim=2, xyz=xyz, cell_type="tri3", cells=tri,
        bfaces=bf, bface_tag=tags,
        boundaries=[Boundary(1, "thermalizing", 301.0), Boundary(2, "thermalizing", 299.0),
                    Boundary(3, "specular"), Boundary(4, "diffuse")],
        C=C, v=v, tau=tau, s=s, w=w, Q=np.zeros(len(tri)), T_ref=300.0, scheme="synthetic",
        precision="mixed", meta={"config": 4, "Kn": kn, "pores": len(pores), "Lx": Lx, "Ly": Ly})


def config4(n_solves=64, seed=4, **kw):
    return [porous_problem(1000 * seed + j, **kw) for j in range(n_solves)]


# ----------------------------------------------------------------------------
# 5: serving stream
# ----------------------------------------------------------------------------

def _rect_request(rng, seed, size_scale=1.0):
    L = np.exp(rng.uniform(np.log(100), np.log(2000))) * NM
    aspect = np.exp(rng.uniform(np.log(0.5), np.log(2.0)))
    N = int(size_scale * np.exp(rng.uniform(np.log(2000), np.log(40000))))
    nx = max(4, int(round(np.sqrt(N * aspect))))
    ny = max(4, int(round(N / nx)))
    xyz, cells, bf, tags = M.structured_quad(np.linspace(0, L * aspect, nx + 1), np.linspace(0, L, ny + 1))
    D = int(rng.choice([32, 64, 96, 128]))
    s, w = inplane_quadrature(D)
    bounds = [Boundary(M.TAG_X0, "thermalizing", 300.0), Boundary(M.TAG_X1, "thermalizing", 300.0),
              Boundary(M.TAG_Y0, "diffuse"), Boundary(M.TAG_Y1, "specular")]
    cen = xyz[cells].mean(axis=1)
    centre = np.array([0.5 * L * aspect, 0.5 * L])
    return "rect2d", 2, xyz, "quad4", cells, bf, tags, bounds, s, w, cen, centre, L


def _box_request(rng, seed, size_scale=1.0):
    L = np.exp(rng.uniform(np.log(100), np.log(2000))) * NM
    N = int(size_scale * np.exp(rng.uniform(np.log(10000), np.log(200000))))
    n = max(4, int(round(N ** (1 / 3))))
    xs = np.linspace(0, L, n + 1)
    xyz, cells = M.structured_hex(xs, xs, xs)
    bf = M.hex_boundary(cells)
    tags = M.box_tags(xyz, bf, (0, 0, 0), (L, L, L), 1e-6 * L)
    D = int(rng.choice([32, 64, 96, 128]))
    npol, naz = {32: (4, 8), 64: (8, 8), 96: (6, 16), 128: (8, 16)}[D]
    s, w = gl_azimuth_quadrature(npol, naz)
    bounds = [Boundary(M.TAG_Z0, "thermalizing", 300.0)] + [
        Boundary(t, "diffuse") for t in (M.TAG_X0, M.TAG_X1, M.TAG_Y0, M.TAG_Y1)] + [
        Boundary(M.TAG_Z1, "specular")]
    cen = xyz[cells].mean(axis=1)
    return "box3d", 3, xyz, "hex8", cells, bf, tags, bounds, s, w, cen, np.array([L / 2, L / 2, L]), L


def _finfet_request(rng, seed, size_scale=1.0):
    N = int(size_scale * np.exp(rng.uniform(np.log(10000), np.log(200000))))
    scale = (N / 144480.0) ** (1 / 3)
    xs, ys, zs = finfet_grid(scale)

    def keep(cx, cy, cz):
        return (cz < 100 * NM) | ((cx > 95 * NM) & (cx < 105 * NM) & (cy > 50 * NM) & (cy < 150 * NM) & (cz < 140 * NM))

    xyz, hexes = M.structured_hex(xs, ys, zs, keep=keep)
    cells = M.hex_to_tets(hexes)
    bf = M.tet_boundary(cells)
    tags = M.tag_by_plane(xyz, bf, [(lambda c: np.abs(c[:, 2]) < 1e-3 * NM, 1)], default=2)
    D = int(rng.choice([32, 64, 96, 128]))
    npol, naz = {32: (4, 8), 64: (8, 8), 96: (6, 16), 128: (8, 16)}[D]
    s, w = gl_azimuth_quadrature(npol, naz)
    bounds = [Boundary(1, "thermalizing", 300.0), Boundary(2, "partial", specularity=0.5)]
    cen = xyz[cells].mean(axis=1)
    return "finfet", 3, xyz, "tet4", cells, bf, tags, bounds, s, w, cen, np.array([100, 100, 140]) * NM, 100 * NM


def serving_request(seed, families=("rect2d", "box3d", "finfet"), size_scale=1.0):
    """One solve request of the serving stream: family uniform over the three,
    bands U{8..32}, Gaussian hot spot with peak log-uniform in [1e16, 1e19] W/m^3.
    size_scale < 1 shrinks the cell-count ranges (test sizes)."""
    rng = np.random.default_rng(seed)
    fam = families[int(rng.integers(0, len(families)))]
    gen = {"rect2d": _rect_request, "box3d": _box_request, "finfet": _finfet_request}[fam]
    kind, dim, xyz, ct, cells, bf, tags, bounds, s, w, cen, centre, L = gen(rng, seed, size_scale)
    B = int(rng.integers(8, 33))
    C, v, tau = bose_einstein_bands(rng, B)
    q0 = np.exp(rng.uniform(np.log(1e16), np.log(1e19)))
    sigma = 0.1 * L
    r2 = np.sum((cen - centre[None, :dim]) ** 2, axis=1)
    Q = q0 * np.exp(-r2 / (2 * sigma ** 2))
    return Problem(name=f"{kind}_{len(cells)}_B{B}_D{len(w)}", dim=dim, xyz=xyz, cell_type=ct, cells=cells,
                   bfaces=bf, bface_tag=tags, boundaries=bounds, C=C, v=v, tau=tau, s=s, w=w, Q=Q,
                   T_ref=300.0, scheme="synthetic", precision="mixed",
                   meta={"config": 5, "family": kind, "seed": seed})


class RequestStream:
    """The requests serving_request(first + j), j < n, generated ahead of use
    on a background thread (at most `ahead` beyond the highest index asked
    for) and dropped with release(j), so a long stream never holds all its
    meshes.  Indexing blocks until the request exists."""

    def __init__(self, first, n, ahead=48, **kw):
        import threading
        self.first, self.n, self.ahead, self.kw = first, n, ahead, kw
        self.items = {}
        self.want = 0
        self.next = 0
        self.cv = threading.Condition()
        self.stop = False
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def _run(self):
        while True:
            with self.cv:
                while not self.stop and (self.next >= self.n or self.next > self.want + self.ahead):
                    self.cv.wait()
                if self.stop:
                    return
                j = self.next
            p = serving_request(self.first + j, **self.kw)
            with self.cv:
                self.items[j] = p
                self.next = j + 1
                self.cv.notify_all()

    def __len__(self):
        return self.n

    def __getitem__(self, j):
        with self.cv:
            self.want = max(self.want, j)
            self.cv.notify_all()
            while j not in self.items:
                if j < self.next:
                    raise KeyError(f"request {j} was released")
                self.cv.wait()
            return self.items[j]

    def release(self, j):
        with self.cv:
            self.items.pop(j, None)

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()


def poisson_arrivals(n, rate, seed=5):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


# ----------------------------------------------------------------------------
# reduced-size variants (parity tests): same recipes, fewer cells/bands/dirs
# ----------------------------------------------------------------------------

def config2_small(n=7, B=5, n_polar=4, n_azim=8, seed=2):
    return config2(n=n, B=B, n_polar=n_polar, n_azim=n_azim, seed=seed)


def config3_small(scale=0.25, B=6, n_polar=4, n_azim=8, seed=3):
    return config3(scale=scale, B=B, n_polar=n_polar, n_azim=n_azim, seed=seed)


def config4_small(n_solves=4, seed=4):
    return [porous_problem(1000 * seed + j, n_lo=150, n_hi=900) for j in range(n_solves)]
