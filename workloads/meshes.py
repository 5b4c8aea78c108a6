"""Seeded synthetic mesh generators (input generation only).

Nothing here computes any part of the transport method: these functions only
produce node coordinates, cell connectivity and tagged boundary faces, the raw
inputs a user would export from a mesher.  Both the GPU path and the oracle
consume the same arrays.

Cell node orderings:
  quad4: counter-clockwise (x,y) corners.
  hex8 : bottom face 0-1-2-3 counter-clockwise seen from +z, then the top face
         4-5-6-7 directly above.
  tri3 : counter-clockwise.
  tet4 : any order (positive orientation is not required by either consumer).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay

# Boundary tags used by the box generators.
TAG_X0, TAG_X1, TAG_Y0, TAG_Y1, TAG_Z0, TAG_Z1 = 1, 2, 3, 4, 5, 6


def structured_quad(xs, ys):
    """Tensor-product quad mesh over the coordinate lines xs (nx+1) and ys (ny+1)."""
    xs = np.asarray(xs, float)
    ys = np.asarray(ys, float)
    nx, ny = len(xs) - 1, len(ys) - 1
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xyz = np.stack([X.ravel(), Y.ravel()], axis=1)

    def nid(i, j):
        return j * (nx + 1) + i

    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    I, J = I.ravel(), J.ravel()
    cells = np.stack([nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)], axis=1)
    bf, tags = [], []
    j = np.arange(ny)
    bf.append(np.stack([nid(0, j), nid(0, j + 1)], 1)); tags.append(np.full(ny, TAG_X0))
    bf.append(np.stack([nid(nx, j), nid(nx, j + 1)], 1)); tags.append(np.full(ny, TAG_X1))
    i = np.arange(nx)
    bf.append(np.stack([nid(i, 0), nid(i + 1, 0)], 1)); tags.append(np.full(nx, TAG_Y0))
    bf.append(np.stack([nid(i, ny), nid(i + 1, ny)], 1)); tags.append(np.full(nx, TAG_Y1))
    return (xyz, cells.astype(np.int64), np.concatenate(bf).astype(np.int64),
            np.concatenate(tags).astype(np.int32))


def _hex_grid_nodes(xs, ys, zs):
    nx, ny = len(xs) - 1, len(ys) - 1
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def nid(i, j, k):
        return (k * (ny + 1) + j) * (nx + 1) + i

    return xyz, nid


def _boundary_faces_by_count(face_nodes):
    """Faces (rows of node ids) that occur exactly once: the domain boundary."""
    key = np.sort(face_nodes, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    return face_nodes[cnt[inv] == 1]


def structured_hex(xs, ys, zs, keep=None):
    """Tensor-product hex mesh.  keep(cx, cy, cz) -> bool mask selects the hexes
    (by centre) that belong to the domain; None keeps all.  Boundary faces are
    the hex faces used once; the caller tags them."""
    xs, ys, zs = (np.asarray(a, float) for a in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    xyz, nid = _hex_grid_nodes(xs, ys, zs)
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    if keep is not None:
        cx = 0.5 * (xs[I] + xs[I + 1]); cy = 0.5 * (ys[J] + ys[J + 1]); cz = 0.5 * (zs[K] + zs[K + 1])
        m = keep(cx, cy, cz)
        I, J, K = I[m], J[m], K[m]
    cells = np.stack([nid(I, J, K), nid(I + 1, J, K), nid(I + 1, J + 1, K), nid(I, J + 1, K),
                      nid(I, J, K + 1), nid(I + 1, J, K + 1), nid(I + 1, J + 1, K + 1), nid(I, J + 1, K + 1)],
                     axis=1).astype(np.int64)
    return _compact(xyz, cells)


def _compact(xyz, cells):
    used = np.unique(cells)
    remap = -np.ones(len(xyz), np.int64)
    remap[used] = np.arange(len(used))
    return xyz[used], remap[cells]


HEX_FACES = np.array([[0, 3, 2, 1], [4, 5, 6, 7], [0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]])
TET_FACES = np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]])


def hex_boundary(cells):
    faces = cells[:, HEX_FACES].reshape(-1, 4)
    return _boundary_faces_by_count(faces)


def hex_to_tets(cells):
    """Split every hex into 6 tets that share its 0->6 diagonal (corner (0,0,0) to
    corner (1,1,1) of the local frame).  The same diagonal direction in every hex
    makes the split conforming across shared faces."""
    # local corner index of offset (a,b,c)
    off = {(0, 0, 0): 0, (1, 0, 0): 1, (1, 1, 0): 2, (0, 1, 0): 3,
           (0, 0, 1): 4, (1, 0, 1): 5, (1, 1, 1): 6, (0, 1, 1): 7}
    tets = []
    axes = np.eye(3, dtype=int)
    for perm in ([0, 1, 2], [0, 2, 1], [1, 0, 2], [1, 2, 0], [2, 0, 1], [2, 1, 0]):
        p0 = np.zeros(3, int)
        p1 = p0 + axes[perm[0]]
        p2 = p1 + axes[perm[1]]
        p3 = p2 + axes[perm[2]]
        tets.append([off[tuple(p)] for p in (p0, p1, p2, p3)])
    tets = np.array(tets)
    return cells[:, tets].reshape(-1, 4)


def tet_boundary(cells):
    faces = cells[:, TET_FACES].reshape(-1, 3)
    return _boundary_faces_by_count(faces)


def tag_by_plane(xyz, bfaces, rules, default):
    """Tag boundary faces by their centroid: rules is a list of
    (predicate(centroid_array)->mask, tag); the first match wins."""
    cen = xyz[bfaces].mean(axis=1)
    tags = np.full(len(bfaces), default, np.int32)
    done = np.zeros(len(bfaces), bool)
    for pred, tag in rules:
        m = pred(cen) & ~done
        tags[m] = tag
        done |= m
    return tags


def box_tags(xyz, bfaces, lo, hi, tol):
    cen = xyz[bfaces].mean(axis=1)
    tags = np.zeros(len(bfaces), np.int32)
    for ax, (t0, t1) in enumerate([(TAG_X0, TAG_X1), (TAG_Y0, TAG_Y1), (TAG_Z0, TAG_Z1)][: xyz.shape[1]]):
        tags[np.abs(cen[:, ax] - lo[ax]) < tol] = t0
        tags[np.abs(cen[:, ax] - hi[ax]) < tol] = t1
    return tags


def graded(a, b, n, ratio=1.0, fine_at="b"):
    """n intervals over [a,b] with geometric grading; ratio = last/first size."""
    if n <= 0:
        return np.array([a, b])[:1]
    if abs(ratio - 1.0) < 1e-12 or n == 1:
        return np.linspace(a, b, n + 1)
    q = ratio ** (1.0 / (n - 1))
    h = q ** np.arange(n)
    h = h / h.sum() * (b - a)
    if fine_at == "b":
        h = h[::-1]
    return a + np.concatenate([[0.0], np.cumsum(h)])


# --------------------------------------------------------------------------
# porous 2D film (Delaunay)
# --------------------------------------------------------------------------

def _segment_points(p0, p1, h):
    n = max(1, int(np.ceil(np.linalg.norm(np.subtract(p1, p0)) / h)))
    t = np.arange(n) / n
    return np.asarray(p0)[None, :] + t[:, None] * (np.asarray(p1) - np.asarray(p0))[None, :]


def porous_film(rng, Lx, Ly, pores, n_target):
    """Triangulate the rectangle [0,Lx]x[0,Ly] minus circular pores
    (list of (cx, cy, r)).  Returns (xyz, tri, bfaces, tags) with tags
    x0=1, x1=2, y-walls=3, pore walls=4; raises RuntimeError if the boundary
    recovery check fails (caller retries with another seed)."""
    area = Lx * Ly - sum(np.pi * r * r for (_, _, r) in pores)
    h = np.sqrt(2.0 * area / n_target)
    # rectangle boundary points (corners included once)
    corners = [(0, 0), (Lx, 0), (Lx, Ly), (0, Ly)]
    bpts = np.concatenate([_segment_points(corners[k], corners[(k + 1) % 4], h) for k in range(4)])
    pore_pts = []
    for (cx, cy, r) in pores:
        n = max(12, int(np.ceil(2 * np.pi * r / h)))
        ang = 2 * np.pi * np.arange(n) / n
        pore_pts.append(np.stack([cx + r * np.cos(ang), cy + r * np.sin(ang)], 1))
    # jittered interior grid
    nx = max(2, int(round(Lx / h)))
    ny = max(2, int(round(Ly / h)))
    gx = (np.arange(nx) + 0.5) * Lx / nx
    gy = (np.arange(ny) + 0.5) * Ly / ny
    GX, GY = np.meshgrid(gx, gy)
    P = np.stack([GX.ravel(), GY.ravel()], 1)
    P = P + rng.uniform(-0.2, 0.2, P.shape) * np.array([Lx / nx, Ly / ny])
    keep = (P[:, 0] > 0.45 * h) & (P[:, 0] < Lx - 0.45 * h) & (P[:, 1] > 0.45 * h) & (P[:, 1] < Ly - 0.45 * h)
    for (cx, cy, r) in pores:
        keep &= np.hypot(P[:, 0] - cx, P[:, 1] - cy) > r + 0.55 * h
    P = P[keep]
    pts = np.concatenate([bpts] + pore_pts + [P])
    tri = Delaunay(pts).simplices.astype(np.int64)
    cen = pts[tri].mean(axis=1)
    inside = np.zeros(len(tri), bool)
    for (cx, cy, r) in pores:
        inside |= np.hypot(cen[:, 0] - cx, cen[:, 1] - cy) < r
    tri = tri[~inside]
    # counter-clockwise orientation
    a, b, c = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    cross = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    if np.any(np.abs(cross) < 1e-12 * h * h):
        raise RuntimeError("degenerate triangle")
    flip = cross < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    edges = tri[:, [[0, 1], [1, 2], [2, 0]]].reshape(-1, 2)
    bfaces = _boundary_faces_by_count(edges)
    ecen = pts[bfaces].mean(axis=1)
    tags = np.zeros(len(bfaces), np.int32)
    tol = 1e-9 * max(Lx, Ly)
    tags[np.abs(ecen[:, 0]) < tol] = 1
    tags[np.abs(ecen[:, 0] - Lx) < tol] = 2
    tags[(np.abs(ecen[:, 1]) < tol) | (np.abs(ecen[:, 1] - Ly) < tol)] = 3
    for (cx, cy, r) in pores:
        d0 = np.hypot(pts[bfaces[:, 0], 0] - cx, pts[bfaces[:, 0], 1] - cy)
        d1 = np.hypot(pts[bfaces[:, 1], 0] - cx, pts[bfaces[:, 1], 1] - cy)
        on = (np.abs(d0 - r) < 1e-9 * r) & (np.abs(d1 - r) < 1e-9 * r)
        tags[on & (tags == 0)] = 4
    if np.any(tags == 0):
        raise RuntimeError("boundary recovery failed")
    used = np.unique(tri)
    remap = -np.ones(len(pts), np.int64)
    remap[used] = np.arange(len(used))
    return pts[used], remap[tri], remap[bfaces], tags
