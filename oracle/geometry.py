"""ORACLE (test infrastructure only): finite-volume geometry from a raw mesh.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product path never does.

The paper caches cell-face connectivity and direction-resolved advection
coefficients once per mesh (Methods, paragraph after Eq. (13)).  Here that is
written out plainly with numpy:

  * faces are matched between cells by their sorted node sets;
  * every face gets ONE area vector S (area times unit normal), computed once
    from its first occurrence, and the two cells that share it see +S and -S,
    so the upwind decision sign(s . S) is the same from both sides;
  * 2D meshes are taken per unit depth: a face is an edge (area = length),
    a cell volume is its area;
  * cell volumes come from the divergence theorem V = (1/d) sum_f x_f . S_f,
    which is exact for the straight-edged / planar-faced cells used here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LOCAL_FACES = {
    "tri3": [(0, 1), (1, 2), (2, 0)],
    "quad4": [(0, 1), (1, 2), (2, 3), (3, 0)],
    "tet4": [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)],
    "hex8": [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)],
}


@dataclass
class Geometry:
    dim: int
    N: int
    F: int
    nbr: np.ndarray      # (N,F) int64: neighbour cell, or -(1 + boundary face index)
    S: np.ndarray        # (N,F,3) outward area vectors
    xf: np.ndarray       # (N,F,3) face centroids
    V: np.ndarray        # (N,) volumes
    xc: np.ndarray       # (N,3) cell centroids (vertex average)
    bf_owner: np.ndarray  # (NBF,) owner cell of each boundary face
    bf_local: np.ndarray  # (NBF,) local face index in the owner
    bf_tag: np.ndarray    # (NBF,) tag


def _area_vector(P):
    """P: (M, k, 3) face vertices in cyclic order."""
    k = P.shape[1]
    if k == 2:   # 2D edge: length times in-plane normal (sign fixed by caller)
        d = P[:, 1] - P[:, 0]
        return np.stack([d[:, 1], -d[:, 0], np.zeros(len(P))], axis=1)
    if k == 3:
        return 0.5 * np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    if k == 4:
        return 0.5 * np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 1])
    raise ValueError(k)


def build(xyz, cell_type, cells, bfaces, bface_tag) -> Geometry:
    xyz = np.asarray(xyz, float)
    dim = xyz.shape[1]
    X = np.zeros((len(xyz), 3))
    X[:, :dim] = xyz
    cells = np.asarray(cells, np.int64)
    N = len(cells)
    lf = np.array(LOCAL_FACES[cell_type])
    F = lf.shape[0]
    fn = cells[:, lf]                       # (N, F, k) node ids of each local face
    k = fn.shape[2]
    flat = fn.reshape(-1, k)
    keys = np.sort(flat, axis=1)
    uniq, first, inv, cnt = np.unique(keys, axis=0, return_index=True, return_inverse=True,
                                      return_counts=True)
    inv = inv.ravel()
    if np.any(cnt > 2):
        raise ValueError("non-manifold face shared by more than two cells")

    xc = X[cells].mean(axis=1)
    # one area vector per unique face, from its first occurrence
    Su = _area_vector(X[flat[first]])
    xfu = X[flat[first]].mean(axis=1)
    owner_first = first // F
    # orient each unique face outward from the cell of its first occurrence
    sgn = np.sign(np.einsum("ij,ij->i", xfu - xc[owner_first], Su))
    if np.any(sgn == 0):
        raise ValueError("degenerate face orientation")
    Su = Su * sgn[:, None]
    S = Su[inv].reshape(N, F, 3).copy()
    xf = xfu[inv].reshape(N, F, 3)
    # occurrences other than the first see the face from the other side
    occ = np.arange(N * F)
    other = occ != first[inv]
    S.reshape(-1, 3)[other] *= -1.0

    # neighbours: pair the two occurrences of each interior face
    nbr = np.full(N * F, -1, np.int64)
    interior = cnt[inv] == 2
    order = np.argsort(inv, kind="stable")
    inv_sorted = inv[order]
    # for faces with two occurrences, consecutive entries in 'order' pair up
    pos = np.flatnonzero(np.r_[inv_sorted[1:] == inv_sorted[:-1], False])
    o1, o2 = order[pos], order[pos + 1]
    nbr[o1] = o2 // F
    nbr[o2] = o1 // F

    # boundary faces must match the tagged list
    bkeys = np.sort(np.asarray(bfaces, np.int64), axis=1)
    bidx = {tuple(r): j for j, r in enumerate(bkeys)}
    bnd_occ = np.flatnonzero(~interior)
    bf_owner = np.zeros(len(bkeys), np.int64)
    bf_local = np.zeros(len(bkeys), np.int64)
    seen = np.zeros(len(bkeys), bool)
    for o in bnd_occ:
        j = bidx.get(tuple(keys[o]))
        if j is None:
            raise ValueError("untagged boundary face")
        nbr[o] = -(1 + j)
        bf_owner[j] = o // F
        bf_local[j] = o % F
        seen[j] = True
    if not np.all(seen):
        raise ValueError("tagged boundary face not on the mesh boundary")
    nbr = nbr.reshape(N, F)

    V = np.einsum("cfk,cfk->c", xf, S) / dim
    if np.any(V <= 0):
        raise ValueError("non-positive cell volume")
    return Geometry(dim=dim, N=N, F=F, nbr=nbr, S=S, xf=xf, V=V, xc=xc,
                    bf_owner=bf_owner, bf_local=bf_local, bf_tag=np.asarray(bface_tag, np.int32))
