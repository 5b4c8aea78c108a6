"""Pins of the oracle's finite-volume geometry against exact mesh facts."""
import numpy as np
import pytest

from oracle import geometry as G
from workloads import configs as C
from workloads import meshes as M

NM = 1e-9


def _meshes():
    p1 = C.config1(n=5)
    p2 = C.config2(n=3, B=1, n_polar=2, n_azim=4)
    p3 = C.config3_small()
    p4 = C.config4_small()[2]
    return [("quad", p1), ("hex", p2), ("tet", p3), ("tri", p4)]


@pytest.mark.parametrize("name,p", _meshes())
def test_closed_cells_and_divergence_theorem(name, p):
    g = G.build(p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    # sum_f S_cf = 0 for every closed cell
    scale = np.linalg.norm(g.S, axis=2).sum(axis=1)
    assert np.max(np.linalg.norm(g.S.sum(axis=1), axis=1) / scale) < 1e-14
    # sum_f x_f (x) S_f = V I (restricted to the mesh dimension): pins the
    # orientation and the magnitude of every area vector
    d = g.dim
    T = np.einsum("cfi,cfj->cij", g.xf, g.S)[:, :d, :d]
    assert np.allclose(T, g.V[:, None, None] * np.eye(d)[None], rtol=0, atol=1e-12 * g.V.max())
    # every interior face is seen from both sides with opposite area vectors
    c, f = np.nonzero(g.nbr >= 0)
    n = g.nbr[c, f]
    back = (g.nbr[n] == c[:, None])
    assert np.all(back.sum(axis=1) == 1)
    fb = np.argmax(back, axis=1)
    assert np.array_equal(g.S[n, fb], -g.S[c, f])


def test_volumes_and_surface_areas():
    # unit-cube-like box split into hexes: total volume and surface
    L = 1000 * NM
    p = C.config2(n=3, B=1, n_polar=2, n_azim=4)
    g = G.build(p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    assert g.V.sum() == pytest.approx(L ** 3, rel=1e-14)
    Sb = np.linalg.norm(g.S[g.bf_owner, g.bf_local], axis=1)
    assert Sb.sum() == pytest.approx(6 * L ** 2, rel=1e-14)
    # every tet of a Kuhn-split box has one sixth of its hex's volume
    xs = np.linspace(0, 1.0, 3)
    xyz, hexes = M.structured_hex(xs, xs, xs)
    tets = M.hex_to_tets(hexes)
    bf = M.tet_boundary(tets)
    gt = G.build(xyz, "tet4", tets, bf, np.ones(len(bf), np.int32))
    assert np.allclose(gt.V, (0.5 ** 3) / 6, rtol=1e-14)
    # FinFET: substrate + fin
    p3 = C.config3_small()
    g3 = G.build(p3.xyz, p3.cell_type, p3.cells, p3.bfaces, p3.bface_tag)
    assert g3.V.sum() == pytest.approx((200 * 200 * 100 + 10 * 100 * 40) * NM ** 3, rel=1e-12)
    # 2D square: areas and perimeter per unit depth
    p1 = C.config1(n=7)
    g1 = G.build(p1.xyz, p1.cell_type, p1.cells, p1.bfaces, p1.bface_tag)
    assert g1.V.sum() == pytest.approx((100 * NM) ** 2, rel=1e-14)
    assert np.linalg.norm(g1.S[g1.bf_owner, g1.bf_local], axis=1).sum() == pytest.approx(400 * NM, rel=1e-14)


def test_porous_area_matches_polygonal_pores():
    p = C.config4_small()[2]
    g = G.build(p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    # the pores are regular polygons inscribed in their circles: each removes
    # (n/2) r^2 sin(2 pi / n) of area; recover n and r from the pore-wall faces
    Lx, Ly = p.meta["Lx"], p.meta["Ly"]
    pore_faces = g.bf_tag == 4
    assert pore_faces.any()
    removed = Lx * Ly - g.V.sum()
    # area enclosed by the pore walls (shoelace over the boundary edges, which
    # with the outward normals of the film is the negative pore area)
    xf = g.xf[g.bf_owner, g.bf_local]
    S = g.S[g.bf_owner, g.bf_local]
    enclosed = -0.5 * np.sum(np.einsum("ij,ij->i", xf[pore_faces], S[pore_faces]))
    assert removed == pytest.approx(enclosed, rel=1e-10)


def test_rejects_bad_meshes():
    xyz, cells, bf, tags = M.structured_quad(np.linspace(0, 1, 3), np.linspace(0, 1, 3))
    with pytest.raises(ValueError):
        G.build(xyz, "quad4", cells, bf[:-1], tags[:-1])        # untagged boundary face
    bad = cells.copy()
    bad[0] = bad[0][[0, 2, 1, 3]]                              # self-intersecting quad
    with pytest.raises(ValueError):
        g = G.build(xyz, "quad4", bad, bf, tags)
        if np.max(np.linalg.norm(g.S.sum(axis=1), axis=1)) > 1e-12:
            raise ValueError("not closed")
