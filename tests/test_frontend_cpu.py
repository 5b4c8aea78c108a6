"""Front end without a GPU: Gmsh files read by the library against the same
meshes given as arrays, band tables, spectral binning, and the oracle's
equivalence of a 3D quadrature over a 2D domain with a one-layer 3D slab
between specular walls (the z-invariant material the 2D reading stands for)."""
import numpy as np
import pytest

import oracle
from paper_2607_03226_amd import frontend as FE
from paper_2607_03226_amd import nbte as N
from workloads import Boundary, Problem
from workloads import configs as C
from workloads import meshes as M
from workloads.tables import gl_azimuth_quadrature

MAKERS = [("quad", C.config1), ("tet", C.config3_small), ("tri", lambda: C.config4_small()[2]),
          ("hex", C.config2_small)]


def _regions(p):
    xc = np.asarray(p.xyz, float)[np.asarray(p.cells)].mean(axis=1)
    return np.where(xc[:, 0] > np.median(xc[:, 0]), 7, 3).astype(np.int32)


@pytest.mark.parametrize("version", ["4.1", "2.2"])
@pytest.mark.parametrize("name,maker", MAKERS)
def test_gmsh_file_gives_the_same_mesh(tmp_path, name, maker, version):
    p = maker()
    reg = _regions(p)
    path = tmp_path / f"{name}.msh"
    FE.write_gmsh(path, p.dim, p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag, reg, version=version)
    a = N.nbte_mesh_create(p.dim, p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    b = N.nbte_mesh_read_gmsh(path)
    ia, ib = N.nbte_mesh_get_info(a), N.nbte_mesh_get_info(b)
    for k in ("dim", "faces_per_cell", "n_cells", "n_bfaces"):
        assert ia[k] == ib[k], k
    assert ib["total_volume"] == pytest.approx(ia["total_volume"], rel=1e-13)
    assert np.array_equal(N.nbte_mesh_get_regions(b), reg)
    assert np.array_equal(N.nbte_mesh_get_regions(a), np.zeros(p.n_cells, np.int32))
    from oracle import geometry as geo
    g = geo.build(p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    assert np.max(np.abs(N.nbte_mesh_get_centroids(b) - g.xc)) <= 1e-15 * np.max(np.abs(g.xc))


def test_gmsh_scale_interior_elements_and_errors(tmp_path):
    p = C.config1()
    path = tmp_path / "m.msh"
    FE.write_gmsh(path, p.dim, np.asarray(p.xyz) / 1e-9, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    b = N.nbte_mesh_read_gmsh(path, scale=1e-9)
    a = N.nbte_mesh_create(p.dim, p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    assert N.nbte_mesh_get_info(b)["total_volume"] == pytest.approx(N.nbte_mesh_get_info(a)["total_volume"],
                                                                    rel=1e-12)
    # an interior edge with a physical group (a material interface) is not a boundary face
    cells = np.asarray(p.cells)
    inner = np.array([[cells[17][1], cells[17][2]]])
    path2 = tmp_path / "iface.msh"
    FE.write_gmsh(path2, p.dim, p.xyz, p.cell_type, p.cells, np.vstack([p.bfaces, inner]),
                  np.r_[p.bface_tag, 9], version="2.2")
    assert N.nbte_mesh_get_info(N.nbte_mesh_read_gmsh(path2))["n_bfaces"] == len(p.bfaces)
    # a missing boundary face is a mesh error; unreadable or binary files are argument errors
    path3 = tmp_path / "open.msh"
    FE.write_gmsh(path3, p.dim, p.xyz, p.cell_type, p.cells, np.asarray(p.bfaces)[1:], p.bface_tag[1:])
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_read_gmsh(path3)
    assert e.value.status == N.ERR_MESH
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_read_gmsh(tmp_path / "nope.msh")
    assert e.value.status == N.ERR_INVALID_ARG
    (tmp_path / "bin.msh").write_text("$MeshFormat\n4.1 1 8\n$EndMeshFormat\n")
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_read_gmsh(tmp_path / "bin.msh")
    assert e.value.status == N.ERR_INVALID_ARG
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_read_gmsh(path, scale=0.0)
    assert e.value.status == N.ERR_INVALID_ARG


def test_band_table_round_trip_and_errors(tmp_path):
    rng = np.random.default_rng(3)
    Cb, vb, tb = rng.uniform(1e5, 1e6, 7), rng.uniform(1e3, 9e3, 7), np.exp(rng.uniform(-28, -20, 7))
    path = tmp_path / "bands.txt"
    FE.save_band_table(path, Cb, vb, tb, comment="seeded test table")
    C2, v2, t2 = FE.load_band_table(path)
    assert np.array_equal(C2, Cb) and np.array_equal(v2, vb) and np.array_equal(t2, tb)
    (tmp_path / "bad.txt").write_text("1.0 2.0\n")
    with pytest.raises(ValueError):
        FE.load_band_table(tmp_path / "bad.txt")
    (tmp_path / "neg.txt").write_text("1.0 -2.0 1e-12\n")
    with pytest.raises(ValueError):
        FE.load_band_table(tmp_path / "neg.txt")


def test_spectral_binning_keeps_capacity_flux_and_conductivity():
    rng = np.random.default_rng(4)
    f = rng.uniform(0.1, 15.0, 500)
    Cm, vm, tm = rng.uniform(1e3, 1e4, 500), rng.uniform(500, 9000, 500), np.exp(rng.uniform(-28, -20, 500))
    Cb, vb, tb, edges = FE.bin_modes(f, Cm, vm, tm, 12)
    assert len(Cb) == 12
    idx = np.clip(np.searchsorted(edges, f, side="right") - 1, 0, 11)
    for b in range(12):
        m = idx == b
        assert Cb[b] == pytest.approx(Cm[m].sum(), rel=1e-13)
        assert Cb[b] * vb[b] == pytest.approx((Cm[m] * vm[m]).sum(), rel=1e-13)
        assert Cb[b] * vb[b] ** 2 * tb[b] == pytest.approx((Cm[m] * vm[m] ** 2 * tm[m]).sum(), rel=1e-12)
    # one mode per band is the identity
    C1, v1, t1, _ = FE.bin_modes(np.arange(5.0), Cm[:5], vm[:5], tm[:5], 5)
    assert np.allclose(C1, Cm[:5], rtol=1e-15) and np.allclose(v1, vm[:5], rtol=1e-15)
    assert np.allclose(t1, tm[:5], rtol=1e-13)


NM = 1e-9


def _bands():
    return np.array([1.2e6, 0.6e6]), np.array([6000.0, 3000.0]), np.array([8e-12, 40e-12])


def test_3d_quadrature_on_2d_domain_equals_one_layer_slab_between_specular_walls():
    """A 2D domain with directions over the sphere stands for a material that
    does not vary along z: the oracle's 2D solve equals its 3D solve of one
    layer of hexahedra (same x-y grid) between specular z walls, cell by cell."""
    xs = np.linspace(0, 80 * NM, 7)
    ys = np.linspace(0, 50 * NM, 5)
    s, w = gl_azimuth_quadrature(4, 8)
    C_, v, tau = _bands()
    xyz2, cells2, bf2, tags2 = M.structured_quad(xs, ys)
    bcs = [Boundary(1, "thermalizing", 301.0), Boundary(2, "thermalizing", 299.0), Boundary(3, "diffuse"),
           Boundary(4, "partial", specularity=0.6), Boundary(5, "specular"), Boundary(6, "specular")]
    rng = np.random.default_rng(8)
    Q2 = rng.uniform(0, 3e17, len(cells2))
    p2 = Problem("z2d", 2, xyz2, "quad4", cells2, bf2, tags2, bcs[:4], C_, v, tau, s, w, Q2)
    xyz3, cells3 = M.structured_hex(xs, ys, np.array([0.0, 20 * NM]))
    bf3 = M.hex_boundary(cells3)
    tags3 = M.box_tags(xyz3, bf3, (0, 0, 0), (80 * NM, 50 * NM, 20 * NM), 1e-6 * NM)
    # structured_quad tags: 1 x=0, 2 x=L, 3 y=0, 4 y=H; box_tags: 1 x=0, 2 x=L, 3 y=0, 4 y=H, 5 z=0, 6 z=top
    xc3 = xyz3[cells3].mean(axis=1)
    xc2 = np.asarray(xyz2)[cells2].mean(axis=1)
    order = [int(np.argmin(np.linalg.norm(xc2 - x[:2], axis=1))) for x in xc3]
    p3 = Problem("z3d", 3, xyz3, "hex8", cells3, bf3, tags3, bcs, C_, v, tau, s, w, Q2[order])
    r2 = oracle.solve(p2, tol=1e-14, max_iter=20000)
    r3 = oracle.solve(p3, tol=1e-14, max_iter=20000)
    scale = np.max(np.abs(r2.T_lattice - 300.0))
    assert np.max(np.abs(r3.T_lattice - r2.T_lattice[order])) / scale < 1e-10
    assert np.max(np.abs(r3.q[:, :2] - r2.q[order, :2])) / np.max(np.abs(r2.q)) < 1e-10
    assert np.max(np.abs(r2.q[:, 2])) < 1e-12 * np.max(np.abs(r2.q))
