"""GPU solves of workloads given the way the paper's front end gives them:
a Gmsh file with tagged boundaries and source regions, and a 3D material
over a 2D domain (directions over the sphere)."""
import json

import numpy as np
import pytest

import oracle
from paper_2607_03226_amd import frontend as FE
from workloads import Boundary, Problem
from workloads import configs as C
from workloads import meshes as M
from workloads.tables import gl_azimuth_quadrature

pytestmark = pytest.mark.gpu
NM = 1e-9


def _N():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_03226_amd import nbte
    return nbte


@pytest.mark.parametrize("maker", [C.config3_small, C.config2_small])
def test_gmsh_file_with_source_region_solves_like_the_arrays(tmp_path, maker):
    """The heat source is placed by the cells' physical group read from the
    file; the solve equals (bitwise) the one of the same mesh given as arrays
    with the same per-cell source, and the oracle's solution."""
    N = _N()
    p = maker()
    xc = np.asarray(p.xyz, float)[np.asarray(p.cells)].mean(axis=1)
    region = np.where(np.linalg.norm(xc - xc.mean(axis=0), axis=1) < 0.3 * np.ptp(xc[:, 0]), 2, 1).astype(np.int32)
    path = tmp_path / "w.msh"
    FE.write_gmsh(path, p.dim, p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag, region)
    mesh = N.nbte_mesh_read_gmsh(path)
    Q = np.where(N.nbte_mesh_get_regions(mesh) == 2, 5e17, 0.0)
    _, hf = N.build_problem(p, mesh=mesh)
    _, ha = N.build_problem(p)
    o = N.make_opts(scheme="synthetic", precision="fp64", T_ref=p.T_ref, tol=1e-12, max_iter=5000)
    a = N.nbte_solve_steady(ha, np.where(region == 2, 5e17, 0.0), o)
    b = N.nbte_solve_steady(hf, Q, o)
    for k in ("T_lattice", "T", "q"):
        assert np.array_equal(a[k], b[k]), k
    pq = Problem(p.name, p.dim, p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag, p.boundaries, p.C, p.v, p.tau,
                 p.s, p.w, np.where(region == 2, 5e17, 0.0))
    r = oracle.solve(pq, tol=1e-13, max_iter=20000, defect_tol=1e-11)
    err = float(np.max(np.abs(b["T_lattice"] - r.T_lattice)) / np.max(np.abs(r.T_lattice - p.T_ref)))
    print(p.name, json.dumps({"err_TL": err}), flush=True)
    assert err < 1e-9


def _diamond_film():
    xs = np.linspace(0, 200 * NM, 25)
    ys = np.linspace(0, 60 * NM, 9)
    xyz, cells, bf, tags = M.structured_quad(xs, ys)
    s, w = gl_azimuth_quadrature(4, 8)         # over the sphere: a 3D material in a 2D domain
    rng = np.random.default_rng(31)
    B = 5
    C_ = rng.uniform(0.3e6, 0.8e6, B)
    v = rng.uniform(3000, 12000, B)
    tau = np.exp(rng.uniform(np.log(2e-12), np.log(2e-9), B))
    xc = np.asarray(xyz)[cells].mean(axis=1)
    Q = 2e17 * np.exp(-((xc[:, 0] - 100 * NM) ** 2 + (xc[:, 1] - 60 * NM) ** 2) / (2 * (15 * NM) ** 2))
    return Problem("film3d", 2, xyz, "quad4", cells, bf, tags,
                   [Boundary(1, "thermalizing", 300.0), Boundary(2, "thermalizing", 300.0),
                    Boundary(3, "partial", specularity=0.4), Boundary(4, "diffuse")],
                   C_, v, tau, s, w, Q, scheme="synthetic")


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("mixed", 1e-6)])
def test_3d_material_on_2d_domain_matches_the_oracle(precision, bar):
    N = _N()
    p = _diamond_film()
    r = oracle.solve(p, tol=1e-13, max_iter=20000, defect_tol=1e-11)
    out = N.solve(p, precision=precision, scheme="synthetic", tol=1e-12 if precision == "fp64" else 1e-8,
                  max_iter=20000, allow_not_converged=True)
    err = {"err_TL": float(np.max(np.abs(out["T_lattice"] - r.T_lattice)) / np.max(np.abs(r.T_lattice - p.T_ref))),
           "err_T": float(np.max(np.abs(out["T"] - r.T)) / np.max(np.abs(r.T - p.T_ref))),
           "err_q": float(np.max(np.linalg.norm(out["q"] - r.q, axis=1)) / np.max(np.linalg.norm(r.q, axis=1)))}
    print("film3d", precision, json.dumps(dict(err, iterations=out["iterations"])), flush=True)
    assert max(err.values()) < bar, err
