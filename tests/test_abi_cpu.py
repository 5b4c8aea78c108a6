"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every declared symbol, the mesh builder reproduces exact geometry,
argument validation returns the documented status codes, and the sweep
schedules respect upwind order."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2607_03226_amd import nbte as N
from workloads import Boundary
from workloads import configs as C
from workloads import meshes as M
from workloads.tables import gl_azimuth_quadrature, inplane_quadrature

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "nbte.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbte_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(N.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    bound = {s[0] for s in N.SIGNATURES}
    assert set(names) <= bound, set(names) - bound
    assert "gfx950" in N.nbte_version()


def _handles(p):
    mesh = N.nbte_mesh_create(p.dim, p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    h = N.nbte_problem_create(mesh)
    return mesh, h


@pytest.mark.parametrize("maker", [C.config1, C.config2_small, C.config3_small, lambda: C.config4_small()[2]])
def test_mesh_info_matches_exact_geometry(maker):
    p = maker()
    mesh = N.nbte_mesh_create(p.dim, p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    info = N.nbte_mesh_get_info(mesh)
    assert info["n_cells"] == p.n_cells and info["n_bfaces"] == len(p.bfaces)
    assert info["max_closure_error"] < 1e-14
    from oracle import geometry
    g = geometry.build(p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    assert info["total_volume"] == pytest.approx(g.V.sum(), rel=1e-13)


def test_mesh_validation_errors():
    xyz, cells, bf, tags = M.structured_quad(np.linspace(0, 1, 4), np.linspace(0, 1, 4))
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_create(2, xyz, "quad4", cells, bf[:-1], tags[:-1])
    assert e.value.status == N.ERR_MESH
    bad = cells.copy()
    bad[0, 0] = 10 ** 6
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_create(2, xyz, "quad4", bad, bf, tags)
    assert e.value.status == N.ERR_MESH
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_create(3, np.c_[xyz, np.zeros(len(xyz))], "quad4", cells, bf, tags)
    assert e.value.status == N.ERR_INVALID_ARG
    nan = xyz.copy(); nan[3, 0] = np.nan
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_create(2, nan, "quad4", cells, bf, tags)
    assert e.value.status == N.ERR_INVALID_ARG
    # inverted cell: faces no longer close consistently / volume not positive
    inv = cells.copy(); inv[4] = inv[4][[0, 2, 1, 3]]
    with pytest.raises(N.NbteError) as e:
        N.nbte_mesh_create(2, xyz, "quad4", inv, bf, tags)
    assert e.value.status == N.ERR_MESH


def test_table_validation_and_state_errors():
    p = C.config1()
    mesh, h = _handles(p)
    with pytest.raises(N.NbteError) as e:
        N.nbte_prepare(h, None, N.make_opts())
    assert e.value.status == N.ERR_STATE
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_bands(h, [1.0], [-1.0], [1e-12])
    assert e.value.status == N.ERR_INVALID_ARG
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_bands(h, [1.0], [1.0], [np.nan])
    assert e.value.status == N.ERR_INVALID_ARG
    s, w = inplane_quadrature(8)
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_quadrature(h, s * 1.01, w)
    assert e.value.status == N.ERR_QUADRATURE
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_quadrature(h, s, -w)
    assert e.value.status == N.ERR_QUADRATURE
    s3, w3 = gl_azimuth_quadrature(2, 4)
    N.nbte_set_quadrature(h, s3, w3)              # 3D directions on a 2D mesh: a z-invariant 3D material
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_boundaries(h, [(1, "partial", 0.0, 1.5)])
    assert e.value.status == N.ERR_BOUNDARY
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_boundaries(h, [(1, "thermalizing", 300.0, 0), (1, "specular", 0, 0)])
    assert e.value.status == N.ERR_BOUNDARY


def _prepare_status(p):
    mesh, h = _handles(p)
    N.nbte_set_bands(h, p.C, p.v, p.tau)
    N.nbte_set_quadrature(h, p.s, p.w)
    N.nbte_set_boundaries(h, [(b.tag, b.kind, b.T_wall, b.specularity) for b in p.boundaries])
    try:
        N.nbte_prepare(h, p.Q, N.make_opts())
    except N.NbteError as e:
        return e.status
    return N.OK


def test_host_setup_errors_come_before_device_errors():
    p = C.config1()
    # no thermalizing wall -> ill-posed
    p.boundaries = [Boundary(t, "specular") for t in (1, 2, 3, 4)]
    assert _prepare_status(p) == N.ERR_ILL_POSED
    # a tag without a condition
    p = C.config1(); p.boundaries = p.boundaries[:3]
    assert _prepare_status(p) == N.ERR_BOUNDARY
    # specular x-wall whose mirror directions are not in the set: with 7
    # half-offset in-plane directions pi - phi_j is never a member
    p = C.config1(D=7)
    p.boundaries = [Boundary(1, "specular"), Boundary(2, "specular"),
                    Boundary(3, "thermalizing", 301.0), Boundary(4, "thermalizing", 299.0)]
    assert _prepare_status(p) == N.ERR_QUADRATURE
    # a valid problem gets through host setup and then needs the GPU
    p = C.config1()
    st = _prepare_status(p)
    assert st in (N.OK, N.ERR_DEVICE)


@pytest.mark.parametrize("maker", [C.config1, C.config2_small, C.config3_small, lambda: C.config4_small()[1]])
def test_schedule_levels_respect_upwind_order(maker):
    p = maker()
    mesh, h = _handles(p)
    N.nbte_set_quadrature(h, p.s, p.w)
    from oracle import geometry
    g = geometry.build(p.xyz, p.cell_type, p.cells, p.bfaces, p.bface_tag)
    for i in range(0, p.n_dirs, max(1, p.n_dirs // 7)):
        perm, lvl = N.nbte_get_schedule(h, i)
        assert np.array_equal(np.sort(perm), np.arange(p.n_cells))
        level = np.empty(p.n_cells, int)
        for l in range(len(lvl) - 1):
            level[perm[lvl[l]:lvl[l + 1]]] = l
        a = np.einsum("cfk,k->cf", g.S, p.s[i])
        c, f = np.nonzero((a < 0) & (g.nbr >= 0))
        assert np.all(level[g.nbr[c, f]] < level[c])
        # levels are as shallow as possible: each cell past level 0 has an upwind neighbour one level up
        deep = level > 0
        has_prev = np.zeros(p.n_cells, bool)
        has_prev[c[level[g.nbr[c, f]] == level[c] - 1]] = True
        assert np.all(has_prev[deep])


def test_footprint_scales_with_precision():
    p = C.config2_small()
    mesh, h = _handles(p)
    N.nbte_set_bands(h, p.C, p.v, p.tau)
    N.nbte_set_quadrature(h, p.s, p.w)
    f32 = N.nbte_problem_footprint(h, "mixed")
    f64 = N.nbte_problem_footprint(h, "fp64")
    # the mixed path holds the distribution, the boundary inflow, the
    # boundary owners' copy of the distribution and the sweep's real-valued
    # streams (coefficients, outflow sum, source, D) in FP32: 4 bytes less
    # per value (inflow rows and boundary owners: at most one per boundary face)
    ndn = p.n_cells * p.n_dirs
    halved = p.n_cells * p.n_bands * p.n_dirs * 4
    assert halved < f64 - f32 <= halved + ndn * (6 + 3) * 4 + 2 * p.n_bands * len(p.bfaces) * p.n_dirs * 4


def test_plane_layout_footprint():
    """The plane layout holds, beyond the cell-major layout's state, the
    reductions' FP64 band sums per (direction, cell) (24 bytes), the boundary
    row index per stream position (4 bytes) and the boundary owners' rows (at
    most one owner per boundary face, D B values each), and the same in both
    precisions but for the rows' storage type; layout 1 forces cell-major."""
    p = C.config2_small()
    mesh, h = _handles(p)
    N.nbte_set_bands(h, p.C, p.v, p.tau)
    N.nbte_set_quadrature(h, p.s, p.w)
    ndn = p.n_cells * p.n_dirs
    rows = len(p.bfaces) * p.n_dirs * p.n_bands
    cell = {}
    for prec, es in (("mixed", 4), ("fp64", 8)):
        N.nbte_set_tuning(h, layout=1)
        cell[prec] = N.nbte_problem_footprint(h, prec)
        N.nbte_set_tuning(h, layout=2)
        planes = N.nbte_problem_footprint(h, prec)
        assert ndn * 28 < planes - cell[prec] <= ndn * 28 + rows * es, (prec, planes - cell[prec])
    N.nbte_set_tuning(h, layout=0)   # auto: a problem this small stays cell-major
    assert N.nbte_problem_footprint(h, "mixed") == cell["mixed"]
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_tuning(h, layout=3)
    assert e.value.status == N.ERR_INVALID_ARG


def test_tuning_validation():
    p = C.config1()
    mesh, h = _handles(p)
    N.nbte_set_tuning(h, lds_bytes=163840, cg_max_iter=12)   # a whole CU's LDS may be asked for
    t = N.nbte_get_tuning(h)
    assert t["lds_bytes"] == 163840 and t["cg_max_iter"] == 12
    for bad in (163841, -2):
        with pytest.raises(N.NbteError) as e:
            N.nbte_set_tuning(h, lds_bytes=bad)
        assert e.value.status == N.ERR_INVALID_ARG
    with pytest.raises(N.NbteError) as e:
        N.nbte_set_tuning(h, cg_max_iter=-1)
    assert e.value.status == N.ERR_INVALID_ARG


def test_tuner_keys_and_candidates():
    from paper_2607_03226_amd import tune
    p2 = C.config2_small()
    k = tune.key(p2, "mixed")
    assert k.startswith(f"{p2.cell_type}|") and k.endswith(f"|B{p2.n_bands}|D{p2.n_dirs}|mixed")
    shapes = tune.candidates(16)
    assert all(s["bands_per_lane"] <= s["bands_per_block"] for s in shapes)
    # one lane per cell (bands per lane = bands per workgroup) is among the candidates up to 8 bands
    assert any(s["bands_per_block"] == s["bands_per_lane"] == 8 for s in shapes)
    # every shape is timed with the default LDS budget and with a whole CU's
    assert {s["lds_bytes"] for s in shapes} == {0, tune.WHOLE_CU_LDS}
    assert len(shapes) == 2 * len({(s["bands_per_block"], s["bands_per_lane"], s["block_size"]) for s in shapes})
    # the committed cache holds a CG cap for the synthetic workloads it covers
    cache = tune.load_cache()
    for entry in cache.values():
        assert entry["shape"].get("cg_max_iter", 8) in (4, 6, 8, 12, 16, 24, 32)


def test_setup_call_validates_before_touching_the_device():
    p = C.config1()
    mesh, h = _handles(p)
    with pytest.raises(N.NbteError) as e:
        N.nbte_problem_setup(h, 7)
    assert e.value.status == N.ERR_INVALID_ARG


def test_counter_traffic_needs_same_source_and_shape(tmp_path, monkeypatch):
    """bench.py reports the committed counter traffic only while the kernel
    source and the sweep's launch shape are the ones it was measured on."""
    import json
    import bench
    (tmp_path / "profiles").mkdir()
    shape = {"bands_per_block": 4, "bands_per_lane": 4, "block_size": 512, "lds_bytes": 0}
    rec = {"kernel_source_sha256_16": "abc", "shape": shape, "traffic_bytes_per_launch": 123.0}
    (tmp_path / "profiles" / "sweep_configX_mixed_counters.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.counter_traffic("configX", "mixed", dict(shape, cg_max_iter=16)) == 123.0
    assert bench.counter_traffic("configX", "mixed", dict(shape, bands_per_lane=2)) is None
    assert bench.counter_traffic("configX", "mixed", None) is None
    assert bench.counter_traffic("configX", "fp64", shape) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "def")
    assert bench.counter_traffic("configX", "mixed", shape) is None


def test_cyclic_upwind_graph_is_ordered_with_lagged_faces():
    """A non-convex (dart) cell closes a cycle in the upwind graph of some
    directions (the mesh is built in the oracle pins, where the oracle's
    direct-solve fallback is checked).  The library's order then lags the
    faces that close the cycles: acyclic directions have none, cyclic ones
    have some, and every other interior upwind neighbour of a cell lies in an
    earlier level."""
    from oracle import geometry as geo
    from tests.test_oracle_pins import dart_mesh
    xyz, cells, bf, tags = dart_mesh()
    mesh = N.nbte_mesh_create(2, xyz, "quad4", cells, bf, tags)
    h = N.nbte_problem_create(mesh)
    s, w = inplane_quadrature(8)
    N.nbte_set_quadrature(h, s, w)
    g = geo.build(xyz, "quad4", cells, bf, tags)
    phi = np.degrees(np.arctan2(s[:, 1], s[:, 0])) % 360
    cyclic = ((phi > 110) & (phi < 190)) | (phi > 290)
    for i in range(len(w)):
        perm, lvl = N.nbte_get_schedule(h, i)
        assert sorted(perm) == [0, 1, 2]
        level = np.empty(3, int)
        for l in range(len(lvl) - 1):
            level[perm[lvl[l]:lvl[l + 1]]] = l
        lc, lf = N.nbte_get_lagged_faces(h, i)
        assert (len(lc) > 0) == bool(cyclic[i]), (i, phi[i], lc)
        lagged = set(zip(lc.tolist(), lf.tolist()))
        for c in range(3):
            for f in range(4):
                n = g.nbr[c, f]
                if n >= 0 and g.S[c, f] @ s[i] < 0 and (c, f) not in lagged:
                    assert level[n] < level[c]
        for c, f in lagged:
            assert g.nbr[c, f] >= 0 and g.S[c, f] @ s[i] < 0


def test_problem_too_large_for_32bit_offsets_is_refused_before_the_device():
    """10,000 quads x 10,000 directions: the FP64 sweep streams (3 + 3 rows
    of 8 bytes per direction and cell) pass 4 GiB, the FP32 ones (4 bytes)
    do not.  The footprint query and the setup call refuse the FP64 solve
    with INVALID_ARG before any device work; the mixed one gets through to
    the device check."""
    xs = np.linspace(0, 1e-6, 101)
    xyz, cells, bf, tags = M.structured_quad(xs, xs)
    mesh = N.nbte_mesh_create(2, xyz, "quad4", cells, bf, tags)
    h = N.nbte_problem_create(mesh)
    N.nbte_set_bands(h, [1e6], [5000.0], [1e-11])
    s, w = inplane_quadrature(10000)
    N.nbte_set_quadrature(h, s, w)
    N.nbte_set_boundaries(h, [(1, "thermalizing", 301.0, 0), (2, "thermalizing", 299.0, 0), (3, "specular", 0, 0),
                              (4, "specular", 0, 0)])
    with pytest.raises(N.NbteError) as e:
        N.nbte_problem_footprint(h, "fp64")
    assert e.value.status == N.ERR_INVALID_ARG and "32-bit" in e.value.message
    with pytest.raises(N.NbteError) as e:
        N.nbte_problem_setup(h, "fp64")
    assert e.value.status == N.ERR_INVALID_ARG
    with pytest.raises(N.NbteError) as e:
        N.nbte_prepare(h, None, N.make_opts(precision="fp64"))
    assert e.value.status == N.ERR_INVALID_ARG
    assert N.nbte_problem_footprint(h, "mixed") > 10000 * 10000 * 4
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(N.NbteError) as e:
            N.nbte_problem_setup(h, "mixed")
        assert e.value.status == N.ERR_DEVICE


def test_counter_summary_scales_by_the_copy_probe(tmp_path):
    """The counter summary scales FETCH_SIZE / WRITE_SIZE (KiB per dispatch)
    by what the same counters read for a device copy of known size."""
    import bench

    def csv(d, rows):
        d.mkdir()
        lines = ["Kernel_Name,Grid_Size,Counter_Name,Counter_Value"]
        lines += [f"{k},{g},{c},{v}" for k, g, c, v in rows]
        (d / "run_counter_collection.csv").write_text("\n".join(lines) + "\n")

    probe = 1 << 30
    csv(tmp_path / "f", [("k_sweep<float>", 100, "FETCH_SIZE", 1000.0)] * 3)
    csv(tmp_path / "w", [("k_sweep<float>", 100, "WRITE_SIZE", 3000.0)] * 3)
    # the copy reads and writes 1 GiB; the counters see 1.25x and 0.5x that
    csv(tmp_path / "cf", [("copyBuffer", 10, "FETCH_SIZE", 1.0), ("copyBuffer", 99, "FETCH_SIZE", 1.25 * probe / 1024)])
    csv(tmp_path / "cw", [("copyBuffer", 99, "WRITE_SIZE", 0.5 * probe / 1024)])
    out = bench.counter_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                                probe)
    assert out["fetch_scale"] == pytest.approx(0.8) and out["write_scale"] == pytest.approx(2.0)
    assert out["traffic_bytes_per_launch"] == pytest.approx(1000 * 1024 * 0.8 + 3000 * 1024 * 2.0)
    assert out["raw_bytes_per_launch"] == pytest.approx(4000 * 1024)
