"""GPU parity of the plane layout of the distribution (tuning layout = 2).

The library stores the distribution either cell-major or, for large
problems, per direction in band-block planes in upwind (level) order; the
reductions then run in two stages and the boundary kernels read a cell-major
copy of the boundary cells' rows.  Every full-size workload above 2^26 values
runs the plane layout through the ordinary parity tests; here the layout is
forced on the small workloads, over every kernel path that touches the
distribution: one sweep against the oracle's exact transport solves, the
launch shapes (ragged band blocks, spilled values, no staging), converged
solves of both schemes and precisions, the FP64 refinement of a stalled
mixed solve (the planes are re-laid for the FP64 launch shape), Anderson
acceleration, second-order face values, BiCGSTAB, cyclic (lagged) faces, the
read-back, and agreement with the cell-major layout.
"""
import numpy as np
import pytest

import oracle
from workloads import configs as C
from test_gpu_parity import SHAPES, _errors, _log, _one_sweep_check, _oracle

pytestmark = pytest.mark.gpu

PLANES = {"layout": 2}


def _N():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_03226_amd import nbte
    return nbte


def _layout(N, out):
    return N.nbte_get_tuning(out["_handles"][1])["layout"]


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-12), ("mixed", None)])
@pytest.mark.parametrize("name,maker", [("config2_small", C.config2_small), ("config3_small", C.config3_small)])
def test_one_sweep_in_planes(name, maker, precision, bar):
    """One sweep from a rough theta in the plane layout, every sampled system
    against the oracle's exact transport solve (mixed: the one-sweep bar of
    the FP32 sweep, 10 sqrt(L) 2^-24)."""
    p = maker()
    rng = np.random.default_rng(11)
    systems = [(int(rng.integers(p.n_bands)), int(rng.integers(p.n_dirs))) for _ in range(10)]
    systems += [(0, 0), (p.n_bands - 1, p.n_dirs - 1)]
    worst, levels = _one_sweep_check(p, precision, systems, None, tuning=PLANES)
    b = bar if bar is not None else 10 * np.sqrt(levels) * 2.0 ** -24
    _log(f"{name}/one_sweep/{precision}/planes", {"err_e": worst, "bar": b})
    assert worst < b


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("bpb,bpl,block,lds", SHAPES)
def test_plane_layout_launch_shapes(bpb, bpl, block, lds, precision):
    """Every launch shape in the plane layout (B = 5 and 6: ragged band
    blocks, hence planes of two widths; spilled values read back from their
    plane rows; no staging) reaches the cell-major solution (FP64, to
    rounding) or the oracle's (mixed bar)."""
    N = _N()
    tuning = {"bands_per_block": bpb, "bands_per_lane": bpl, "block_size": block, "lds_bytes": lds, **PLANES}
    for name, maker in (("config2_small", C.config2_small), ("config3_small", C.config3_small)):
        p = maker()
        if precision == "fp64":
            base = N.solve(p, precision="fp64", scheme="synthetic", tol=1e-12, max_iter=3000, tuning={"layout": 1})
            out = N.solve(p, precision="fp64", scheme="synthetic", tol=1e-12, max_iter=3000, tuning=tuning)
            dev = np.max(np.abs(base["T_lattice"] - p.T_ref))
            assert np.max(np.abs(out["T_lattice"] - base["T_lattice"])) / dev < 1e-11
            qs = np.max(np.linalg.norm(base["q"], axis=1))
            assert np.max(np.linalg.norm(out["q"] - base["q"], axis=1)) / qs < 1e-10
        else:
            ref = _oracle(name, p)
            out = N.solve(p, precision="mixed", scheme="synthetic", tol=1e-8, max_iter=3000, tuning=tuning)
            rec = _errors(out, ref, p.T_ref)
            _log(f"{name}/planes/shape{bpb}-{bpl}-{block}-{lds}/mixed", rec)
            assert max(rec["err_TL"], rec["err_T"], rec["err_q"]) < 1e-6, rec
        assert _layout(N, out) == 2


CASES = [
    ("config1", C.config1, "sequential"),
    ("config4_small_0", lambda: C.config4_small()[0], "synthetic"),
    ("config4_small_3", lambda: C.config4_small()[3], "synthetic"),
    ("porous_10k", lambda: C.porous_problem(4242, n_lo=9000, n_hi=11000), "synthetic"),
    ("serving_5001", lambda: C.serving_request(5001, size_scale=0.03), "synthetic"),
]


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("mixed", 1e-6)])
@pytest.mark.parametrize("name,maker,scheme", CASES)
def test_plane_layout_converged_parity(name, maker, scheme, precision, bar):
    N = _N()
    p = maker()
    ref = _oracle(name, p)
    tol = 1e-12 if precision == "fp64" else 1e-8
    out = N.solve(p, precision=precision, scheme=scheme, tol=tol, max_iter=5000, allow_not_converged=True,
                  tuning=PLANES)
    rec = _errors(out, ref, p.T_ref)
    rec.update(iterations=out["iterations"], energy_defect=out["energy_defect"])
    _log(f"{name}/{precision}/planes", rec)
    assert rec["err_TL"] < bar and rec["err_T"] < bar and rec["err_q"] < bar, rec
    if precision == "fp64":
        assert out["energy_defect"] < 1e-9


def test_planes_and_cell_major_agree_and_read_back():
    """Three iterations of each layout from the same start: the same
    temperatures to rounding, and the distribution read back by cell equal
    to rounding for sampled (band, direction) systems."""
    N = _N()
    p = C.config3_small()
    outs = {}
    for lay in (1, 2):
        mesh, h = N.build_problem(p)
        N.nbte_set_tuning(h, layout=lay)
        N.nbte_prepare(h, p.Q, N.make_opts(scheme=p.scheme, precision="fp64", T_ref=p.T_ref))
        N.nbte_iterate(h, 3, check=True)
        r = N.nbte_read_result(h)
        dist = {(b, i): N.nbte_get_distribution(h, b, i) for b, i in ((0, 0), (1, 7), (p.n_bands - 1, p.n_dirs - 1))}
        outs[lay] = (r, dist, (mesh, h))
    (r1, d1, _), (r2, d2, _) = outs[1], outs[2]
    dev = np.max(np.abs(r1["T_lattice"] - p.T_ref))
    assert np.max(np.abs(r1["T_lattice"] - r2["T_lattice"])) / dev < 1e-12
    for k in d1:
        assert np.max(np.abs(d1[k] - d2[k])) / np.max(np.abs(d1[k])) < 1e-12


def test_stalled_mixed_solve_continues_in_fp64_planes():
    """Refinement in the plane layout: the FP32 planes are widened into the
    planes of the FP64 launch shape (and the boundary rows with them)."""
    N = _N()
    p = C.config1()
    ref = _oracle("config1", p)
    mesh, h = N.build_problem(p)
    N.nbte_set_tuning(h, **PLANES)
    out = N.nbte_solve_steady(h, p.Q, N.make_opts(scheme="sequential", precision="mixed", T_ref=p.T_ref, tol=1e-11,
                                                   max_iter=20000))
    st = N.nbte_get_stats(h)
    rec = _errors(out, ref, p.T_ref)
    rec.update(iterations=out["iterations"], refined_at=st["refined_at"])
    _log("config1/mixed_refined/planes", rec)
    assert st["refined_at"] > 0
    assert max(rec["err_TL"], rec["err_T"], rec["err_q"]) < 1e-9, rec


def test_plane_layout_with_acceleration():
    N = _N()
    p = C.config3_small()
    ref = _oracle("config3_small", p)
    out = N.solve(p, precision="fp64", scheme="synthetic", tol=1e-12, max_iter=5000, tuning=PLANES, accel=5)
    rec = _errors(out, ref, p.T_ref)
    _log("config3_small/fp64/planes/accel", rec)
    assert max(rec["err_TL"], rec["err_T"], rec["err_q"]) < 1e-9, rec


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-9), ("mixed", 1e-6)])
@pytest.mark.parametrize("name", ["config2_small", "tiny_tet"])
def test_plane_layout_second_order(name, precision, bar):
    """Second-order face values: the gradients read the planes through the
    position table (on meshes where the deferred correction contracts)."""
    from test_oracle_pins import tiny_tet
    N = _N()
    p = C.config2_small() if name == "config2_small" else tiny_tet(np.random.default_rng(5))
    r = oracle.solve(p, scheme="synthetic", tol=1e-13, max_iter=20000, defect_tol=1e-11, order=2)
    tol = 1e-12 if precision == "fp64" else 1e-8
    out = N.solve(p, precision=precision, scheme="synthetic", tol=tol, max_iter=20000, allow_not_converged=True,
                  order=2, tuning=PLANES)
    s = np.max(np.abs(r.T_lattice - p.T_ref))
    err = float(np.max(np.abs(out["T_lattice"] - r.T_lattice)) / s)
    errq = float(np.max(np.linalg.norm(out["q"] - r.q, axis=1)) / np.max(np.linalg.norm(r.q, axis=1)))
    _log(f"{name}/{precision}/planes/order2", {"err_TL": err, "err_q": errq})
    assert err < bar and errq < bar


def test_plane_layout_bicgstab():
    N = _N()
    p = C.config1()
    ref = _oracle("config1", p)
    out = N.solve(p, precision="fp64", scheme="sequential", tol=1e-12, max_iter=5000,
                  tuning={"inner_solver": 1, **PLANES})
    rec = _errors(out, ref, p.T_ref)
    _log("config1/fp64/planes/bicgstab", rec)
    assert max(rec["err_TL"], rec["err_T"], rec["err_q"]) < 1e-9, rec


def test_plane_layout_cyclic_mesh():
    """Lagged faces read the upwind cell's previous value through the
    position table."""
    from test_oracle_pins import tiny_dart
    N = _N()
    p = tiny_dart(np.random.default_rng(17), B=3, D=16)
    r = oracle.solve(p, scheme="sequential", tol=1e-14, max_iter=20000)
    out = N.solve(p, precision="fp64", scheme="sequential", tol=1e-12, max_iter=20000, tuning=PLANES)
    s = np.max(np.abs(r.T_lattice - p.T_ref))
    err = float(np.max(np.abs(out["T_lattice"] - r.T_lattice)) / s)
    _log("dart/fp64/planes", {"err_TL": err})
    assert err < 1e-9
