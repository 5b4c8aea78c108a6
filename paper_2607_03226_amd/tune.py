"""Autotuner of the sweep launch shape and the iteration settings.

For a problem it times candidate shapes (bands per workgroup, bands per lane,
workgroup size, LDS budget) through the C ABI's HIP-event phase timers and
keeps the fastest; it then picks the CG iteration cap of the diffusion
correction (synthetic schemes) and the Anderson depth of the outer iteration
together, by time-to-converge.  Results are cached in tune_cache.json next to this file,
keyed by (cell type, cell-count bucket, bands, directions, precision), and
looked up by nbte.solve(..., tuning="auto").
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

from . import nbte as N

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def key(problem, precision):
    bucket = int(round(math.log2(max(problem.n_cells, 1)) * 2))   # half-octave buckets
    return f"{problem.cell_type}|{bucket}|B{problem.n_bands}|D{problem.n_dirs}|{precision}"


def load_cache():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def save_cache(cache):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def lookup(problem, precision):
    return load_cache().get(key(problem, precision), {}).get("shape")


def settings(problem, precision, h):
    """The cached settings to run a built problem with (None if its workload
    class was never tuned).  A cached Anderson depth is dropped when the
    problem's upwind graphs have lagged (cyclic) faces: the library does not
    accelerate those, and the cache entry is shared by every mesh of the class."""
    shape = lookup(problem, precision)
    if shape and shape.get("accel_depth", 0) > 0:
        if any(len(N.nbte_get_lagged_faces(h, d)[0]) for d in range(problem.n_dirs)):
            shape = dict(shape, accel_depth=0)
    return shape


WHOLE_CU_LDS = 163840   # a CU's LDS: one sweep workgroup per CU, every value staged where it fits


def candidates(B):
    """Launch shapes to time: bands per workgroup, bands per lane (several lanes
    per cell, or one lane per cell sweeping every band of the block),
    workgroup size, and the LDS budget (the default, or a whole CU's: fewer
    workgroups per CU but no values spilled to HBM; config 3 mixed: 1.74 ->
    1.45 ms)."""
    bpbs = [b for b in (1, 2, 4, 8, 16, 32) if b <= B] + ([B] if B not in (1, 2, 4, 8, 16, 32) and B <= 64 else [])
    out = []
    for bpb, block in itertools.product(bpbs, (128, 256, 512)):
        bpls = {1, 2, 4} | ({bpb} if bpb <= 8 else set())
        for bpl in sorted(bpls):
            if bpl > bpb or (bpb + bpl - 1) // bpl > 64:
                continue
            for lds in (0, WHOLE_CU_LDS):
                out.append({"bands_per_block": bpb, "bands_per_lane": bpl, "block_size": block, "lds_bytes": lds})
    return out


def time_shape(h, problem, precision, shape, iters=4):
    N.nbte_set_tuning(h, **shape)
    opts = N.make_opts(scheme="sequential", precision=precision, T_ref=problem.T_ref, time_phases=True,
                       T_init=[problem.T_ref + 0.5] * problem.n_cells)
    N.nbte_prepare(h, problem.Q, opts)
    N.nbte_iterate(h, 1, check=True)          # warm-up (first-launch costs)
    st0 = N.nbte_get_stats(h)
    N.nbte_iterate(h, iters, check=True)
    st = N.nbte_get_stats(h)
    n = st["sweep_launches"] - st0["sweep_launches"]
    return (st["ms_sweep"] - st0["ms_sweep"]) / max(n, 1)


def time_to_converge(h, problem, precision, shape, tol=1e-8, max_iter=20000, reps=2):
    """Wall time of a whole steady solve (setup cached) with a launch shape."""
    N.nbte_set_tuning(h, **shape)
    opts = N.make_opts(scheme=problem.scheme, precision=precision, T_ref=problem.T_ref, tol=tol, max_iter=max_iter)
    N.nbte_solve_steady(h, problem.Q, opts)        # setup for this shape and precision
    best, iters = float("inf"), 0
    for _ in range(reps):
        t = time.perf_counter()
        out = N.nbte_solve_steady(h, problem.Q, opts)
        best = min(best, time.perf_counter() - t)
        iters = out["iterations"]
    return best, iters


def tune_convergence(h, problem, precision, shape, cg_choices=(4, 8, 16, 32), accel_choices=(0, 5, 8),
                     verbose=True):
    """The iteration settings by time-to-converge on a fixed launch shape: the
    correction's CG iteration cap (synthetic schemes; fewer CG launches per
    iteration against more outer iterations) jointly with the Anderson depth
    of the outer iteration (0 = plain).  Returns the shape with both set."""
    caps = cg_choices if problem.scheme != "sequential" and cg_choices else (shape.get("cg_max_iter", 0),)
    conv = []
    for acc in accel_choices:
        for cg in caps:
            trial = dict(shape, cg_max_iter=cg, accel_depth=acc)
            try:
                sec, it = time_to_converge(h, problem, precision, trial)
            except N.NbteError as e:      # e.g. acceleration on a mesh with lagged faces
                if verbose:
                    print(f"tune: {problem.name} {precision} accel {acc} cg {cg}: {e}", flush=True)
                continue
            conv.append((sec, acc, cg))
            if verbose:
                print(f"tune: {problem.name} {precision} accel_depth {acc} cg_max_iter {cg}: converged in {it} "
                      f"iterations, {sec:.4f} s", flush=True)
    sec, acc, cg = min(conv)
    return dict(shape, cg_max_iter=cg, accel_depth=acc)


def tune(problem, precision="mixed", shapes=None, iters=4, verbose=True, write=True,
         cg_choices=(4, 8, 16, 32), accel_choices=(0, 5, 8)):
    """Fastest sweep shape by sweep time; then the correction's CG iteration
    cap and the outer Anderson depth by time-to-converge (tune_convergence)."""
    mesh, h = N.build_problem(problem)
    table = []
    t0 = time.time()
    for shape in shapes or candidates(problem.n_bands):
        try:
            ms = time_shape(h, problem, precision, shape, iters)
        except N.NbteError as e:
            if verbose:
                print(f"tune: {shape} rejected: {e}", flush=True)
            continue
        table.append((ms, shape))
        if verbose:
            ups = problem.updates_per_sweep / (ms * 1e-3)
            print(f"tune: {problem.name} {precision} {shape} sweep {ms:.4f} ms ({ups:.3e} updates/s)", flush=True)
    table.sort(key=lambda t: t[0])
    best_ms, best = table[0]
    best = tune_convergence(h, problem, precision, dict(best), cg_choices, accel_choices, verbose)
    if write:
        cache = load_cache()
        cache[key(problem, precision)] = {"shape": best, "sweep_ms": best_ms, "workload": problem.name,
                                          "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S"),
                                          "seconds": time.time() - t0}
        save_cache(cache)
    return best, best_ms, table


def retune_convergence(problem, precision="mixed", verbose=True, **kw):
    """Redo only the iteration settings of a cached entry (its launch shape kept)."""
    cache = load_cache()
    k = key(problem, precision)
    if k not in cache:
        return tune(problem, precision, verbose=verbose)[0]
    mesh, h = N.build_problem(problem)
    shape = {a: b for a, b in cache[k]["shape"].items() if a not in ("cg_max_iter", "accel_depth")}
    best = tune_convergence(h, problem, precision, shape, verbose=verbose, **kw)
    cache = load_cache()
    cache[k]["shape"] = best
    cache[k]["converge_tuned_at"] = time.strftime("%Y-%m-%d %H:%M:%S")
    save_cache(cache)
    return best


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import configs as C
    if sys.argv[1:2] == ["--converge"]:
        for name in sys.argv[2:]:
            p = {"config1": C.config1, "config2": C.config2, "config3": C.config3}[name]()
            for prec in ("mixed", "fp64"):
                print(f"tune: BEST {name} {prec} {retune_convergence(p, prec)}", flush=True)
        sys.exit(0)
    names = sys.argv[1:] or ["config2"]
    for name in names:
        if name == "config4":
            # one representative film per cache key (size bucket) of the batch
            seen = set()
            for p in C.config4():
                k = key(p, "mixed")
                if k in seen:
                    continue
                seen.add(k)
                for prec in ("mixed", "fp64"):
                    best, ms, _ = tune(p, prec, verbose=False)
                    print(f"tune: BEST config4/{p.name} {prec} {best} {ms:.4f} ms", flush=True)
            continue
        p = {"config1": C.config1, "config2": C.config2, "config3": C.config3}[name]()
        for prec in ("mixed", "fp64"):
            best, ms, _ = tune(p, prec)
            print(f"tune: BEST {name} {prec} {best} {ms:.4f} ms", flush=True)
