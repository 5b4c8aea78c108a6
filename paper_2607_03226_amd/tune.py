"""Autotuner of the sweep launch shape and the correction's CG cap.

For a problem it times candidate shapes (bands per workgroup, bands per lane,
workgroup size, LDS budget) through the C ABI's HIP-event phase timers and
keeps the fastest; for the synthetic schemes it then picks the CG iteration
cap of the diffusion correction by time-to-converge.  Results are cached in tune_cache.json next to this file,
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


def tune(problem, precision="mixed", shapes=None, iters=4, verbose=True, write=True,
         cg_choices=(4, 6, 8, 12, 16, 24, 32)):
    """Fastest sweep shape by sweep time; then, for the synthetic schemes, the
    correction's CG iteration cap by time-to-converge (fewer CG launches per
    iteration against more outer iterations)."""
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
    best = dict(best)
    if problem.scheme != "sequential" and cg_choices:
        conv = []
        for cg in cg_choices:
            sec, it = time_to_converge(h, problem, precision, dict(best, cg_max_iter=cg))
            conv.append((sec, cg))
            if verbose:
                print(f"tune: {problem.name} {precision} cg_max_iter {cg}: converged in {it} iterations, {sec:.4f} s",
                      flush=True)
        best["cg_max_iter"] = min(conv)[1]
    if write:
        cache = load_cache()
        cache[key(problem, precision)] = {"shape": best, "sweep_ms": best_ms, "workload": problem.name,
                                          "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S"),
                                          "seconds": time.time() - t0}
        save_cache(cache)
    return best, best_ms, table


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from workloads import configs as C
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
