"""Benchmark of the steady BTE transport path on one MI355X.

A step is one full iteration of the hot path over the whole workload:
lagged boundary inflow, the transport sweep of every (band, direction)
system, the FP64 band x direction reductions, the FP64 synthetic diffusion
correction and the FP64 residual.  value = cell*band*direction updates per
second over the timed steps (inputs resident in HBM).

Default workload: the FinFET-like device (144,480 tetrahedra, 32 bands, 96
directions, Gaussian heat source, partially specular walls), FP32-stored
sweeps with FP64 reductions, synthetic scheme.  --workload config2 runs the
3D non-gray box (24^3 = 13,824 hexahedra, 16 bands, 128 directions).

Also reported on the same line:
  roofline      the sweep kernel's algorithmic bytes per launch / its mean
                HIP-event duration in the timed region, against 8 TB/s.  The
                bytes per update are the method's: the distribution read and
                written once (2 x 4 B in FP32) plus one cached coefficient per
                face, direction and cell shared by the bands (F x 4 B / B);
                the kernel's own stream bytes are reported beside them;
  cpu_baseline  the oracle on this host's cores for a bounded number of
                iterations of the same workload, plus its single-thread
                sweep rate on a sample of (band, direction) systems;
  converge      time-to-converge of the mixed and the FP64 path (same
                stopping rule), plain and with Anderson acceleration of the
                outer iteration (--accel), with their error against the
                stored oracle reference.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload config1..config5]
  config4: the 64-solve batch (time to converge, batched vs one by one);
  config5: the serving stream (p50/p99 latency, solves/s).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell·band·dir updates/s & time-to-converge (mixed vs FP64 @1e-6 rel); p50/p99"
UNIT = "cell·band·dir updates/s"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    from workloads import configs as C
    return {"config1": C.config1, "config2": C.config2, "config3": C.config3}[name]()


def problem_shape(N, tune, p, precision, h):
    shape = tune.settings(p, precision, h)
    if shape:
        N.nbte_set_tuning(h, **shape)
    return shape


def bench_batch(args, N, tune):
    """Config 4: 64 independent porous-film solves in one batch (one launch per
    kernel per iteration for all of them) against the same solves one by one."""
    import torch
    from workloads import configs as C
    probs = C.config4()
    log(f"bench: {len(probs)} porous solves, {sum(p.n_cells for p in probs)} cells")
    ups = [p.updates_per_sweep for p in probs]
    tol, max_iter = 1e-8, 20000
    out = {}
    for prec in ("mixed", "fp64"):
        batch = N.nbte_batch_create()
        keep = []
        for p in probs:
            mesh, h = N.build_problem(p)
            problem_shape(N, tune, p, prec, h)
            keep.append((mesh, h))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the iteration-independent setup of every film, 16 at a time on the
        # host threads (the library call releases the interpreter lock), then
        # admission (initial guess) in order
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=16) as ex:
            list(ex.map(lambda ph: N.nbte_problem_setup(ph[1], prec), keep))
        for p, (mesh, h) in zip(probs, keep):
            N.nbte_batch_admit(batch, h, p.Q, N.make_opts(scheme=p.scheme, precision=prec, T_ref=p.T_ref, tol=tol,
                                                          max_iter=max_iter))
        t_setup = time.perf_counter() - t0
        iters = {}
        while len(iters) < len(probs):
            N.nbte_batch_step(batch, 8)
            done, _ = N.nbte_batch_poll(batch)
            for h in done:
                if h.handle.value not in iters:
                    iters[h.handle.value] = N.nbte_read_result(h)["iterations"]
                    N.nbte_batch_remove(batch, h)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        total = sum(u * iters[h.handle.value] for u, (m, h) in zip(ups, keep))
        out[f"batched_{prec}"] = {"seconds": dt, "setup_s": t_setup, "updates": total, "updates_per_s": total / dt,
                                  "iterations_max": max(iters.values()), "iterations_sum": sum(iters.values())}
        log(f"bench: batched {prec}: {out[f'batched_{prec}']}")
        del batch, keep
    # the same solves one after the other (FP64, per solve)
    t0 = time.perf_counter()
    for p in probs:
        N.solve(p, precision="fp64", scheme=p.scheme, tol=tol, max_iter=max_iter, tuning="auto")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["sequential_fp64"] = {"seconds": dt}
    out["speedup_batched_mixed_vs_sequential_fp64"] = dt / out["batched_mixed"]["seconds"]
    log(f"bench: one by one fp64: {dt:.3f} s")
    return out


def bench_serving(args, N):
    """Config 5: Poisson request stream, continuous batching with admission by
    device-memory footprint; p50/p99 latency and solves/s."""
    import torch
    from paper_2607_03226_amd import serve
    from workloads import configs as C
    # requests generated on a background thread ahead of their arrival and
    # released once served (a 2000-request stream never holds all its meshes)
    reqs = C.RequestStream(5000, args.requests)
    cal = [C.serving_request(9000 + j) for j in range(args.calibration_requests)]   # all arrive at t = 0
    # admission budget: 70 % of the device memory (the rest for the setup of
    # waiting requests, torch and the runtime)
    budget = int(0.7 * torch.cuda.get_device_properties(0).total_memory)
    sat = serve.calibrate(cal, budget, tol=1e-8, tuning="auto")
    rate = args.load * sat
    arrivals = C.poisson_arrivals(len(reqs), rate, seed=5)
    log(f"bench: serving {len(reqs)} requests at {rate:.3f} /s ({args.load} x saturated {sat:.3f} /s over "
        f"{args.calibration_requests} requests), budget {budget / 2**30:.0f} GiB")
    ups = {}

    def note(msg):
        log(msg)

    served, summary = serve.serve(reqs, arrivals, budget, tol=1e-8, tuning="auto", progress=50, progress_log=note)
    reqs.close()
    summary["arrival_rate_per_s"] = rate
    summary["load_factor"] = args.load
    summary["saturated_solves_per_s"] = sat
    summary["calibration_requests"] = args.calibration_requests
    summary["updates"] = sum(s.updates for s in served)
    log(f"bench: serving {summary}")
    return summary


def method_bytes_per_update(p, precision):
    """Algorithmic bytes per cell x band x direction update of the method's
    transport step (Methods, Eqs. (13)-(14)): the distribution read and
    written once, 2 s_e, plus the per-(face, direction) coefficient of each
    cell, cached once and shared by the B bands, F s_c / B, plus the per-cell
    geometry and fields, (16 F + 48) / (B D)."""
    es = 4 if precision == "mixed" else 8
    F = {"tri3": 3, "quad4": 4, "tet4": 4, "hex8": 6}[p.cell_type]
    return 2 * es + F * es / p.n_bands + (16 * F + 48) / (p.n_bands * p.n_dirs)


PLANES_MIN_VALUES = 1 << 26   # the library's automatic layout choice (plane layout from 2^26 values)


def sweep_algorithmic_bytes(p, precision):
    """Compulsory HBM bytes of one launch of this library's sweep: every distribution value
    written once; the level-ordered streams of every (direction, cell) read
    once (cell (cell-major layout only), slot, up to F-1 upwind references,
    their coefficients, the outflow sum, the imbalance term D and the source,
    the real-valued ones in the storage type); the boundary inflow of every
    incoming (face, direction) read once.  Returns (bytes per launch, bytes
    per update)."""
    es = 4 if precision == "mixed" else 8
    N, B, D = p.n_cells, p.n_bands, p.n_dirs
    F = {"tri3": 3, "quad4": 4, "tet4": 4, "hex8": 6}[p.cell_type]
    mi = {"tri3": 2, "quad4": 2, "tet4": 3, "hex8": 3}[p.cell_type]   # most upwind faces of one cell
    dist = N * B * D * es
    cell = 0 if N * B * D >= PLANES_MIN_VALUES else 4
    streams = D * N * (cell + 4 + 4 * mi + es * (mi + 3))
    inflow = len(p.bfaces) * (D // 2) * B * es             # incoming half of the directions
    total = dist + streams + inflow
    return total, total / (N * B * D)


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2607_03226_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def _shape_key(shape):
    """the launch-shape settings that select the sweep kernel and its work"""
    keys = ("bands_per_block", "bands_per_lane", "block_size", "lds_bytes")
    return {k: int(shape[k]) for k in keys if shape and k in shape} if shape else None


def counter_traffic(workload_name, precision, shape):
    """HBM traffic per sweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source with the launch
    shape the bench uses now."""
    path = os.path.join(ROOT, "profiles", f"sweep_{workload_name}_{precision}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if d.get("shape") != _shape_key(shape):
        return None
    return d.get("traffic_bytes_per_launch")


def _counter_rows(d):
    """rows of a rocprofv3 --pmc CSV output directory"""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _median_counter(rows, name_part, counter, pick_largest_grid=False):
    vals = [(int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows
            if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        return None
    if pick_largest_grid:
        g = max(v[0] for v in vals)
        vals = [v for v in vals if v[0] == g]
    xs = sorted(v[1] for v in vals)
    return xs[len(xs) // 2]


def _tuned_shape(workload_name, precision):
    """the launch shape bench.py runs a workload with (autotuner cache)"""
    from paper_2607_03226_amd import tune
    return tune.lookup(workload(workload_name), precision)


def counter_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, probe_bytes):
    """The sweep's HBM traffic per launch from four rocprofv3 --pmc runs
    (FETCH_SIZE and WRITE_SIZE of the bench, then of the copy probe).  The
    counters (KiB per dispatch) are scaled by what they read for a device
    copy of probe_bytes; the raw sum is kept beside the scaled one."""
    fetch = _median_counter(_counter_rows(fetch_dir), "k_sweep", "FETCH_SIZE")
    write = _median_counter(_counter_rows(write_dir), "k_sweep", "WRITE_SIZE")
    cf = _median_counter(_counter_rows(copy_fetch_dir), "copyBuffer", "FETCH_SIZE", pick_largest_grid=True)
    cw = _median_counter(_counter_rows(copy_write_dir), "copyBuffer", "WRITE_SIZE", pick_largest_grid=True)
    ffac, wfac = probe_bytes / (cf * 1024.0), probe_bytes / (cw * 1024.0)
    return {"fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
            "copy_probe_bytes": probe_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
            "fetch_scale": ffac, "write_scale": wfac,
            "traffic_bytes_per_launch": fetch * 1024.0 * ffac + write * 1024.0 * wfac,
            "raw_bytes_per_launch": (fetch + write) * 1024.0}


def summarize_counters(args):
    """Write profiles/sweep_<workload>_<precision>_counters.json from the four
    rocprofv3 --pmc output directories."""
    fd, wd, cfd, cwd = args.summarize
    probe = args.copy_probe_bytes
    out = {"kernel": "k_sweep", "workload": args.workload, "precision": args.precision}
    out.update(counter_summary(fd, wd, cfd, cwd, probe))
    out.update({"kernel_source_sha256_16": kernel_source_hash(),
                "shape": _shape_key(_tuned_shape(args.workload, args.precision)),
                "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o run -- python bench.py "
                             f"--workload {args.workload} --precision {args.precision} "
                             f"--steps {args.steps} --warmup {args.warmup} --no-cpu --no-converge",
                             "rocprofv3 --pmc WRITE_SIZE (same)",
                             f"rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE -- python bench.py --copy-probe {probe >> 20}"]})
    path = os.path.join(ROOT, "profiles", f"sweep_{args.workload}_{args.precision}_counters.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def _host_cpu():
    """core count and model of the host the CPU baseline ran on"""
    info = {"nproc": os.cpu_count()}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    try:
        info["sched_affinity"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return info


def cpu_baseline(p, max_iters, seconds, one_thread_seconds=5.0):
    """The oracle's full synthetic iterations on the host cores (OpenMP over
    the band x direction systems), as many as fit in about `seconds` (at
    least one, at most max_iters); then its single-thread sweep rate: the
    exact transport solve of (band, direction) systems, one after the other
    on one core, for about `one_thread_seconds`."""
    import oracle
    t0 = time.perf_counter()
    su = oracle.prepare(p)
    # the correction's sparse LU is iteration-independent setup (factorized
    # once, then reused by every iteration), so it is made before the timed
    # region; the iterations start from the uniform reference temperature
    # (the rate does not depend on the start, and the Fourier guess would be
    # another factorization)
    oracle.diffusion_operator(su)
    t_setup = time.perf_counter() - t0
    threads = oracle.threads()
    theta = np.zeros(su.g.N)
    e = np.broadcast_to(oracle.equilibrium(su, theta)[:, None, :], (p.n_bands, p.n_dirs, su.g.N))
    t0 = time.perf_counter()
    iters = 0
    while iters < max(1, max_iters) and (iters == 0 or time.perf_counter() - t0 < seconds):
        iters += 1
        inflow = oracle.boundary_inflow(su, e)
        e, outflux = oracle.transport(su, theta, inflow)
        ts, _, _ = oracle.moments(su, e)
        r = su.Q - oracle.divergence(su, outflux)
        flows = oracle.boundary_flows(su, e, inflow)
        refl = su.bc_kind != 0
        np.add.at(r, su.g.bf_owner[refl], flows[refl] / su.g.V[su.g.bf_owner[refl]])
        theta = ts + oracle.diffusion_operator(su)[1].solve(su.g.V * r)
    dt = time.perf_counter() - t0
    # one core: systems in a seeded order, each solved exactly by the C sweep
    rng = np.random.default_rng(0)
    order = [(int(b), int(i)) for b, i in zip(rng.integers(p.n_bands, size=4096), rng.integers(p.n_dirs, size=4096))]
    t1 = time.perf_counter()
    k = 0
    while k < len(order) and (k < 4 or time.perf_counter() - t1 < one_thread_seconds):
        oracle.transport_systems(su, theta, inflow, order[k:k + 4])
        k += 4
    dt1 = time.perf_counter() - t1
    return {"value": p.updates_per_sweep * iters / dt, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{iters} full synthetic iterations of {p.name} (FP64, OpenMP over band x direction "
                      f"systems on {threads} threads), setup {t_setup:.1f} s excluded (geometry, tables and "
                      f"the correction's sparse LU)", "seconds": dt, "setup_seconds": t_setup,
            "one_thread_sweep": {"value": p.n_cells * k / dt1, "unit": UNIT, "cores": 1, "seconds": dt1,
                                 "sample": f"exact transport solves of {k} seeded (band, direction) systems "
                                           f"of {p.name}, one core"},
            "host": _host_cpu()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="config3", choices=["config1", "config2", "config3", "config4", "config5"])
    ap.add_argument("--requests", type=int, default=2000, help="config5: number of requests")
    ap.add_argument("--calibration-requests", type=int, default=64,
                    help="config5: requests of the saturated-rate calibration (all arriving at once)")
    ap.add_argument("--load", type=float, default=0.7,
                    help="config5: arrival rate as a fraction of the calibrated saturated rate")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--cpu-iters", type=int, default=40, help="most oracle iterations of the CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU baseline sample length (about)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--accel", type=int, default=-1,
                    help="Anderson depth of the accelerated time-to-converge legs (-1: the autotuner's)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    ap.add_argument("--summarize", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the sweep's counter traffic summary from rocprofv3 --pmc outputs and exit")
    ap.add_argument("--copy-probe-bytes", type=int, default=1 << 30)
    args = ap.parse_args()
    if args.summarize:
        summarize_counters(args)
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the per-GPU path is what "
              "is measured (every solve and batch lives on one GPU; nothing here uses a second)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        n = args.copy_probe << 17                 # float64 elements of MIB MiB
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}), flush=True)
        return
    from paper_2607_03226_amd import nbte as N
    from paper_2607_03226_amd import tune

    if args.workload in ("config4", "config5"):
        t0 = time.perf_counter()
        extra = bench_batch(args, N, tune) if args.workload == "config4" else bench_serving(args, N)
        dt = time.perf_counter() - t0
        if args.workload == "config4":
            value, name = extra["batched_mixed"]["updates_per_s"], "porous_films_64_B8_D32"
        else:
            value, name = extra["updates"] / extra["span_s"], f"serving_stream_{args.requests}"
        # the oracle on one solve of the workload: the median film of the batch,
        # or the stream's first request
        cpu = None
        if not args.no_cpu:
            from workloads import configs as C
            if args.workload == "config4":
                films = C.config4()
                ups = [q.updates_per_sweep for q in films]
                sample = films[int(np.argsort(ups)[len(ups) // 2])]
            else:
                sample = C.serving_request(5000)
            cpu = cpu_baseline(sample, max(args.cpu_iters, 1000), args.cpu_seconds)   # bounded by the seconds
            log(f"bench: cpu baseline {cpu}")
        line = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": None, "warmup": None,
                "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32-stored/f32-sweep/f64-reductions", "data": "synthetic",
                "config": {"workload": name}, "roofline": None, "cpu_baseline": cpu,
                args.workload == "config4" and "batch" or "serving": extra, "seconds": dt}
        print(json.dumps(line), flush=True)
        return

    p = workload(args.workload)
    log(f"bench: workload {p.name} N={p.n_cells} B={p.n_bands} D={p.n_dirs} precision {args.precision}")
    mesh, h = N.build_problem(p)
    shape = tune.lookup(p, args.precision)
    # the timed step is one plain iteration of the method: the tuned launch
    # shape and CG cap, no Anderson mixing (that changes the iteration count
    # to converge, timed in the converge legs below, not the step)
    if shape:
        shape = dict(shape, accel_depth=0)
        N.nbte_set_tuning(h, **shape)
    log(f"bench: sweep shape {shape or 'library default'}")
    # timed region 1 (the value): the production form, iterations replayed
    # from HIP graphs with no timing events between the kernels
    opts = N.make_opts(scheme=p.scheme, precision=args.precision, T_ref=p.T_ref)
    N.nbte_prepare(h, p.Q, opts)
    N.nbte_iterate(h, args.warmup, check=True)
    torch.cuda.synchronize()
    N.nbte_prepare(h, p.Q, opts)
    N.nbte_iterate(h, args.warmup, check=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = N.nbte_iterate(h, args.steps, check=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ups = p.updates_per_sweep
    value = ups * args.steps / dt
    # timed region 2 (the kernel): the same steps launched one by one with HIP
    # events recorded by the library on its stream around each phase; the
    # sweep's mean event-to-event time is the roofline's launch duration
    opts_t = N.make_opts(scheme=p.scheme, precision=args.precision, T_ref=p.T_ref, time_phases=True)
    N.nbte_prepare(h, p.Q, opts_t)
    N.nbte_iterate(h, args.warmup, check=True)
    st0 = N.nbte_get_stats(h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    N.nbte_iterate(h, args.steps, check=True)
    torch.cuda.synchronize()
    dt_events = time.perf_counter() - t1
    st = N.nbte_get_stats(h)
    launches = st["sweep_launches"] - st0["sweep_launches"]
    ms_sweep = (st["ms_sweep"] - st0["ms_sweep"]) / max(launches, 1)
    phases = {k: (st[k] - st0[k]) / max(launches, 1) for k in ("ms_bc", "ms_sweep", "ms_moments", "ms_synthetic", "ms_update")}
    log(f"bench: {args.steps} steps in {dt:.4f} s -> {value:.4e} updates/s (graphs); with phase events "
        f"{dt_events / args.steps * 1e3:.4f} ms/step; sweep {ms_sweep:.4f} ms; residual {res:.2e}")

    per_update = method_bytes_per_update(p, args.precision)
    alg_bytes = per_update * ups
    achieved = alg_bytes / (ms_sweep * 1e-3) / 1e9
    own_bytes, own_per_update = sweep_algorithmic_bytes(p, args.precision)
    traffic = counter_traffic(args.workload, args.precision, shape)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_sweep", "algorithmic_bytes_per_update": per_update,
                "algorithmic_bytes_per_launch": alg_bytes,
                "kernel_stream_bytes_per_update": own_per_update,
                "frac_kernel_stream_bytes": own_bytes / (ms_sweep * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "sweep_ms_mean": ms_sweep, "sweep_updates_per_s": ups / (ms_sweep * 1e-3)}

    converge = None
    if not args.no_converge:
        converge = {}
        ref_path = os.path.join(ROOT, "tests", "golden", f"{args.workload}_reference.npz")
        ref = np.load(ref_path) if os.path.exists(ref_path) else None
        # mixed: the tuned form (launch shape, CG cap and Anderson depth from the
        # autotuner cache, or --accel); fp64: the plain FP64 per-system path (its
        # tuned shape and CG cap, no acceleration); plus the mixed path without
        # acceleration and the FP64 path with it, for the two effects apart
        def depth(prec):
            if args.accel >= 0:
                return args.accel
            return int((tune.lookup(p, prec) or {}).get("accel_depth", 0))
        legs = [("mixed", "mixed", depth("mixed")), ("fp64", "fp64", 0),
                ("mixed_plain", "mixed", 0), ("fp64_accelerated", "fp64", depth("fp64"))]
        for leg, prec, acc in legs:
            sh = dict(tune.lookup(p, prec) or {}, accel_depth=acc)
            N.nbte_set_tuning(h, **sh)
            o2 = N.make_opts(scheme=p.scheme, precision=prec, T_ref=p.T_ref, tol=1e-8, max_iter=20000)
            N.nbte_solve_steady(h, p.Q, o2)       # setup for this precision cached by the first call
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            out = N.nbte_solve_steady(h, p.Q, o2)
            torch.cuda.synchronize()
            t_conv = time.perf_counter() - t1
            rec = {"seconds": t_conv, "iterations": out["iterations"], "residual": out["residual"],
                   "energy_defect": out["energy_defect"], "precision": prec, "accel_depth": acc,
                   "cg_max_iter": int(sh.get("cg_max_iter", 0))}
            if ref is not None:
                c = ref["cells"] if "cells" in ref.files else slice(None)
                rec["err_TL"] = float(np.max(np.abs(out["T_lattice"][c] - ref["T_lattice"])) / ref["scale_TL"])
                rec["err_T"] = float(np.max(np.abs(out["T"][c] - ref["T"])) / ref["scale_T"])
                rec["err_q"] = float(np.max(np.linalg.norm(out["q"][c] - ref["q"], axis=1)) / ref["scale_q"])
                rec["cells_compared"] = int(len(ref["T_lattice"]))
            converge[leg] = rec
            log(f"bench: converge {leg}: {rec}")
        converge["speedup_mixed_vs_fp64"] = converge["fp64"]["seconds"] / converge["mixed"]["seconds"]
        converge["speedup_precision_alone"] = converge["fp64"]["seconds"] / converge["mixed_plain"]["seconds"]
        converge["speedup_acceleration_alone_fp64"] = (converge["fp64"]["seconds"] /
                                                        converge["fp64_accelerated"]["seconds"])

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(p, args.cpu_iters, args.cpu_seconds)
        log(f"bench: cpu baseline {cpu}")

    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-stored/f32-sweep/f64-reductions" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": p.name, "cells": p.n_cells, "bands": p.n_bands, "directions": p.n_dirs,
                   "cell_type": p.cell_type, "scheme": p.scheme, "precision": args.precision,
                   "updates_per_step": ups},
        "roofline": roofline, "cpu_baseline": cpu, "converge": converge,
        "phases_ms_per_step": phases, "ms_per_step_with_phase_events": dt_events / args.steps * 1e3,
        "sweep_shape": {k: st[k] for k in ("bands_per_block", "bands_per_lane", "block_size", "lds_slots",
                                           "spilled_values", "max_levels")},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
