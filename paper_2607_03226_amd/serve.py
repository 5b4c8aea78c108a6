"""Serving loop: continuous batching of steady-solve requests over the C ABI.

Requests arrive over time.  Each is set up on the host (mesh, band table,
quadrature, boundaries: the per-geometry setup counts in its latency) and
admitted into the running batch as soon as its device footprint fits the
budget (nbte_batch_admit refuses it otherwise and it waits, first come first
served).  Every step advances all running solves together (one launch per
kernel for all of them, replayed from a HIP graph); a solve leaves the batch
as soon as the device stops it at its tolerance, and its result is read while
the others keep running.  New requests are set up and admitted while the
enqueued step runs on the GPU; their device setup starts only once their
footprint fits the budget beside the running solves (see serve()).

serve() returns per-request latency (finish - arrival), p50/p99 and the
throughput in solves/s.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import nbte as N


@dataclass
class Served:
    index: int
    name: str
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    iterations: int = 0
    residual: float = float("nan")
    converged: bool = False
    updates: int = 0            # cell x band x direction updates of its iterations
    result: dict = field(default=None, repr=False)

    @property
    def latency(self):
        return self.finished - self.arrival


def percentile(x, q):
    x = np.sort(np.asarray(x, dtype=float))
    if len(x) == 0:
        return float("nan")
    return float(np.percentile(x, q))


def serve(requests, arrivals, budget_bytes, precision="mixed", tol=1e-8, max_iter=20000, step=8,
          keep_results=False, tuning=None, clock=time.perf_counter, log=None, lookahead=4, progress=0,
          progress_log=print):
    """Run the request stream.

    requests  list of problem descriptions (see nbte.build_problem)
    arrivals  arrival times in seconds from the start (non-decreasing)
    budget    device bytes the running solves and the set-up waiting requests
              may hold together (0: no limit)
    tuning    None, "auto" (autotuner cache) or a dict of launch-shape settings
    lookahead waiting requests whose setup runs ahead on host threads
    progress  report every `progress` finished requests through progress_log
    requests may be a sequence that builds requests on demand and has
    release(j) (workloads.configs.RequestStream): served ones are released.
    Returns (list of Served, summary dict).
    """
    n = len(requests)
    batch = N.nbte_batch_create(budget_bytes)
    served = [Served(j, "", float(arrivals[j])) for j in range(n)]
    release = getattr(requests, "release", None)   # streams generated on demand drop served requests
    queue = collections.deque()
    handles = {}                # handle value -> (index, mesh, problem handle)
    next_arrival = 0
    done_count = 0
    t0 = clock()
    peak = [0]                  # most device bytes held by members and set-up waiting requests

    def now():
        return clock() - t0

    # Setup of waiting requests, on host threads for the first `lookahead`
    # requests in the queue while the GPU steps the batch.  The host part
    # (mesh, tables, the footprint query) holds no device memory; the device
    # part (nbte_problem_setup: schedules, streams, state) starts only once
    # the request's footprint is reserved next to the batch's members and the
    # other reservations, in queue order, so members plus set-up requests
    # never hold more than the budget.  A reservation becomes the member's
    # charge at admission.
    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=max(1, lookahead))
    host_built, dev_built, reserved = {}, {}, {}

    def host_part(j):
        p = requests[j]
        served[j].name = p.name
        mesh, h = N.build_problem(p)
        if tuning == "auto":
            from . import tune
            shape = tune.settings(p, precision, h)
            if shape:
                N.nbte_set_tuning(h, **shape)
        elif tuning:
            N.nbte_set_tuning(h, **tuning)
        return mesh, h, N.nbte_problem_footprint(h, precision)

    def dev_part(j):
        mesh, h, _ = host_built[j].result()
        N.nbte_problem_setup(h, precision)
        return mesh, h

    def held():
        return N.nbte_batch_get_info(batch)["bytes_in_use"] + sum(reserved.values())

    def start_setups():
        ahead = list(queue)[:max(1, lookahead)]
        for j in ahead:
            if j not in host_built:
                host_built[j] = pool.submit(host_part, j)
        for j in ahead:                       # reservations in queue order
            if j in dev_built:
                continue
            if not host_built[j].done():
                break
            foot = host_built[j].result()[2]
            if budget_bytes > 0 and held() + foot > budget_bytes:
                break
            reserved[j] = foot
            peak[0] = max(peak[0], held())
            dev_built[j] = pool.submit(dev_part, j)

    def admit_waiting():
        while queue:
            start_setups()
            j = queue[0]
            p = requests[j]
            if j not in dev_built:
                if handles:
                    return            # running solves free memory, or the host part is still running
                host_built[j].result()
                start_setups()
                if j not in dev_built:
                    raise RuntimeError(f"request {j} ({p.name}) does not fit the budget even alone")
            mesh, h = dev_built[j].result()
            opts = N.make_opts(scheme=p.scheme, precision=precision, T_ref=p.T_ref, tol=tol, max_iter=max_iter)
            try:
                N.nbte_batch_admit(batch, h, p.Q, opts)
            except N.NbteError as e:
                if e.status != N.ERR_OUT_OF_MEMORY:
                    raise
                if not handles:
                    raise RuntimeError(f"request {j} ({p.name}) does not fit the budget even alone") from e
                return              # wait for running solves to leave
            queue.popleft()
            del reserved[j], host_built[j], dev_built[j]
            peak[0] = max(peak[0], held())
            handles[h.handle.value] = (j, mesh, h)
            served[j].admitted = now()
            if log:
                log(f"serve: t={served[j].admitted:.3f} s admitted {j} {p.name}")

    while done_count < n:
        t = now()
        while next_arrival < n and arrivals[next_arrival] <= t:
            queue.append(next_arrival)
            next_arrival += 1
        if not handles:
            admit_waiting()
            if not handles:
                if next_arrival < n:
                    time.sleep(max(0.0, arrivals[next_arrival] - now()))
                continue
        N.nbte_batch_step(batch, step)          # asynchronous
        admit_waiting()                          # host setup overlaps the step on the GPU
        finished, _ = N.nbte_batch_poll(batch)
        for h in finished:
            j, mesh, hh = handles.pop(h.handle.value)
            out = N.nbte_read_result(h)
            N.nbte_batch_remove(batch, h)
            s = served[j]
            s.finished = now()
            s.iterations = out["iterations"]
            s.updates = requests[j].updates_per_sweep * s.iterations
            s.residual = out["residual"]
            s.converged = bool(out["residual"] <= tol)
            if keep_results:
                s.result = {k: out[k] for k in ("T_lattice", "T", "q", "iterations", "residual", "energy_defect")}
            done_count += 1
            if log:
                log(f"serve: t={s.finished:.3f} s finished {j} {s.name} in {s.iterations} iterations, "
                    f"latency {s.latency:.3f} s")
            del mesh, hh
            if release:
                release(j)
            if progress and done_count % progress == 0:
                progress_log(f"serve: {done_count}/{n} finished at t={now():.1f} s")
    pool.shutdown(wait=True)
    lat = [s.latency for s in served]
    span = max(s.finished for s in served) - min(s.arrival for s in served)
    summary = {"requests": n, "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
               "mean_s": float(np.mean(lat)), "solves_per_s": n / span if span > 0 else float("inf"),
               "span_s": span, "all_converged": all(s.converged for s in served),
               "budget_bytes": int(budget_bytes), "peak_bytes_held": int(peak[0])}
    return served, summary


def calibrate(requests, budget_bytes, **kw):
    """Saturated throughput: every request arrives at t = 0."""
    _, summary = serve(requests, np.zeros(len(requests)), budget_bytes, **kw)
    return summary["solves_per_s"]
