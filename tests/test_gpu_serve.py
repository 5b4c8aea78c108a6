"""GPU serving loop: continuous batching (requests admitted by device-memory
footprint while others run) gives every request the result it gets alone."""
import numpy as np
import pytest

from workloads import configs as C

pytestmark = pytest.mark.gpu


def _N():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_03226_amd import nbte
    return nbte


def test_serving_results_equal_alone():
    N = _N()
    from paper_2607_03226_amd import serve
    reqs = [C.serving_request(5000 + j, size_scale=0.03) for j in range(10)]
    arrivals = C.poisson_arrivals(len(reqs), rate=40.0, seed=55)
    foot = []
    for p in reqs:
        mesh, h = N.build_problem(p)
        foot.append(N.nbte_problem_footprint(h, "mixed"))
    # room for about three requests at a time: later ones wait for admission
    budget = int(3 * np.median(foot)) + max(foot)
    served, summary = serve.serve(reqs, arrivals, budget, precision="mixed", tol=1e-8, max_iter=5000, step=4,
                                  keep_results=True)
    assert summary["all_converged"]
    # members and the waiting requests set up ahead never held more than the budget
    assert 0 < summary["peak_bytes_held"] <= budget
    assert summary["p50_s"] <= summary["p99_s"]
    assert all(s.admitted >= s.arrival and s.finished > s.admitted for s in served)
    # the mix really overlapped: some request was admitted before an earlier one finished
    assert any(b.admitted < a.finished for a in served for b in served if b.index > a.index)
    for s, p in zip(served, reqs):
        alone = N.solve(p, precision="mixed", scheme=p.scheme, tol=1e-8, max_iter=5000)
        assert s.result["iterations"] == alone["iterations"], p.name
        for k in ("T_lattice", "T", "q"):
            assert np.array_equal(s.result[k], alone[k]), (p.name, k)
