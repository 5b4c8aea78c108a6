"""The allocation-free distribution read against the allocating one, through
the C ABI: two calls in a row on one GPU, the second on a smaller problem (the
shared staging array keeps the first call's values beyond the second mesh's
cells, which must not leak into the result), every (band, direction) sampled
bitwise equal; an unprepared problem is refused."""
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


def _prepared(N, p, precision):
    mesh, h = N.build_problem(p)
    N.nbte_prepare(h, p.Q, N.make_opts(scheme=p.scheme, precision=precision, T_ref=p.T_ref))
    N.nbte_iterate(h, 3)
    return mesh, h


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_read_equals_allocating_read(precision):
    N = _N()
    big, small = C.config2_small(), C.config1()
    assert big.n_cells > small.n_cells
    for p in (big, small):
        mesh, h = _prepared(N, p, precision)
        rng = np.random.default_rng(p.n_cells)
        systems = [(0, 0), (p.n_bands - 1, p.n_dirs - 1)]
        systems += [(int(rng.integers(p.n_bands)), int(rng.integers(p.n_dirs))) for _ in range(4)]
        for b, i in systems:
            a = N.nbte_get_distribution(h, b, i)
            z = N.nbte_get_distribution_noalloc(h, b, i)
            assert z.shape == (p.n_cells,)
            assert np.all(np.isfinite(z))
            np.testing.assert_array_equal(z, a)


def test_noalloc_read_refuses_unprepared_and_out_of_range():
    N = _N()
    p = C.config1()
    mesh, h = N.build_problem(p)
    with pytest.raises(N.NbteError) as e:
        N.nbte_get_distribution_noalloc(h, 0, 0)
    assert e.value.status == N.ERR_STATE
    N.nbte_prepare(h, p.Q, N.make_opts(scheme=p.scheme, precision="fp64", T_ref=p.T_ref))
    with pytest.raises(N.NbteError) as e:
        N.nbte_get_distribution_noalloc(h, p.n_bands, 0)
    assert e.value.status == N.ERR_INVALID_ARG
