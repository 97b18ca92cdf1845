"""The allocation-free OMP entry point (discover_omp_noalloc) against
discover_omp through the C ABI: the same kernels on the same data, so the
results must be identical, on two calls in a row, the second with a
smaller problem (the shared scratch keeps the first call's contents), and
in both orders of warm start.  A problem too large for the fixed scratch is
refused before any launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _problem(torch, rng, S, n):
    F = rng.normal(size=(S, n)) + rng.uniform(-1, 1, size=(S, 1))
    y = 1.0 + 2.0 * F[3] - 1.5 * F[S // 2] + 0.5 * F[S - 1] + 0.05 * rng.normal(size=n)
    ids = rng.permutation(10 * S)[:S]
    dv = lambda a, dt=None: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    return dv(F), dv(ids, torch.int64), dv(y)


def test_omp_noalloc_equals_omp(torch):
    import paper_2602_06986_amd as D
    ctx = D.Context(0)
    try:
        rng = np.random.default_rng(77)
        for S, n, Dm, init in ((900, 1500, 8, None), (120, 200, 4, (5, 7))):
            F, ids, y = _problem(torch, rng, S, n)
            it = None if init is None else torch.tensor(init, dtype=torch.int32, device="cuda")
            ref = ctx.omp(F, ids, y, Dm, it)
            got = ctx.omp_noalloc(F, ids, y, Dm, it)
            torch.cuda.synchronize()
            for a, b, what in zip(got, ref, ("active", "coef", "rmse", "resid")):
                x, z = a.cpu().numpy(), b.cpu().numpy()
                assert np.array_equal(x, z, equal_nan=x.dtype.kind == "f"), (S, what)
        # about 80 MB of standardised rows: more than the fixed scratch
        F, ids, y = _problem(torch, rng, 5000, 2000)
        with pytest.raises(D.DiscoverError) as e:
            ctx.omp_noalloc(F, ids, y, 4)
        assert e.value.code == -1 and "work space" in str(e.value)
    finally:
        ctx.close()
