"""bddc_apply_noalloc (the allocation-free variant of bddc_apply) against
bddc_apply through the C ABI: the same preconditioned vectors, bit for bit
(the same kernels in the same order on the same inputs), on two calls in a
row, the second on a smaller problem, so that the static work array carries
the first call's contents into the second; also with two right-hand sides.
The library's device allocations go through torch's caching allocator, whose
allocation count must not move during the allocation-free calls."""
import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _factored(p, tau=None):
    from paper_0910_5863_amd import BDDC
    b = BDDC()
    b.setup(p, "ce")
    if tau is not None:
        b.adapt(tau)
    b.factor()
    return b


def _rhs(n, nrhs, seed):
    r = np.stack([meshgen.random_vector(n, seed + k) for k in range(nrhs)], axis=1)
    return torch.from_numpy(r).to("cuda:0").t().contiguous().t()   # column-major (n, nrhs)


def _allocations():
    return torch.cuda.memory_stats(0).get("allocation.all.allocated", 0)


def test_noalloc_apply_matches_apply_twice_second_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    big = meshgen.poisson_16()
    small = meshgen.small_elasticity_layers(8, 2, contrast=1e4)
    assert small.n_glob < big.n_glob
    for p, tau, nrhs, seed in ((big, None, 2, 11), (small, 10.0, 1, 23)):
        b = _factored(p, tau)
        r = _rhs(p.n_glob, nrhs, seed)
        z_ref = b.apply(r)
        torch.cuda.synchronize()
        z = torch.full_like(z_ref, float("nan"))
        before = _allocations()
        b.apply_noalloc(r, z)
        torch.cuda.synchronize()
        assert _allocations() == before
        assert torch.equal(z, z_ref), (p.name, float((z - z_ref).abs().max()))
        b.close()
