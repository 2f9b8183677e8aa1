"""Several right-hand sides at once, through the C ABI.

bddc_apply and bddc_pcg_solve take up to 8 columns per block: every factor is
read once per application for the whole block, and the block PCG runs its
columns in lock step with their own scalars and stop tests.  Each column's
arithmetic is the same for every block width, so
- a column of a block apply has the bits of the same column applied alone,
  and matches the oracle element by element;
- a column of a block solve has the bits (solution, iterations, residual
  history, kappa) of the same load solved alone, including loads that
  converge at different iterations, a zero load and columns past the block
  width (nrhs = 11 runs as 8 + 3);
- every column matches the oracle's solution of its load to 1e-8.
"""
import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5863_amd import BDDC
    return BDDC


_cache = {}


def _problem():
    if "p" not in _cache:
        from oracle.solver import OracleBDDC
        p = meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3)
        _cache["p"] = p
        _cache["o"] = OracleBDDC(p, "ce")
    return _cache["p"], _cache["o"]


def _loads(p, k, seed=0):
    """k loads: the mesh's own, scaled and random ones, and one zero column."""
    rng = np.random.default_rng(seed)
    F = np.empty((p.n_glob, k))
    for j in range(k):
        if j == 0:
            F[:, j] = p.f
        elif j == 2:
            F[:, j] = 0.0
        elif j % 3 == 1:
            F[:, j] = (1.0 + j) * p.f + 1e-3 * rng.standard_normal(p.n_glob)
        else:
            F[:, j] = rng.standard_normal(p.n_glob)
    return F


def maxrel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("nrhs", [2, 3, 8, 11])
def test_block_apply_bits_and_oracle(nrhs):
    BDDC = _gpu()
    p, o = _problem()
    b = BDDC()
    b.setup(p, "ce")
    b.factor()
    R = np.stack([meshgen.random_vector(p.n_glob, 100 + j) for j in range(nrhs)], axis=1)
    Z = b.apply(torch.from_numpy(R)).cpu().numpy()
    for j in range(nrhs):
        z1 = b.apply(torch.from_numpy(R[:, j].copy())).cpu().numpy()[:, 0]
        assert np.array_equal(Z[:, j], z1), (nrhs, j)
        zr = o.apply(R[:, j])
        assert maxrel(Z[:, j], zr) < 1e-9, (nrhs, j, maxrel(Z[:, j], zr))
    b.close()


def _block_vs_single(b, F):
    u_blk, info_blk = b.pcg_solve(torch.from_numpy(F))
    u_blk = u_blk.cpu().numpy()
    for j in range(F.shape[1]):
        u1, i1 = b.pcg_solve(torch.from_numpy(F[:, j].copy()))
        h1 = b.pcg_history()
        u1 = u1.cpu().numpy()[:, 0]
        ib, is_ = info_blk[j], i1[0]
        assert np.array_equal(u_blk[:, j], u1), j
        assert (ib.iters, ib.converged, ib.refinements) == (is_.iters, is_.converged, is_.refinements), j
        assert ib.relres == is_.relres and ib.kappa == is_.kappa or (ib.iters == 0 and is_.iters == 0), j
        assert ib.true_relres == is_.true_relres, j
        if j == 0:
            assert np.array_equal(b.pcg_history(), h1)
    return u_blk, info_blk


@pytest.mark.parametrize("nrhs", [5, 11])
def test_block_pcg_bits_and_oracle(nrhs):
    BDDC = _gpu()
    p, o = _problem()
    b = BDDC()
    b.setup(p, "ce")
    b.factor()
    F = _loads(p, nrhs)
    U, infos = _block_vs_single(b, F)
    iters = [i.iters for i in infos]
    assert infos[2].iters == 0 and infos[2].converged and not U[:, 2].any()
    assert len(set(i for k, i in enumerate(iters) if k != 2)) >= 2, iters  # columns stop apart
    for j in (0, 1, 3, nrhs - 1):
        ref = o.solve(F[:, j])
        assert np.linalg.norm(U[:, j] - ref["u"]) / np.linalg.norm(ref["u"]) < 1e-8, j
        assert maxrel(U[:, j], ref["u"]) < 1e-8, j
    b.close()


def test_block_pcg_fp32_and_adaptive():
    """FP32 local factors (flexible beta) and adaptive constraints: block
    columns keep the bits of single solves; the adaptive solution of the
    mesh's load matches the oracle's."""
    BDDC = _gpu()
    from oracle.solver import OracleBDDC
    from oracle.adapt import adapt
    p, o = _problem()
    ad = adapt(o.S, o.itf, o.cons, 5.0)
    ref = OracleBDDC(p, "ce", extra_rows=ad["rows"]).solve()
    for prec in (64, 32):
        b = BDDC(factor_precision=prec)
        b.setup(p, "ce")
        b.adapt(5.0)
        b.factor()
        F = _loads(p, 4, seed=1)
        U, infos = _block_vs_single(b, F)
        assert np.linalg.norm(U[:, 0] - ref["u"]) / np.linalg.norm(ref["u"]) < 1e-8, prec
        b.close()


def test_block_pcg_per_substructure_launches():
    """The unbatched launch mode also runs blocks: its columns match its own
    single solves bit for bit and the batched mode's to rounding."""
    BDDC = _gpu()
    p, _ = _problem()
    F = _loads(p, 3, seed=2)
    b = BDDC(per_substructure_launches=True)
    b.setup(p, "ce")
    b.factor()
    U, _ = _block_vs_single(b, F)
    b.close()
    b = BDDC()
    b.setup(p, "ce")
    b.factor()
    U2, _ = b.pcg_solve(torch.from_numpy(F))
    U2 = U2.cpu().numpy()
    for j in range(3):
        if j != 2:
            assert maxrel(U[:, j], U2[:, j]) < 1e-10, j
    b.close()


def test_block_pcg_no_convergence_reports_every_column():
    BDDC = _gpu()
    p, _ = _problem()
    b = BDDC()
    b.setup(p, "ce")
    b.factor()
    F = _loads(p, 4, seed=3)
    U, infos = b.pcg_solve(torch.from_numpy(F), maxit=3, raise_on_fail=False)
    assert [i.iters for i in infos] == [3, 3, 0, 3]
    assert [bool(i.converged) for i in infos] == [False, False, True, False]
    b.close()
