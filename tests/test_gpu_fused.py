"""The fused Cholesky against one launch per step, through the C ABI.

Every batched Cholesky of the library (the interior fronts, the pair-side
eliminations and reduced pair matrices of the adaptive selection, K_rr and the
coarse matrix) runs either as one fused launch whose tasks wait on per-entry
counters (``chol_launch=2``) or as one launch per step of the blocked
factorization (``chol_launch=1``); the default (0) picks per call by size.
All run the same tile code on the same data in the same per-entry order, so
the factor, and everything computed from it, is the same bit for bit: the
adaptive constraints (omega, Nc), the PCG history and the solution.  The
solution also matches the oracle's (1e-8).
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


def _run(BDDC, p, chol_launch, tau=None, prec=64, edges=False):
    b = BDDC(chol_launch=chol_launch, factor_precision=prec)
    b.setup(p, "ce", adaptive_edges=edges)
    ai = b.adapt(tau) if tau is not None else None
    b.factor()
    u, info = b.pcg_solve(torch.from_numpy(p.f))
    out = (u.cpu().numpy()[:, 0], info[0], ai, b.pcg_history().copy(), b.info().fp32_fallbacks)
    b.close()
    return out


CASES = [
    ("elast8_kmeans", lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3), None),
    ("elast8_kmeans_tau5", lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3), 5.0),
    ("elast12_kmeans_tau3", lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 12, 8, contrast=1e4), 3.0),
    ("poisson16", meshgen.poisson_16, None),
]


@pytest.mark.parametrize("name,make,tau", CASES, ids=[c[0] for c in CASES])
def test_fused_factor_bitwise_equals_step_launches(name, make, tau):
    BDDC = _gpu()
    p = make()
    uf, inf, af, hf, _ = _run(BDDC, p, 2, tau)
    us, ins, as_, hs, _ = _run(BDDC, p, 1, tau)
    ud, ind, _, _, _ = _run(BDDC, p, 0, tau)
    assert np.array_equal(uf, us), name
    assert np.array_equal(ud, us), name
    assert (inf.iters, inf.kappa, inf.relres, inf.true_relres) == (ins.iters, ins.kappa, ins.relres,
                                                                   ins.true_relres), name
    assert np.array_equal(hf, hs), name
    if tau is not None:
        assert (af.omega, af.nc, af.n_added) == (as_.omega, as_.nc, as_.n_added), name
    assert inf.converged, name


def test_fused_factor_matches_the_oracle():
    BDDC = _gpu()
    from oracle.solver import OracleBDDC
    from oracle.adapt import adapt
    p = meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3)
    o = OracleBDDC(p, "ce")
    ad = adapt(o.S, o.itf, o.cons, 5.0)
    ref = OracleBDDC(p, "ce", extra_rows=ad["rows"]).solve()
    u, info, ai, _, _ = _run(BDDC, p, 2, 5.0)
    err = np.abs(u - ref["u"]).max() / np.abs(ref["u"]).max()
    assert err < 1e-8, err


def test_fused_factor_fp32_bitwise_equals_step_launches():
    """FP32 local factors: the FP32 Cholesky of K_rr runs fused too."""
    BDDC = _gpu()
    p = meshgen.small_kmeans(meshgen.ELASTICITY, 12, 8, contrast=1e4)
    uf, inf, _, _, ff = _run(BDDC, p, 2, 3.0, prec=32)
    us, ins, _, _, fs = _run(BDDC, p, 1, 3.0, prec=32)
    assert np.array_equal(uf, us)
    assert inf.iters == ins.iters and ff == fs
