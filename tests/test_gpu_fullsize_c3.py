"""Parity at the 64^3 k-means size, the workload ``bench.py`` times by
default: 3D elasticity on 64^3 elements split by seeded k-means into 64
uneven substructures, 5% of the elements at E = 1e5, adaptive tau = 10 with
the adaptive edge rows kept (Sec. 3 after Proposition 1), GEMM autotuner on;
against the oracle's stored reference results for the same mesh
(``tests/golden/kmeans64.*``; tolerances in ``fullsize_golden``):
- glob counts and Nc before and after adaptation, edge rows per edge;
- every face: eigenvalues, number selected, span of the face rows;
- omega, PCG iterations and kappa, lambda_min >= 1;
- the solution element by element, the true residual of the assembled
  system at most 1e-8 of r_0, and two solves give the same bits;
- with the FP32 local factor (factor_precision = 32), the same solution
  tolerance: the outer FP64 PCG and its true-residual check recover the
  accuracy; the error against the oracle is printed.  Its preconditioner is
  not the oracle's (FP32 factors), so its iterations are only printed;
- every batched Cholesky run one launch per step, or fused into one launch
  per factorization: the same bits as the default.
"""
import numpy as np
import pytest

import meshgen
import fullsize_golden as fg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_state = {}
LAM_TOL = 1e-6


def _run():
    if 64 in _state:
        return _state
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5863_amd import BDDC
    g, arrays = fg.load("kmeans64")
    p = meshgen.elasticity_kmeans_64()
    f = torch.from_numpy(p.f).to("cuda:0")
    _state.update(g=g, arrays=arrays, p=p)
    for prec in (64, 32):
        b = BDDC(factor_precision=prec, autotune=True)
        b.setup(p, "ce", adaptive_edges=True)
        info0 = b.info()
        ai = b.adapt(g["tau"])
        b.factor()
        u, pinfo = b.pcg_solve(f)
        res = dict(info0=info0, ai=ai, u=u.cpu().numpy()[:, 0], pinfo=pinfo[0])
        if prec == 64:
            res["adapt_errs"] = fg.check_adapt(g, arrays, ai, b, lam_tol=LAM_TOL, span_tol=LAM_TOL)
            fg.check_edge_rows(g, b)
            u2, _ = b.pcg_solve(f)
            res["u2"] = u2.cpu().numpy()[:, 0]
        b.close()
        del b, u
        torch.cuda.empty_cache()
        _state[prec] = res
    return _state


def test_c3_structure():
    st = _run()
    fg.check_structure(st["g"], st[64]["info0"])
    assert st[64]["info0"].n_glob == 811200


def test_c3_adaptive_selection():
    st = _run()
    e = st[64]["adapt_errs"]
    print(f"eigenvalue differences (relative): max {e.max():.2e}, median {np.median(e):.2e}")
    assert st[64]["ai"].n_added_edge == sum(st["g"]["edge_rows"].values())


@pytest.mark.parametrize("prec", [64, 32])
def test_c3_solution(prec):
    st = _run()
    pi = st[prec]["pinfo"]
    err = fg.check_solution(st["g"], st["arrays"], st[prec]["u"], pi, same_preconditioner=prec == 64)
    print(f"fp{prec}: max-rel error {err:.2e}, iterations {pi.iters} "
          f"(oracle {st['g']['pcg']['iters']}), true residual {pi.true_relres:.2e}, "
          f"refinements {pi.refinements} ({pi.refine_iters} iterations)")
    if prec == 64:
        assert np.array_equal(st[64]["u"], st[64]["u2"])


def test_c3_fp32_fallback_keeps_k_rr():
    """tau = 2 with FP32 local factors: at this size one substructure's FP32
    factorization meets a non-positive pivot and is factored again in FP64.
    The coarse matrix is the Galerkin product of the basis with the unfactored
    K_rr, so the fallback must leave K_rr in place (built from the factor it
    was indefinite: no coarse factorization).  The FP32 solve then converges
    and matches the FP64 solve of the same constraints element-wise to 1e-8.
    (Its preconditioner is inexact, so the bound lambda_min >= 1 of the exact
    one does not apply: measured 0.047.)"""
    st = _run()
    from paper_0910_5863_amd import BDDC
    p = st["p"]
    f = torch.from_numpy(p.f).to("cuda:0")
    out = {}
    for prec in (64, 32):
        b = BDDC(factor_precision=prec, autotune=True)
        b.setup(p, "ce", adaptive_edges=True)
        b.adapt(2.0)
        b.factor()
        u, pinfo = b.pcg_solve(f)
        out[prec] = (u.cpu().numpy()[:, 0], pinfo[0], b.info().fp32_fallbacks)
        b.close()
        del b, u
        torch.cuda.empty_cache()
    (u64, i64, _), (u32, i32, nfb) = out[64], out[32]
    print(f"fp32 at tau 2: {nfb} fallback(s), iterations {i32.iters} (fp64 {i64.iters}), "
          f"lambda_min {i32.lmin:.6f}")
    assert nfb >= 1
    assert i32.converged and i64.converged
    err = float(np.abs(u32 - u64).max() / np.abs(u64).max())
    print(f"fp32 against fp64 at tau 2: max-rel difference {err:.2e}")
    assert err < 1e-8, err


@pytest.mark.parametrize("chol_launch", [1, 2])
def test_c3_cholesky_launch_modes_bitwise(chol_launch):
    """Every batched Cholesky of the step (interior fronts, pair eliminations,
    K_rr, the coarse matrix) one launch per step (1) or fused into one launch
    per factorization (2): the solution has the bits of the default run (0,
    which fuses the smaller batches), as do omega, Nc and the iterations."""
    st = _run()
    from paper_0910_5863_amd import BDDC
    g, p = st["g"], st["p"]
    b = BDDC(autotune=True, chol_launch=chol_launch)
    b.setup(p, "ce", adaptive_edges=True)
    ai = b.adapt(g["tau"])
    b.factor()
    u, pinfo = b.pcg_solve(torch.from_numpy(p.f).to("cuda:0"))
    u = u.cpu().numpy()[:, 0]
    b.close()
    torch.cuda.empty_cache()
    ref = st[64]
    assert (ai.omega, ai.nc) == (ref["ai"].omega, ref["ai"].nc)
    assert pinfo[0].iters == ref["pinfo"].iters
    assert np.array_equal(u, ref["u"])
