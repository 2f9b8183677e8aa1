"""Parity at full size: the 48^3 layered elasticity workload (4 x 4 x 4
substructures of 12^3, adaptive tau = 10, edge parts of the adaptive rows
dropped) in the configuration ``bench.py --workload elasticity48`` times
(GEMM autotuner on), against the oracle's stored reference results for the
same mesh (``tests/golden/elasticity48.*``, Algorithm 2 by blocks and dense
pair eigensolves on every face; tolerances in ``fullsize_golden``):
- glob counts and Nc before and after adaptation;
- every face: eigenvalues, number selected, span of the rows;
- omega, PCG iterations and kappa, lambda_min >= 1;
- the solution element by element against the oracle's, and the true
  residual of the assembled system at most 1e-8 of r_0;
- the true residual again from the oracle's own assembled matrix;
- two solves give the same bits.
"""
import numpy as np
import pytest

import meshgen
import fullsize_golden as fg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_state = {}


def _run():
    if "b" in _state:
        return _state
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5863_amd import BDDC
    g, arrays = fg.load("elasticity48")
    p = meshgen.elasticity_layers_48()
    b = BDDC(autotune=True)
    b.setup(p, "ce")
    info0 = b.info()
    ai = b.adapt(g["tau"])
    b.factor()
    f = torch.from_numpy(p.f).to("cuda:0")
    u, pinfo = b.pcg_solve(f)
    u2, _ = b.pcg_solve(f)
    _state.update(g=g, arrays=arrays, p=p, b=b, info0=info0, ai=ai, u=u.cpu().numpy()[:, 0],
                  u2=u2.cpu().numpy()[:, 0], pinfo=pinfo[0])
    return _state


def test_fullsize_structure():
    st = _run()
    fg.check_structure(st["g"], st["info0"])
    assert st["info0"].n_glob == 345744


def test_fullsize_adaptive_selection():
    st = _run()
    errs = fg.check_adapt(st["g"], st["arrays"], st["ai"], st["b"])
    print(f"largest eigenvalue difference {errs.max():.2e} (relative)")


def test_fullsize_solution():
    st = _run()
    err = fg.check_solution(st["g"], st["arrays"], st["u"], st["pinfo"])
    pi = st["pinfo"]
    print(f"max-rel error {err:.2e}, iterations {pi.iters} (oracle {st['g']['pcg']['iters']}), "
          f"true residual {pi.true_relres:.2e} (floor {pi.residual_floor:.2e}), refinements {pi.refinements} "
          f"({pi.refine_iters} iterations)")
    assert np.array_equal(st["u"], st["u2"])


def test_fullsize_true_residual_from_the_oracle():
    """The oracle's assembled matrix: the residual of the GPU solution is at
    most 1e-8 of r_0 or twice eps || |K| |u| ||, the rounding scale of the
    product (which the oracle's own solution to 1e-11 also reaches)."""
    from oracle.fem import Substructures
    st = _run()
    K = Substructures(st["p"]).assembled()
    u = st["u"]
    r = np.linalg.norm(st["p"].f - K @ u)
    scale = np.finfo(float).eps * np.linalg.norm(abs(K) @ np.abs(u))
    print(f"true residual {r / st['g']['r0']:.2e} r0, rounding scale {scale / st['g']['r0']:.2e} r0")
    assert r <= max(1e-8 * st["g"]["r0"], 2.0 * scale), (r / st["g"]["r0"], scale / st["g"]["r0"])
