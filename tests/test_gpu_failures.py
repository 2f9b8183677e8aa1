"""Numerical and resource failures reported through the C ABI's status codes
(every kernel still exits normally: the conditions are data the host checks).

- BDDC_ERR_NOT_SPD: a substructure with negative coefficients makes its
  interior (Dirichlet) matrix indefinite; the factorization reports the
  substructure and the pivot.
- BDDC_ERR_NO_CONVERGENCE: PCG limited to two iterations stops short of the
  tolerance; the info record still holds the iterations and the residual.
- BDDC_ERR_OOM: a request whose footprint alone exceeds the server's
  admission budget is refused at submission.
- A context that failed can be set up again and solves normally.
"""
import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5863_amd import BDDC, BddcError, Server
    return BDDC, BddcError, Server


def test_negative_coefficient_is_not_spd():
    BDDC, BddcError, _ = _gpu()
    p = meshgen.poisson_16()
    bad = meshgen.poisson_16()
    bad.coef = p.coef.copy()
    bad.coef[p.elem_sub == 3] = -1.0
    b = BDDC()
    b.setup(bad, "ce")
    with pytest.raises(BddcError) as e:
        b.factor()
    assert e.value.code == 4
    assert "substructure 3" in str(e.value)
    # the same context accepts a valid problem afterwards
    b.setup(p, "ce")
    b.factor()
    u, info = b.pcg_solve(torch.from_numpy(p.f))
    assert info[0].converged
    b.close()


def test_iteration_limit_is_no_convergence():
    BDDC, BddcError, _ = _gpu()
    p = meshgen.small_elasticity_layers(6, 2, contrast=1e3)
    b = BDDC()
    b.setup(p, "ce")
    b.factor()
    f = torch.from_numpy(p.f)
    with pytest.raises(BddcError) as e:
        b.pcg_solve(f, maxit=2)
    assert e.value.code == 6
    u, info = b.pcg_solve(f, maxit=2, raise_on_fail=False)
    assert info[0].iters == 2 and not info[0].converged
    assert info[0].relres > 1e-8
    u, info = b.pcg_solve(f)
    assert info[0].converged and info[0].iters > 2
    b.close()


def test_request_above_the_budget_is_refused():
    _, BddcError, Server = _gpu()
    p = meshgen.poisson_16()
    srv = Server(max_active=1, hbm_budget_bytes=1e5)
    with pytest.raises(BddcError) as e:
        srv.submit(p, 0.0)
    assert e.value.code == 3
    srv.close()
    # with room for it the same request is served
    srv = Server(max_active=1)
    u, info = srv.wait(srv.submit(p, 0.0))
    assert info.state == 2 and info.pcg.converged
    assert np.all(np.isfinite(u))
    srv.close()
