"""GEMM tile autotuning (bddc_options.autotune).

Every tile shape the tuner may pick accumulates each output entry over K in
the same order, and the trials restore the product's output before the final
launch, so a context with the tuner on must give the same bits as one with it
off: on the first call of each shape (trials run) and on later calls (the
table is used).  Tolerance 0.
"""
import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(BDDC, p, autotune):
    b = BDDC(autotune=autotune)
    b.setup(p, "ce")
    ai = b.adapt(10.0)
    b.factor()
    u, info = b.pcg_solve(torch.from_numpy(p.f))
    out = (u.cpu().numpy()[:, 0], ai.nc, ai.omega, info[0].iters, b.info().autotune_entries)
    b.close()
    return out


def test_autotune_same_bits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5863_amd import BDDC
    p = meshgen.small_elasticity_layers(12, 3, contrast=1e4)
    u0, nc0, om0, it0, _ = _run(BDDC, p, False)
    u1, nc1, om1, it1, n1 = _run(BDDC, p, True)    # tunes every new shape
    u2, nc2, om2, it2, n2 = _run(BDDC, p, True)    # uses the table
    assert n1 > 0 and n2 == n1
    assert (nc0, om0, it0) == (nc1, om1, it1) == (nc2, om2, it2)
    assert np.array_equal(u0, u1) and np.array_equal(u0, u2)
