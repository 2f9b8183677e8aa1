"""Pins of the oracle's preconditioner and PCG: the three equivalent forms,
t-independence, the spectrum bound, exactness and agreement with a direct
solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import meshgen
from oracle.fem import Substructures
from oracle.interface import Interface
from oracle.cov import Constraints
from oracle.bddc import Algorithm2, Lemma1KKT, ProjectedOriginal
from oracle.solver import OracleBDDC, direct_solve
from oracle.pcg import pcg, lanczos_extremes


@pytest.fixture(scope="module")
def small():
    p = meshgen.small_elasticity_layers(6, 2, contrast=1e3)
    S = Substructures(p)
    itf = Interface(S)
    cons = Constraints(itf, "ce")
    return p, S, itf, cons, Algorithm2(S, itf, cons)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_algorithm2_equals_lemma1_and_projection(small):
    p, S, itf, cons, a2 = small
    r = a2.harm.apply_T(meshgen.random_vector(S.n_glob, 0))
    z = a2.apply(r)
    assert rel(z, Lemma1KKT(a2).apply(r)) < 1e-10
    assert rel(z, ProjectedOriginal(a2).apply(r)) < 1e-10


def test_t_independence(small):
    p, S, itf, cons, a2 = small
    r = a2.harm.apply_T(meshgen.random_vector(S.n_glob, 1))
    for t in (1e-3, 7.0, 1e4):
        assert rel(Algorithm2(S, itf, cons, t=t).apply(r), a2.apply(r)) < 1e-10


def test_corners_only_special_case():
    # D^c empty: M = (I-P) E R^c (A^c)^{-1} R^cT E^T (I-P)^T  (eq. (BDDC-simple))
    p = meshgen.small_elasticity_layers(6, 2, contrast=10.0)
    S = Substructures(p)
    itf = Interface(S)
    cons = Constraints(itf, "c")
    a2 = Algorithm2(S, itf, cons)
    assert a2.Dbar.shape[0] == 0
    Ac = (a2.cs.Rc.T @ a2.A @ a2.cs.Rc).tocsc()
    r = a2.harm.apply_T(meshgen.random_vector(S.n_glob, 2))
    w = spla.spsolve(Ac, a2.cs.Rc.T @ (a2.E.T @ r))
    z = a2.harm.apply(a2.E @ (a2.cs.Rc @ w))
    assert rel(a2.apply(r), z) < 1e-10


def test_preconditioner_symmetric_positive(small):
    p, S, itf, cons, a2 = small
    r1 = a2.harm.apply_T(meshgen.random_vector(S.n_glob, 3))
    r2 = a2.harm.apply_T(meshgen.random_vector(S.n_glob, 4))
    a, b = r2 @ a2.apply(r1), r1 @ a2.apply(r2)
    assert abs(a - b) < 1e-10 * abs(a)
    assert r1 @ a2.apply(r1) > 0


def test_pcg_matches_direct_c1():
    p = meshgen.poisson_16()
    o = OracleBDDC(p, "ce")
    out = o.solve(rtol=1e-13)
    ud = direct_solve(p)
    assert rel(out["u"], ud) < 1e-10
    out8 = o.solve()
    assert out8["relres"] <= 1e-8
    assert out8["lmin"] >= 1 - 1e-10                 # Theorem 1


@pytest.mark.parametrize("mode", ["c", "ce", "cef"])
def test_spectrum_bound_and_direct_elasticity(mode):
    p = meshgen.small_elasticity_layers(6, 2, contrast=1e2)
    o = OracleBDDC(p, mode)
    out = o.solve(rtol=1e-12)
    assert out["lmin"] >= 1 - 1e-10
    assert rel(out["u"], direct_solve(p)) < 1e-9


def test_more_constraints_better_conditioning():
    p = meshgen.small_elasticity_layers(6, 2, contrast=1e3)
    k = [OracleBDDC(p, m).solve()["kappa"] for m in ("c", "ce", "cef")]
    assert k[0] >= k[1] >= k[2] * (1 - 1e-8)


def test_exact_when_every_interface_dof_constrained():
    # H^avg = I on every glob: the constrained space is U and BDDC is exact
    p = meshgen.small_elasticity_layers(6, 2, contrast=1e3)
    o = OracleBDDC(p, "all")
    out = o.solve()
    assert out["iters"] == 1
    assert abs(out["kappa"] - 1.0) < 1e-10


def test_lanczos_recovers_known_spectrum():
    ev = np.array([1.0, 2.0, 3.5, 7.0, 11.0])
    A = np.diag(ev)
    f = np.ones(5)
    out = pcg(lambda v: A @ v, f, lambda v: v.copy(), np.zeros(5), rtol=1e-14)
    lmin, lmax = lanczos_extremes(out["alphas"], out["betas"])
    assert abs(lmin - 1.0) < 1e-10 and abs(lmax - 11.0) < 1e-10
