"""Pins of the oracle's adaptive face constraints: reduction, Proposition 1,
compatibility Lemma, null-space inclusion, and the exactness of the pair
problem when there are only two substructures."""
import numpy as np
import pytest

import meshgen
from oracle.fem import Substructures
from oracle.interface import Interface
from oracle.cov import Constraints
from oracle.adapt import PairProblem, schur_dense, adapt
from oracle.bddc import Algorithm2
from oracle.solver import OracleBDDC


@pytest.fixture(scope="module")
def layered():
    p = meshgen.small_elasticity_layers(6, 2, contrast=1e4)
    S = Substructures(p)
    itf = Interface(S)
    cons = Constraints(itf, "ce")
    Sd = {s: schur_dense(S, itf, s) for s in range(S.n_sub)}
    return p, S, itf, cons, Sd


def test_reduced_equals_unreduced(layered):
    p, S, itf, cons, Sd = layered
    for fg in itf.face_ids[:4]:
        la, _ = PairProblem(S, itf, cons, fg, Sd, reduced=True).solve()
        lb, _ = PairProblem(S, itf, cons, fg, Sd, reduced=False).solve()
        top = 8
        np.testing.assert_allclose(la[-top:], lb[-top:], rtol=1e-8)


def test_eigenvalues_real_nonnegative_null_inclusion(layered):
    p, S, itf, cons, Sd = layered
    pp = PairProblem(S, itf, cons, itf.face_ids[0], Sd, reduced=False)
    lam, W = pp.solve()
    assert lam.min() > -1e-8 * lam.max()
    ev, V = np.linalg.eigh(pp.B)
    N = V[:, np.abs(ev) < 1e-10 * ev.max()]
    assert N.shape[1] > 0
    assert np.abs(pp.C @ N).max() < 1e-8 * np.abs(pp.C).max()


def test_proposition1_opposite_entries(layered):
    # d has matching entries of opposite sign on the two copies of every
    # shared interface dof
    p, S, itf, cons, Sd = layered
    pp = PairProblem(S, itf, cons, itf.face_ids[1], Sd, reduced=False)
    lam, W = pp.solve()
    d = pp.rows(W[:, -3:])
    a = pp.face_part(d, itf)
    b = pp.other_face_part(d, itf)
    np.testing.assert_allclose(a, -b, atol=1e-10 * np.abs(d).max())


def test_lemma_added_constraints_compatible(layered):
    # L(w) = 0 for every w continuous across the pair interface
    p, S, itf, cons, Sd = layered
    pp = PairProblem(S, itf, cons, itf.face_ids[2], Sd, reduced=False)
    lam, W = pp.solve()
    d = pp.rows(W[:, -4:])
    rng = np.random.default_rng(0)
    x = np.zeros(pp.n)
    vals = rng.standard_normal(S.n_glob)
    for s in (pp.i, pp.j):
        x[pp.col[s]] = vals[pp.side[s]["X"]]
    assert np.abs(d @ x).max() < 1e-9 * np.abs(d).max() * np.abs(x).sum()


def _two_substructures(contrast=1e3, kind=meshgen.ELASTICITY):
    nel = (8, 4, 4)
    coef = meshgen.coef_layers(nel, 1, values=(1.0, contrast))
    return meshgen.cube_problem(kind, nel, (2, 1, 1), coef=coef, dirichlet_face=("x", 0.0))


def _exact_lmax(o):
    """Largest eigenvalue of the preconditioned reduced operator, dense."""
    S, itf = o.S, o.itf
    harm = o.M.harm
    K = o.K.toarray()
    iface = np.flatnonzero(itf.mult > 1)
    n = iface.size
    Mmat = np.zeros((n, n))
    for k in range(n):
        r = np.zeros(S.n_glob)
        r[iface[k]] = 1.0
        Mmat[:, k] = o.M.apply(r)[iface]
    interior = np.flatnonzero(itf.mult == 1)
    KII = K[np.ix_(interior, interior)]
    Sch = K[np.ix_(iface, iface)] - K[np.ix_(iface, interior)] @ np.linalg.solve(
        KII, K[np.ix_(interior, iface)])
    ev = np.linalg.eigvals(Mmat @ Sch).real
    return ev.max(), ev.min()


@pytest.mark.parametrize("tau", [10.0, 3.0])
def test_two_substructures_corollary_exact(tau):
    # with two substructures the pair problem is the global problem: after
    # adding the eigenvectors with lambda >= tau the largest eigenvalue of the
    # preconditioned operator is the largest unselected one (Corollary)
    p = _two_substructures()
    o = OracleBDDC(p, "ce")
    lmax0, lmin0 = _exact_lmax(o)
    ad0 = adapt(o.S, o.itf, o.cons, np.inf)
    assert abs(lmax0 - ad0["omega"]) < 1e-7 * lmax0
    ad = adapt(o.S, o.itf, o.cons, tau)
    o2 = OracleBDDC(p, "ce", extra_face_rows=ad["rows"])
    lmax, lmin = _exact_lmax(o2)
    assert lmin > 1 - 1e-9
    assert abs(lmax - ad["omega"]) < 1e-7 * lmax
    out = o2.solve()
    assert out["kappa"] <= tau


def test_adaptivity_reduces_condition_number(layered):
    p, S, itf, cons, Sd = layered
    k0 = OracleBDDC(p, "ce").solve()
    ad = adapt(S, itf, cons, 10.0, Sd=Sd)
    o = OracleBDDC(p, "ce", extra_face_rows=ad["rows"])
    out = o.solve()
    assert out["kappa"] < k0["kappa"]
    assert out["kappa"] < 1.5 * 10.0
    assert out["Nc"] == o.cons.Nc() > 0
