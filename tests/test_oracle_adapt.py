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
    o2 = OracleBDDC(p, "ce", extra_rows=ad["rows"])
    lmax, lmin = _exact_lmax(o2)
    assert lmin > 1 - 1e-9
    assert abs(lmax - ad["omega"]) < 1e-7 * lmax
    out = o2.solve()
    assert out["kappa"] <= tau


def test_adaptivity_reduces_condition_number(layered):
    p, S, itf, cons, Sd = layered
    k0 = OracleBDDC(p, "ce").solve()
    ad = adapt(S, itf, cons, 10.0, Sd=Sd)
    o = OracleBDDC(p, "ce", extra_rows=ad["rows"])
    out = o.solve()
    assert out["kappa"] < k0["kappa"]
    assert out["kappa"] < 1.5 * 10.0
    assert out["Nc"] == o.cons.Nc() > 0


@pytest.mark.parametrize("case", ["layers", "kmeans"])
def test_kept_edge_rows_bound_every_pair_problem(case, layered):
    """Sec. 3 after Proposition 1: splitting each row d into its face part and
    one row per edge of the face's closure gives constraints at least as
    strong as d itself, so every pair problem re-solved on the new constraint
    set has its largest eigenvalue at most the largest unselected one
    (Corollary with eq. (complement)); hence omega~ <= tau.  Dropping the
    edge rows (Remark after Proposition 1) loses this: on the layered mesh a
    re-solved pair exceeds the indicator."""
    if case == "layers":
        p, S, itf, cons, Sd = layered
        tau = 10.0
    else:
        p = meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3)
        S = Substructures(p)
        itf = Interface(S)
        cons = Constraints(itf, "ce")
        Sd = {s: schur_dense(S, itf, s) for s in range(S.n_sub)}
        tau = 5.0
    ad = adapt(S, itf, cons, tau, Sd=Sd, edges=True)
    edge_rows = [g for g in ad["rows"] if itf.globs[g]["kind"] == "edge"]
    assert edge_rows
    again = adapt(S, itf, Constraints(itf, "ce", ad["rows"]), np.inf, Sd=Sd)
    assert again["omega"] <= ad["omega"] * (1 + 1e-8) < tau
    if case == "layers":
        ad0 = adapt(S, itf, cons, tau, Sd=Sd)
        assert ad0["omega"] == ad["omega"]
        again0 = adapt(S, itf, Constraints(itf, "ce", ad0["rows"]), np.inf, Sd=Sd)
        assert again0["omega"] > 1.1 * ad0["omega"]


def test_kept_edge_rows_are_split_parts_of_d(layered):
    """Each kept edge row is, up to scale, the part of a face row's d on one
    edge of the closure, and the corresponding face row the part on the face:
    together with zero corner entries they reassemble d (Proposition 1 gives
    the other side's copy as the negative)."""
    p, S, itf, cons, Sd = layered
    fg = itf.face_ids[0]
    from oracle.adapt import PairProblem
    pp = PairProblem(S, itf, cons, fg, Sd)
    lam, W = pp.solve()
    d = pp.rows(W[:, -1:])
    parts = pp.edge_parts(d, itf)
    assert parts
    globs = [(fg, pp.face_part(d, itf))] + parts
    rebuilt = np.zeros_like(d)
    for s, sign in ((pp.i, 1.0), (pp.j, -1.0)):
        m = {g: k for k, g in enumerate(pp.side[s]["X"])}
        for gi, part in globs:
            c = [pp.col[s][m[g]] for g in itf.globs[gi]["dofs"]]
            rebuilt[:, c] = sign * part
    np.testing.assert_allclose(rebuilt, d, rtol=0, atol=1e-10 * np.abs(d).max())


def test_three_eigenvectors_match_face_average_count(layered):
    """Sec. 7: three dominant eigenvectors per face give as many constraints
    as the arithmetic face averages (three per face in elasticity)."""
    p, S, itf, cons, Sd = layered
    ad = adapt(S, itf, cons, np.inf, Sd=Sd, count=3)
    assert all(k == 3 for k in ad["k"].values())
    c3 = Constraints(itf, "ce", ad["rows"])
    assert c3.Nc() == Constraints(itf, "cef").Nc() == cons.Nc() + 3 * len(itf.face_ids)
    # the indicator is the fourth eigenvalue, maximized over faces
    assert ad["omega"] == max(l[3] for l in ad["lam"].values())


def test_two_substructures_corollary_count():
    """With two substructures and the k dominant eigenvectors added, the
    largest eigenvalue of the preconditioned operator is lambda_{k+1}."""
    p = _two_substructures()
    o = OracleBDDC(p, "ce")
    ad = adapt(o.S, o.itf, o.cons, np.inf, count=3)
    o2 = OracleBDDC(p, "ce", extra_rows=ad["rows"])
    lmax, lmin = _exact_lmax(o2)
    lam = ad["lam"][o.itf.face_ids[0]]
    assert abs(lmax - lam[3]) < 1e-7 * lmax
    assert lmin > 1 - 1e-9
