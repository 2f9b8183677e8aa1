"""GPU parity of the adaptive face constraints (Algorithm 1) against the
oracle's dense factor-space eigensolves of eq. (eig-matrix).

The device reduces each pair problem exactly (jump space, parallel sum) and
runs batched LOBPCG to a relative residual of 1e-8, so eigenvalues agree to
about 1e-10 relative when they are separated; 1e-6 is asserted.  Selected rows
are compared as subspaces (eigenvectors of repeated eigenvalues are not
unique): principal-angle cosines within 1e-6 of one.
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


CASES = {
    "layers8": (lambda: meshgen.small_elasticity_layers(8, 2, contrast=1e4), 10.0),
    "layers6x3": (lambda: meshgen.small_elasticity_layers(6, 3, contrast=1e5), 10.0),
    "kmeans_elast": (lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3), 5.0),
    "kmeans_poisson": (lambda: meshgen.small_kmeans(meshgen.POISSON, 10, 5), 2.0),
}

_cache = {}


def oracle_for(name):
    if name not in _cache:
        from oracle.solver import OracleBDDC
        from oracle.adapt import adapt, schur_dense
        make, tau = CASES[name]
        p = make()
        o = OracleBDDC(p, "ce")
        Sd = {s: schur_dense(o.S, o.itf, s) for s in range(o.S.n_sub)}
        ad = adapt(o.S, o.itf, o.cons, tau, Sd=Sd)
        o2 = OracleBDDC(p, "ce", extra_rows=ad["rows"])
        _cache[name] = (p, tau, o, ad, o2)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_adapt_eigenvalues_rows_and_solve(name):
    BDDC = _gpu()
    p, tau, o, ad, o2 = oracle_for(name)
    b = BDDC()
    b.setup(p, "ce")
    info = b.adapt(tau)
    assert info.unconverged == 0
    assert info.nc == o2.cons.Nc()
    assert abs(info.omega - ad["omega"]) <= 1e-6 * max(1.0, ad["omega"])
    faces = o.itf.face_ids
    for f, gi in enumerate(faces):
        lam_ref = ad["lam"][gi]                      # descending, all eigenvalues
        lam = b.face_eigs(f)
        k = int(np.sum(lam_ref >= tau))
        m = min(len(lam), k + 1)
        np.testing.assert_allclose(lam[:m], lam_ref[:m], rtol=1e-6)
        rows, dofs, subs = b.face_rows(f)
        assert np.array_equal(dofs, o.itf.globs[gi]["dofs"])
        assert rows.shape[0] == k
        if k:
            ref = ad["rows"][gi]
            qa, _ = np.linalg.qr(rows.T)
            qb, _ = np.linalg.qr(ref.T)
            cos = np.linalg.svd(qa.T @ qb)[1]
            assert cos.min() > 1 - 1e-6, (f, cos)
    b.factor()
    u, pinfo = b.pcg_solve(torch.from_numpy(p.f))
    ref = o2.solve()
    uu = u.cpu().numpy()[:, 0]
    assert np.linalg.norm(uu - ref["u"]) / np.linalg.norm(ref["u"]) < 1e-8
    assert abs(pinfo[0].iters - ref["iters"]) <= max(2, int(0.05 * ref["iters"]))
    b.close()


def test_adapt_replaces_rows_and_reuses_schur():
    """A second bddc_adapt replaces the rows of the first: adapting at tau = 2
    and then at tau = 10 gives the constraints, indicator and solution of a
    single adaptation at tau = 10 on a fresh context."""
    BDDC = _gpu()
    p, tau, o, ad, o2 = oracle_for("layers8")
    ref = BDDC()
    ref.setup(p, "ce")
    i_ref = ref.adapt(tau)
    ref.factor()
    f = torch.from_numpy(p.f)
    u_ref, _ = ref.pcg_solve(f)
    b = BDDC()
    b.setup(p, "ce")
    i2 = b.adapt(2.0)
    assert i2.nc > i_ref.nc
    i10 = b.adapt(tau)
    assert i10.nc == i_ref.nc == o2.cons.Nc()
    assert i10.omega == i_ref.omega
    b.factor()
    u, info = b.pcg_solve(f)
    assert info[0].iters > 0
    assert torch.equal(u.cpu(), u_ref.cpu())
    # a second factor recomputes the Schur complements it consumed
    b.factor()
    u2, _ = b.pcg_solve(f)
    assert torch.equal(u2.cpu(), u_ref.cpu())


def _same_span(a, b, tol=1e-6):
    """Row spaces of a and b agree: equal numerical rank (singular values
    above tol of the largest) and principal-angle cosines within tol of one."""
    sa, va = np.linalg.svd(a)[1:]
    sb, vb = np.linalg.svd(b)[1:]
    ra, rb = int(np.sum(sa > tol * sa[0])), int(np.sum(sb > tol * sb[0]))
    assert ra == rb, (sa / sa[0], sb / sb[0])
    cos = np.linalg.svd(va[:ra] @ vb[:rb].T)[1]
    assert cos.min() > 1 - tol, cos


EDGE_CASES = {
    "layers6x2": (lambda: meshgen.small_elasticity_layers(6, 2, contrast=1e4), 10.0),
    "kmeans_elast": (lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3), 5.0),
}


@pytest.mark.parametrize("name", list(EDGE_CASES))
def test_adapt_keeps_edge_rows(name):
    """adaptive_edges: every selected row is split into a face row and one
    row per edge of the face's closure (Sec. 3 after Proposition 1).  The
    edge rows, Nc, omega and the solution match the oracle's; edge rows are
    compared per edge as row spaces, since eigenvectors of repeated
    eigenvalues, and hence their rows, are not unique."""
    BDDC = _gpu()
    from oracle.solver import OracleBDDC
    from oracle.adapt import adapt, schur_dense
    make, tau = EDGE_CASES[name]
    p = make()
    o = OracleBDDC(p, "ce")
    Sd = {s: schur_dense(o.S, o.itf, s) for s in range(o.S.n_sub)}
    ad = adapt(o.S, o.itf, o.cons, tau, Sd=Sd, edges=True)
    o2 = OracleBDDC(p, "ce", extra_rows=ad["rows"])
    b = BDDC()
    b.setup(p, "ce", adaptive_edges=True)
    info = b.adapt(tau)
    assert info.unconverged == 0
    assert abs(info.omega - ad["omega"]) <= 1e-6 * max(1.0, ad["omega"])
    n_edge_rows = sum(len(r) for g, r in ad["rows"].items() if o.itf.globs[g]["kind"] == "edge")
    assert n_edge_rows > 0 and info.n_added_edge == n_edge_rows
    assert info.nc == o2.cons.Nc()
    for e, gi in enumerate(o.itf.edge_ids):
        rows, dofs = b.edge_rows(e)
        assert np.array_equal(dofs, o.itf.globs[gi]["dofs"])
        ref = ad["rows"].get(gi)
        assert rows.shape[0] == (0 if ref is None else len(ref))
        if rows.shape[0]:
            _same_span(rows, ref)
    for f, gi in enumerate(o.itf.face_ids):
        rows, _, _ = b.face_rows(f)
        ref = ad["rows"].get(gi)
        assert rows.shape[0] == (0 if ref is None else len(ref))
        if rows.shape[0]:
            _same_span(rows, ref)
    b.factor()
    u, pinfo = b.pcg_solve(torch.from_numpy(p.f))
    ref = o2.solve()
    uu = u.cpu().numpy()[:, 0]
    assert np.linalg.norm(uu - ref["u"]) / np.linalg.norm(ref["u"]) < 1e-8
    assert abs(pinfo[0].iters - ref["iters"]) <= 2
    b.close()


@pytest.mark.parametrize("name", ["layers8", "kmeans_poisson"])
def test_adapt_three_dominant_eigenvectors(name):
    """bddc_adapt_count(3), the "3eigv" variant of Sec. 7: three rows per
    face from the dominant eigenvectors whatever their eigenvalues; Nc, the
    indicator (the largest fourth eigenvalue), the rows and the solution
    match the oracle's count mode."""
    BDDC = _gpu()
    from oracle.solver import OracleBDDC
    from oracle.adapt import adapt, schur_dense
    make, _ = CASES[name]
    p = make()
    o = OracleBDDC(p, "ce")
    Sd = {s: schur_dense(o.S, o.itf, s) for s in range(o.S.n_sub)}
    ad = adapt(o.S, o.itf, o.cons, np.inf, Sd=Sd, count=3)
    o2 = OracleBDDC(p, "ce", extra_rows=ad["rows"])
    b = BDDC()
    b.setup(p, "ce")
    info = b.adapt_count(3)
    assert info.unconverged == 0
    assert info.n_added == 3 * len(o.itf.face_ids)
    assert info.nc == o2.cons.Nc()
    assert abs(info.omega - ad["omega"]) <= 1e-6 * max(1.0, ad["omega"])
    for f, gi in enumerate(o.itf.face_ids):
        lam_ref = ad["lam"][gi]
        np.testing.assert_allclose(b.face_eigs(f)[:4], lam_ref[:4], rtol=1e-6)
        rows, _, _ = b.face_rows(f)
        assert rows.shape[0] == 3
        _same_span(rows, ad["rows"][gi])
    b.factor()
    u, pinfo = b.pcg_solve(torch.from_numpy(p.f))
    ref = o2.solve()
    uu = u.cpu().numpy()[:, 0]
    assert np.linalg.norm(uu - ref["u"]) / np.linalg.norm(ref["u"]) < 1e-8
    assert abs(pinfo[0].iters - ref["iters"]) <= 2
    b.close()
