"""Pins of the oracle's interface classification, spaces and change of variables
against the numbers the paper prints and against exact algebraic identities."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen
from oracle.fem import Substructures
from oracle.interface import Interface
from oracle.cov import Constraints, GlobTransform
from oracle.bddc import CornerSpace, original_constraints, projection, Algorithm2

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def fig3():
    p = meshgen.cube_problem(meshgen.ELASTICITY, 8, 2, dirichlet_face=None)
    S = Substructures(p)
    itf = Interface(S)
    cons = Constraints(itf, "ce")
    cs = CornerSpace(S, itf)
    return p, S, itf, cons, cs


def _dbar(itf, cons, cs):
    rows, cols, vals = [], [], []
    nr = 0
    for gi, gl in enumerate(itf.globs):
        G = cons.G[gi]
        subs = sorted(gl["subs"])
        for k in range(G.m):
            idx = [cs.wc[s][itf.pos[s][gi][G.perm[k]]] for s in subs]
            for l in range(1, len(idx)):
                rows += [nr, nr]
                cols += [idx[0], idx[l]]
                vals += [1.0, -1.0]
                nr += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(nr, cs.n))


def test_fig3_counts(fig3):
    g = load("fig3_structure.json")
    p, S, itf, cons, cs = fig3
    c = itf.counts()
    assert c["corners"] == g["corners"]
    assert c["edges"] == g["edges"]
    assert c["faces"] == g["faces"]
    assert S.n_glob == g["dofs"]
    assert cons.Nc() == g["rows_D"]
    assert cs.n == g["size_Wc"]


def test_fig3_projection_nnz(fig3):
    g = load("fig3_structure.json")
    p, S, itf, cons, cs = fig3
    Dc = original_constraints(S, itf, cons, cs)
    assert Dc.shape[0] == g["rows_D"]
    assert projection(Dc).nnz == g["nnz_Pi"]
    Db = _dbar(itf, cons, cs)
    assert projection(Db).nnz == g["nnz_Pibar"]


def test_dbar_is_dc_times_T(fig3):
    # after the change of variables every row of D^c T has one +1 and one -1
    p, S, itf, cons, cs = fig3
    Dc = original_constraints(S, itf, cons, cs).toarray()
    T = sp.block_diag([cons.T_i(i) for i in range(S.n_sub)]).tocsr()
    Rc = cs.Rc
    # D^c T acting on W^c: W^c -> W (Rc) -> T on W -> back (T keeps corners)
    DT = Dc @ (Rc.T @ T @ Rc).toarray() / np.maximum(1.0, (Rc.T @ Rc).diagonal())
    DT[np.abs(DT) < 1e-12] = 0
    for row in DT:
        nz = row[row != 0]
        assert len(nz) == 2
        assert sorted(np.sign(nz)) == [-1.0, 1.0]
        assert abs(abs(nz[0]) - abs(nz[1])) < 1e-12


def test_worked_example_unit_average():
    g = load("worked_example.json")
    n = g["n"]
    G = GlobTransform(np.ones((1, n)))
    assert G.m == 1
    np.testing.assert_allclose(np.abs(G.U), g["U"])
    assert list(G.perm) == g["perm"]
    T = G.T * np.sign(G.U[0, 0])            # U = [1] up to the QR sign
    T[1:, 1:] = G.T[1:, 1:]
    np.testing.assert_allclose(T[0], g["T_first_row"], atol=1e-15)
    np.testing.assert_allclose(T[1:], np.hstack([np.zeros((n - 1, 1)), np.eye(n - 1)]))


def test_change_of_variables_inverse_and_averages():
    rng = np.random.default_rng(1)
    H = rng.standard_normal((3, 9))
    G = GlobTransform(H)
    Hfull = np.zeros((9, 9))
    Hfull[:3] = np.hstack([G.U, G.V])
    Hfull[3:, 3:] = np.eye(6)
    K = np.eye(9)[G.perm]                       # K w = w[perm]
    # new variable k is stored at position perm[k]: positional H = K^T H K
    Hpos = K.T @ Hfull @ K
    np.testing.assert_allclose(Hpos @ G.T, np.eye(9), atol=1e-12)
    # the explicit variables are Q^T (H^avg w)
    w = rng.standard_normal(9)
    y = Hfull @ K @ w
    np.testing.assert_allclose(G.Q @ y[:3], H @ w, atol=1e-12)


def test_drop_rule_removes_dependent_rows():
    rng = np.random.default_rng(2)
    H = rng.standard_normal((2, 7))
    H3 = np.vstack([H, H[0] + 2 * H[1]])
    G = GlobTransform(H3)
    assert G.m == 2 and G.dropped == 1


def test_E_is_projection_and_partition_of_unity():
    p = meshgen.small_elasticity_layers(6, 2, contrast=1e3)
    S = Substructures(p)
    itf = Interface(S)
    E = itf.E()
    R = S.R()
    np.testing.assert_allclose((E @ R).toarray(), np.eye(S.n_glob), atol=1e-14)
    RE = (R @ E).toarray()
    np.testing.assert_allclose(RE @ RE, RE, atol=1e-13)


def test_c1_structure():
    p = meshgen.poisson_16()
    S = Substructures(p)
    itf = Interface(S)
    cons = Constraints(itf, "ce")
    assert itf.counts() == dict(corners=6, edges=6, faces=12)
    assert cons.Nc() == 18
    assert all(gl["dofs"].size == 7 for gl in itf.globs if gl["kind"] == "edge")


def test_nc_convention_faces():
    # c+e+f adds one arithmetic average per component on every face shared by
    # two substructures: Nc(c+e+f) - Nc(c+e) = 3 * faces in the paper's tables
    g = load("nc_tables.json")
    for prob in g["problems"]:
        assert prob["Nc_cef"] - prob["Nc_ce"] == 3 * prob["faces"]
    p = meshgen.small_elasticity_layers(6, 2, contrast=1.0)
    S = Substructures(p)
    itf = Interface(S)
    ce, cef = Constraints(itf, "ce"), Constraints(itf, "cef")
    assert cef.Nc() - ce.Nc() == 3 * itf.counts()["faces"]


def test_kmeans_corner_augmentation_assumption2():
    p = meshgen.small_kmeans(meshgen.ELASTICITY, 10, 6)
    S = Substructures(p)
    itf = Interface(S)
    ns = itf.node_subs
    corners = set(itf.corner_nodes_all)
    from oracle.interface import _noncollinear_count
    for gi in itf.face_ids:
        i, j = itf.globs[gi]["subs"]
        pts = [p.xyz[n] for n, s in enumerate(ns) if i in s and j in s and n in corners]
        assert _noncollinear_count(pts) >= 3
