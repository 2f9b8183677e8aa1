"""Pins of the oracle's finite element layer against closed forms and invariants."""
import numpy as np
import pytest

import meshgen
from oracle.fem import element_matrices, Substructures, elasticity_D


def unit_cube():
    xyz, hex8 = meshgen.grid_mesh(1, 1, 1)
    return xyz, hex8


def test_poisson_unit_cube_closed_form():
    # Q1 Laplacian on the unit cube: diagonal 1/3, edge neighbours 0,
    # face diagonals -1/12, body diagonal -1/12 (exact integration).
    xyz, hex8 = unit_cube()
    K = element_matrices(xyz, hex8, np.array([1.0]), 0, 0.0)[0]
    off = meshgen.HEX_OFFSETS
    for a in range(8):
        for b in range(8):
            nd = int(np.abs(off[a] - off[b]).sum())
            expect = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[nd]
            assert K[a, b] == pytest.approx(expect, abs=1e-15)


def test_poisson_scaling_with_h_and_k():
    xyz, hex8 = meshgen.grid_mesh(4, 4, 4)      # h = 1/4
    K = element_matrices(xyz, hex8[:1], np.array([3.0]), 0, 0.0)[0]
    xyz1, hex1 = unit_cube()
    K1 = element_matrices(xyz1, hex1, np.array([1.0]), 0, 0.0)[0]
    np.testing.assert_allclose(K, 3.0 * 0.25 * K1, rtol=1e-14, atol=1e-16)


def rigid_modes(X):
    n = X.shape[0]
    Rm = np.zeros((3 * n, 6))
    for a in range(n):
        x, y, z = X[a]
        Rm[3 * a:3 * a + 3, :3] = np.eye(3)
        Rm[3 * a:3 * a + 3, 3] = [0, -z, y]
        Rm[3 * a:3 * a + 3, 4] = [z, 0, -x]
        Rm[3 * a:3 * a + 3, 5] = [-y, x, 0]
    return Rm


def test_elasticity_element_rigid_null_space():
    xyz, hex8 = unit_cube()
    K = element_matrices(xyz, hex8, np.array([2.5]), 1, 0.3)[0]
    np.testing.assert_allclose(K, K.T, atol=1e-14)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 6
    assert ev.min() > -1e-12
    Rm = rigid_modes(xyz[hex8[0]])
    assert np.abs(K @ Rm).max() < 1e-12


def test_elasticity_D_matrix_uniaxial_strain():
    # uniaxial strain e_xx = 1: sigma_xx = lambda + 2 mu, sigma_yy = lambda
    E, nu = 2.0, 0.25
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    s = elasticity_D(E, nu) @ np.array([1.0, 0, 0, 0, 0, 0])
    np.testing.assert_allclose(s, [lam + 2 * mu, lam, lam, 0, 0, 0], rtol=1e-15)


def test_floating_substructure_null_spaces():
    for kind, dim in ((0, 1), (1, 6)):
        p = meshgen.cube_problem(kind, 4, 2, dirichlet_face=None)
        S = Substructures(p)
        A = S.A[0].toarray()
        ev = np.linalg.eigvalsh(A)
        assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == dim


def test_patch_test_linear_field():
    # a linear displacement field produces zero nodal forces at interior nodes
    p = meshgen.cube_problem(1, 4, 2, dirichlet_face=None)
    S = Substructures(p)
    K = S.assembled()
    rng = np.random.default_rng(0)
    B = rng.standard_normal((3, 3))
    u = (p.xyz @ B.T + rng.standard_normal(3)).ravel()
    f = K @ u
    x = p.xyz
    interior = np.all((x > 1e-12) & (x < 1 - 1e-12), axis=1)
    fi = f.reshape(-1, 3)[interior]
    assert np.abs(fi).max() < 1e-12 * np.abs(f).max()


def test_assembled_matrix_spd_with_dirichlet():
    p = meshgen.poisson_16()
    S = Substructures(p)
    K = S.assembled()
    assert abs(K - K.T).max() < 1e-14
    assert K.shape == (p.n_glob, p.n_glob)
    assert p.n_glob == 17 ** 3 - 17 ** 2
