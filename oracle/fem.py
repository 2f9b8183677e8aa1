"""Oracle: finite element substructure matrices (Sec. 2, eq. (block-operators)).

A_i is the subassembly of element matrices of the elements of substructure i
only; it is symmetric positive semidefinite.  Elements are trilinear (Q1)
hexahedra integrated with the 2x2x2 Gauss rule (exact for affine cubes).
Parity: pinned by the closed-form unit-cube Laplacian, the rigid-body null
space of the elasticity element and the patch test (tests/test_oracle_fem.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# reference coordinates of the hex8 nodes
XI = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
               [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
_g = 1.0 / np.sqrt(3.0)
GAUSS = np.array([[a, b, c] for c in (-_g, _g) for b in (-_g, _g) for a in (-_g, _g)])


def shape_grad_ref(p):
    """dN_a/dxi at reference point p, shape (8, 3)."""
    x, y, z = p
    g = np.empty((8, 3))
    for a in range(8):
        xa, ya, za = XI[a]
        g[a, 0] = xa * (1 + ya * y) * (1 + za * z) / 8.0
        g[a, 1] = ya * (1 + xa * x) * (1 + za * z) / 8.0
        g[a, 2] = za * (1 + xa * x) * (1 + ya * y) / 8.0
    return g


_DN_REF = np.stack([shape_grad_ref(p) for p in GAUSS])   # (8 gp, 8 nodes, 3)


def elasticity_D(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def element_matrices(xyz, hex8, coef, kind, nu):
    """Element stiffness matrices, shape (n_e, 8*dpn, 8*dpn)."""
    X = xyz[hex8]                                       # (ne, 8, 3)
    ne = X.shape[0]
    dpn = 1 if kind == 0 else 3
    K = np.zeros((ne, 8 * dpn, 8 * dpn))
    for q in range(8):
        dN = _DN_REF[q]                                 # (8,3)
        J = np.einsum("ai,eaj->eij", dN, X)             # J[e,i,j] = d x_j / d xi_i
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        G = np.einsum("eij,aj->eai", Jinv, dN)          # dN_a/dx_i
        if kind == 0:
            K += coef[:, None, None] * detJ[:, None, None] * np.einsum("eai,ebi->eab", G, G)
        else:
            B = np.zeros((ne, 6, 24))
            for a in range(8):
                gx, gy, gz = G[:, a, 0], G[:, a, 1], G[:, a, 2]
                B[:, 0, 3 * a + 0] = gx
                B[:, 1, 3 * a + 1] = gy
                B[:, 2, 3 * a + 2] = gz
                B[:, 3, 3 * a + 1] = gz
                B[:, 3, 3 * a + 2] = gy
                B[:, 4, 3 * a + 0] = gz
                B[:, 4, 3 * a + 2] = gx
                B[:, 5, 3 * a + 0] = gy
                B[:, 5, 3 * a + 1] = gx
            D = elasticity_D(1.0, nu)
            DB = np.einsum("kl,elj->ekj", D, B)
            K += (coef * detJ)[:, None, None] * (B.transpose(0, 2, 1) @ DB)
    return K


class Substructures:
    """Local dof numbering and matrices of every substructure.

    For substructure i: ``nodes[i]`` (global node ids, ascending), ``gdof[i]``
    (global free-dof id of each local dof; Dirichlet dofs removed), and the
    sparse SPSD ``A[i]`` on those dofs (Sec. 2: A_i from elements of Omega_i
    only).  Local dofs are node-major, component-minor over the free dofs."""

    def __init__(self, prob):
        self.prob = prob
        dpn = prob.dpn
        nfull = prob.n_nodes * dpn
        free = prob.free_dofs
        full2glob = -np.ones(nfull, dtype=np.int64)
        full2glob[free] = np.arange(free.size)
        self.full2glob = full2glob
        self.n_glob = free.size
        Ke = element_matrices(prob.xyz, prob.hex8, prob.coef, prob.kind, prob.nu)
        edofs = (dpn * prob.hex8[:, :, None] + np.arange(dpn)[None, None, :]).reshape(
            prob.n_elems, 8 * dpn)
        self.nodes, self.gdof, self.A = [], [], []
        for i in range(prob.n_sub):
            els = np.flatnonzero(prob.elem_sub == i)
            nodes = np.unique(prob.hex8[els])
            fulld = (dpn * nodes[:, None] + np.arange(dpn)[None, :]).ravel()
            g = full2glob[fulld]
            keep = g >= 0
            loc_of_full = -np.ones(nfull, dtype=np.int64)
            loc_of_full[fulld[keep]] = np.arange(int(keep.sum()))
            ld = loc_of_full[edofs[els]]                         # (ne_i, 8dpn)
            rows = np.repeat(ld, ld.shape[1], axis=1).ravel()
            cols = np.tile(ld, (1, ld.shape[1])).ravel()
            vals = Ke[els].reshape(len(els), -1).ravel()
            m = (rows >= 0) & (cols >= 0)
            n_i = int(keep.sum())
            Ai = sp.csr_matrix((vals[m], (rows[m], cols[m])), shape=(n_i, n_i))
            Ai.sum_duplicates()
            self.nodes.append(nodes)
            self.gdof.append(g[keep])
            self.A.append(Ai)
        self.n_sub = prob.n_sub

    def R_i(self, i):
        """0-1 restriction U -> W_i as a sparse matrix (n_i x n_glob)."""
        n_i = self.gdof[i].size
        return sp.csr_matrix((np.ones(n_i), (np.arange(n_i), self.gdof[i])),
                             shape=(n_i, self.n_glob))

    def R(self):
        """Global-to-local map R: U -> W (eq. (var) and below), stacked."""
        return sp.vstack([self.R_i(i) for i in range(self.n_sub)]).tocsr()

    def A_block(self):
        return sp.block_diag(self.A).tocsr()

    def assembled(self):
        """R^T A R, the global stiffness matrix (eq. (assembled))."""
        R = self.R()
        return (R.T @ self.A_block() @ R).tocsr()
