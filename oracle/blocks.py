"""Oracle: Algorithm 2 (Sec. 5) by blocks, for meshes whose global form does
not fit.

The literal form in ``bddc.py`` factors the whole regularized matrix
A~ = Pibar R^cT T^T A T R^c Pibar + t (I - Pibar) at once.  Its solution is
reached here by the block elimination that the Remark after Algorithm 2
describes (the primal assembly of the coarse dofs), written out with
per-substructure sparse factors and one dense coarse matrix:

* In the new variables of Sec. 5, every explicit variable (the first m_g new
  variables of a glob, eq. (T)) and every corner dof is a coarse ("pi") dof;
  all other local dofs, interiors included, are "r" dofs of their
  substructure.
* range(Pibar) holds the vectors whose copies of each explicit variable agree
  (Pibar averages over copies, eq. (projection) with Dbar^c).  On it A~ acts as
  Pibar K Pibar, so for a right-hand side b = Pibar b the solution is
  wbar = Rt y with (Rt^T K Rt) y = Rt^T b, where Rt maps one value per coarse
  dof to all of its copies (the primal assembly).
* That system is solved by eliminating each substructure's r block:
  Phi_i = -K_rr^-1 K_rpi, S_pi^i = K_pipi + K_pir Phi_i, S_c = sum_i R_pi^T
  S_pi^i R_pi (dense, Cholesky), then
  g = sum_i R_pi^T (b_pi + Phi_i^T b_r),  y_pi = S_c^-1 g,
  y_r = K_rr^-1 b_r + Phi_i R_pi y_pi.

The preconditioner is then M r = (I - P) E T R^c wbar, exactly as in the
literal form; tests pin this class to ``bddc.Algorithm2`` on small meshes.
Local K_rr blocks keep their interiors (sparse LU, SciPy's SuperLU).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bddc import HarmonicExtension


def _splu(M):
    return spla.splu(sp.csc_matrix(M), permc_spec="MMD_AT_PLUS_A",
                     diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))


class CoarseNumbering:
    """Coarse dofs: the global corner dofs (ascending), then one per explicit
    variable (glob order, then row order k).  Per substructure: the local
    positions of its coarse dofs and their coarse indices."""

    def __init__(self, S, itf, cons):
        n_corner = itf.corner_dofs.size
        cidx = -np.ones(S.n_glob, dtype=np.int64)
        cidx[itf.corner_dofs] = np.arange(n_corner)
        goff = np.zeros(len(itf.globs) + 1, dtype=np.int64)
        goff[1:] = np.cumsum([g.m for g in cons.G])
        self.n = int(n_corner + goff[-1])
        self.n_corner = n_corner
        self.pos, self.idx = [], []
        for i in range(S.n_sub):
            g = S.gdof[i]
            lc = np.flatnonzero(cidx[g] >= 0)
            pos = list(lc)
            idx = list(cidx[g[lc]])
            for gi, k, lp in cons.explicit_positions(i):
                pos.append(lp)
                idx.append(n_corner + goff[gi] + k)
            self.pos.append(np.asarray(pos, dtype=np.int64))
            self.idx.append(np.asarray(idx, dtype=np.int64))


class LocalBlocks:
    """One substructure in the new variables: K^i = T_i^T A_i T_i split into
    r and pi, the sparse factor of K_rr, Phi_i and S_pi^i.  ``coarse`` may
    give (Phi_i, S_pi^i) computed elsewhere from the same inputs (for instance
    in a worker process, since the sparse factor cannot be sent back)."""

    def __init__(self, A_i, T_i, pi_pos, coarse=None):
        K = (T_i.T @ A_i @ T_i).tocsr()
        n = K.shape[0]
        mask = np.ones(n, dtype=bool)
        mask[pi_pos] = False
        self.r = np.flatnonzero(mask)
        self.p = np.asarray(pi_pos, dtype=np.int64)
        Kr = K[self.r]
        self.lu = _splu(Kr[:, self.r])
        self.T = T_i
        if coarse is not None:
            self.Phi, self.Spi = coarse
            return
        Krp = Kr[:, self.p].toarray()
        self.Phi = -self.lu.solve(Krp) if self.p.size else np.zeros((self.r.size, 0))
        Kpp = K[self.p][:, self.p].toarray()
        Spi = Kpp + Krp.T @ self.Phi
        self.Spi = 0.5 * (Spi + Spi.T)


class Algorithm2Blocks:
    """M_BDDC of Algorithm 2 through per-substructure blocks and a dense
    coarse matrix (see the module docstring).

    ``local`` may hold prebuilt LocalBlocks (for instance with their coarse
    blocks computed in worker processes); by default they are built here, one
    substructure after another."""

    def __init__(self, S, itf, cons, local=None, harm=None):
        self.S, self.itf, self.cons = S, itf, cons
        self.cn = CoarseNumbering(S, itf, cons)
        if local is None:
            local = [LocalBlocks(S.A[i], cons.T_i(i), self.cn.pos[i]) for i in range(S.n_sub)]
        self.local = local
        Sc = np.zeros((self.cn.n, self.cn.n))
        for i, lb in enumerate(local):
            ix = self.cn.idx[i]
            Sc[np.ix_(ix, ix)] += lb.Spi
        self.Sc = Sc
        self.chol = sla.cho_factor(Sc, lower=True) if self.cn.n else None
        self.harm = HarmonicExtension(S, itf) if harm is None else harm

    def local_rhs(self, r):
        """b_i = T_i^T (delta_i * R_i r) for every substructure (T^T E^T r)."""
        return [lb.T.T @ (self.itf.delta[i] * r[self.S.gdof[i]]) for i, lb in enumerate(self.local)]

    def solve_new(self, b):
        """The primal solve: local vectors x_i (new variables, r and pi parts)
        with copies of every coarse dof equal."""
        yr = []
        g = np.zeros(self.cn.n)
        for i, lb in enumerate(self.local):
            br = b[i][lb.r]
            y = lb.lu.solve(br)
            yr.append(y)
            np.add.at(g, self.cn.idx[i], b[i][lb.p] + lb.Phi.T @ br)
        ypi = sla.cho_solve(self.chol, g) if self.cn.n else g
        x = []
        for i, lb in enumerate(self.local):
            xi = np.empty(lb.r.size + lb.p.size)
            yp = ypi[self.cn.idx[i]]
            xi[lb.r] = yr[i] + lb.Phi @ yp
            xi[lb.p] = yp
            x.append(xi)
        return x

    def apply(self, r):
        """M_BDDC r = (I - P) E T R^c wbar (no (I-P)^T on the right-hand side,
        per the Remark after Lemma 1)."""
        x = self.solve_new(self.local_rhs(r))
        u = np.zeros(self.S.n_glob)
        for i, lb in enumerate(self.local):
            np.add.at(u, self.S.gdof[i], self.itf.delta[i] * (lb.T @ x[i]))
        return self.harm.apply(u)
