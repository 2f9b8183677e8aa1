"""Oracle: the BDDC preconditioner in its algebraic form (Algorithm 2, Sec. 5),
evaluated literally with global sparse matrices, plus the two equivalent forms
used as cross-checks on small meshes: the saddle-point system of Lemma 1
(eq. (BDDC-system)) and the Pi-projected regularized system (eq.
(BDDC-regular)), both in the original variables.

Algorithm 2:   A~ wbar_c = Pibar R^cT T^T E^T r,
               A~ = Pibar R^cT T^T A T R^c Pibar + t (I - Pibar),
               M r = (I - P) E T R^c wbar_c.
(I - P) is the discrete harmonic extension: interior values are replaced by
-A_II^{-1} A_IG u_G in each substructure (Sec. 2).  t is the largest diagonal
entry of R^cT T^T A T R^c (Sec. 4 suggests the largest diagonal entry of A^c;
the paper does not fix it further); the result does not depend on it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _splu_spd(M):
    return spla.splu(sp.csc_matrix(M), permc_spec="MMD_AT_PLUS_A",
                     diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))


class HarmonicExtension:
    """(I - P) on global vectors, and its transpose, from per-substructure
    Dirichlet problems A_II (Sec. 2: P is N independent Dirichlet solves)."""

    def __init__(self, S, itf):
        self.S, self.itf = S, itf
        self.lu, self.AIG = [], []
        for i in range(S.n_sub):
            I, G = itf.interior[i], itf.iface[i]
            Ai = S.A[i]
            AII = Ai[I][:, I]
            self.lu.append(_splu_spd(AII) if I.size else None)
            self.AIG.append(Ai[I][:, G])

    def interior_solve(self, f):
        """u with u_I = A_II^{-1} f_I in every substructure and u_G = 0."""
        S, itf = self.S, self.itf
        u = np.zeros(S.n_glob)
        for i in range(S.n_sub):
            gI = S.gdof[i][itf.interior[i]]
            if gI.size:
                u[gI] = self.lu[i].solve(f[gI])
        return u

    def apply(self, u):
        """(I - P) u for a global vector u."""
        S, itf = self.S, self.itf
        z = u.copy()
        for i in range(S.n_sub):
            g = S.gdof[i]
            gI, gG = g[itf.interior[i]], g[itf.iface[i]]
            if gI.size:
                z[gI] = -self.lu[i].solve(self.AIG[i] @ u[gG])
        return z

    def apply_T(self, r):
        """(I - P)^T r: interior entries become zero, interface entries receive
        -A_GI A_II^{-1} r_I from every substructure."""
        S, itf = self.S, self.itf
        z = r.copy()
        for i in range(S.n_sub):
            g = S.gdof[i]
            gI, gG = g[itf.interior[i]], g[itf.iface[i]]
            if gI.size:
                y = self.lu[i].solve(r[gI])
                z[gG] -= self.AIG[i].T @ y
                z[gI] = 0.0
        return z


class CornerSpace:
    """W^c: local dofs with the corner dofs merged; R^c: W^c -> W (eq.
    (c-subassembly) and above)."""

    def __init__(self, S, itf):
        corner = np.zeros(S.n_glob, dtype=bool)
        corner[itf.corner_dofs] = True
        idx_of_corner = -np.ones(S.n_glob, dtype=np.int64)
        wc = []
        nxt = 0
        for i in range(S.n_sub):
            g = S.gdof[i]
            w = np.empty(g.size, dtype=np.int64)
            for l, gg in enumerate(g):
                if corner[gg]:
                    if idx_of_corner[gg] < 0:
                        idx_of_corner[gg] = nxt
                        nxt += 1
                    w[l] = idx_of_corner[gg]
                else:
                    w[l] = nxt
                    nxt += 1
            wc.append(w)
        self.wc = wc
        self.n = nxt
        self.offsets = np.concatenate([[0], np.cumsum([g.size for g in S.gdof])])
        nW = int(self.offsets[-1])
        self.Rc = sp.csr_matrix((np.ones(nW), (np.arange(nW), np.concatenate(wc))),
                                shape=(nW, self.n))


class Algorithm2:
    """The preconditioner M_BDDC with the generalized change of variables."""

    def __init__(self, S, itf, cons, t=None):
        self.S, self.itf, self.cons = S, itf, cons
        self.cs = CornerSpace(S, itf)
        cs = self.cs
        self.T = sp.block_diag([cons.T_i(i) for i in range(S.n_sub)]).tocsr()
        self.A = S.A_block()
        self.E = itf.E()
        self.Kc = (cs.Rc.T @ self.T.T @ self.A @ self.T @ cs.Rc).tocsr()
        # Dbar^c: one +1 / -1 pair per row, coupling copies of an explicit
        # variable (Sec. 5, after eq. (BDDC-ch-var))
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
        self.Dbar = sp.csr_matrix((vals, (rows, cols)), shape=(nr, cs.n))
        self.Pibar = projection(self.Dbar)
        self.t = float(self.Kc.diagonal().max()) if t is None else float(t)
        I = sp.identity(cs.n, format="csr")
        self.Atil = (self.Pibar @ self.Kc @ self.Pibar + self.t * (I - self.Pibar)).tocsc()
        self.lu = _splu_spd(self.Atil)
        self.harm = HarmonicExtension(S, itf)

    def apply(self, r):
        """M_BDDC r per Algorithm 2 (E^T r on the right-hand side, no (I-P)^T,
        per the Remark after Lemma 1)."""
        cs = self.cs
        b = self.Pibar @ (cs.Rc.T @ (self.T.T @ (self.E.T @ r)))
        wbar = self.lu.solve(b)
        u = self.E @ (self.T @ (cs.Rc @ wbar))
        return self.harm.apply(u)


def projection(D):
    """Orthogonal projection onto null D: I - D^T (D D^T)^{-1} D (eq.
    (projection))."""
    n = D.shape[1]
    I = sp.identity(n, format="csr")
    if D.shape[0] == 0:
        return I
    D = sp.csr_matrix(D)
    DDt = (D @ D.T).toarray()
    Minv = np.linalg.inv(DDt)
    # (D D^T)^-1 is block diagonal (one block per glob and constraint); drop
    # the rounding-level entries outside the blocks before the sparse product
    Minv[np.abs(Minv) < 1e-13 * np.abs(Minv).max()] = 0.0
    P = I - D.T @ sp.csr_matrix(Minv) @ D
    P = sp.csr_matrix(P)
    P.data[np.abs(P.data) < 1e-14] = 0.0
    P.eliminate_zeros()
    return P


def original_constraints(S, itf, cons, cs):
    """D^c = D R^c in the original variables: for every glob, every kept
    constraint functional h_k (row k of [U V] K) and every further copy,
    h_k w_{s0} - h_k w_{s}  (eq. (Wtilde), (BDDC-Dc))."""
    rows, cols, vals = [], [], []
    nr = 0
    for gi, gl in enumerate(itf.globs):
        G = cons.G[gi]
        if G.m == 0:
            continue
        subs = sorted(gl["subs"])
        Rk = np.hstack([G.U, G.V])              # rows over permuted glob dofs
        for k in range(G.m):
            h = np.empty(G.n)
            h[G.perm] = Rk[k]
            for l in range(1, len(subs)):
                for s, sign in ((subs[0], 1.0), (subs[l], -1.0)):
                    p = itf.pos[s][gi]
                    nz = np.abs(h) > 0
                    rows += [nr] * int(nz.sum())
                    cols += list(cs.wc[s][p[nz]])
                    vals += list(sign * h[nz])
                nr += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(nr, cs.n))


class Lemma1KKT:
    """Cross-check: the saddle-point form (eq. (BDDC-system)) in the original
    variables, M r = (I - P) E R^c w_c (eq. (BDDC-prec)).  Dense; tiny meshes."""

    def __init__(self, alg2: Algorithm2):
        S, itf, cons = alg2.S, alg2.itf, alg2.cons
        cs = alg2.cs
        self.alg2 = alg2
        self.Ac = (cs.Rc.T @ alg2.A @ cs.Rc).toarray()
        self.Dc = original_constraints(S, itf, cons, cs).toarray()
        m = self.Dc.shape[0]
        n = cs.n
        K = np.zeros((n + m, n + m))
        K[:n, :n] = self.Ac
        K[:n, n:] = self.Dc.T
        K[n:, :n] = self.Dc
        self.K = K

    def apply(self, r):
        a = self.alg2
        rhs = a.cs.Rc.T @ (a.E.T @ a.harm.apply_T(r))
        n = a.cs.n
        sol = np.linalg.solve(self.K, np.concatenate([rhs, np.zeros(self.Dc.shape[0])]))
        return a.harm.apply(a.E @ (a.cs.Rc @ sol[:n]))


class ProjectedOriginal:
    """Cross-check: [Pi A^c Pi + t (I - Pi)] w_c = Pi R^cT E^T (I-P)^T r with
    Pi the projection onto null D^c in the original variables (eq.
    (BDDC-regular)).  Dense; tiny meshes."""

    def __init__(self, alg2: Algorithm2, t=None):
        kkt = Lemma1KKT(alg2)
        self.alg2 = alg2
        Dc = kkt.Dc
        n = alg2.cs.n
        if Dc.shape[0]:
            self.Pi = np.eye(n) - Dc.T @ np.linalg.solve(Dc @ Dc.T, Dc)
        else:
            self.Pi = np.eye(n)
        self.t = float(np.max(np.diag(kkt.Ac))) if t is None else t
        self.M = self.Pi @ kkt.Ac @ self.Pi + self.t * (np.eye(n) - self.Pi)

    def apply(self, r):
        a = self.alg2
        rhs = self.Pi @ (a.cs.Rc.T @ (a.E.T @ a.harm.apply_T(r)))
        w = np.linalg.solve(self.M, rhs)
        return a.harm.apply(a.E @ (a.cs.Rc @ w))
