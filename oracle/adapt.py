"""Oracle: adaptive selection of face constraints (Sec. 3, Algorithm 1).

For every pair of substructures (i, j) that share a face, the generalized
eigenproblem in matrix form (eq. (eig-matrix))

    Pi (I - E)^T S^c (I - E) Pi w = lambda Pi S^c Pi w,
    S^c = (I - P)^T A^c (I - P)   (pair quantities),

is solved densely in the factor space modulo null(Pi S^c Pi) (eq.
(eig-nullspace)).  Here S^c acts on interface values: it is the pair's
block-diagonal Schur complement with the corners shared by i and j merged.
Pi projects onto the null space of D^c_ij, the constraints of the globs that
both substructures share.  E_ij averages the two copies of every shared
non-corner dof with the weights renormalized over {i, j}.

Eigenvectors with lambda >= tau (or, with ``count``, the ``count`` dominant
ones of every face: the "3eigv" variant of Sec. 7) give rows
d = w^T Pi (I-E)^T S^c (I-E) Pi (eq. (d-def)).  Each row is split into one row
over the face and one row over each edge in the face's closure (Sec. 3 after
Proposition 1), so that D^c D^cT stays block diagonal by glob.  By default the
edge rows are dropped, as in the computations of the paper (Remark after
Proposition 1); ``edges=True`` keeps them.  The condition number indicator
(eq. (cond-ind)) reported is the largest eigenvalue that was *not* selected,
maximized over pairs.

Reading (paper silent): an edge part whose largest entry is at most
EDGE_DROP times the largest entry of its whole row d is rounding residue (the
edge's existing constraints already annihilate it) and gives no row.

Reduction (``reduced=True``, default): interface dofs of i that are not shared
with j do not enter (I - E); their values are free in the denominator, so they
are eliminated by a Schur complement of the denominator form onto the shared
dofs while the numerator keeps the unreduced block.  By the minimax principle
(Lemma, Courant-Fisher-Weyl) the nonzero eigenpairs are unchanged; the tests
compare both forms on small meshes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .bddc import _splu_spd

EDGE_DROP = 1e-8


def schur_dense(S, itf, i):
    """Dense Schur complement of A_i onto its interface dofs (original basis)."""
    A = S.A[i]
    I, G = itf.interior[i], itf.iface[i]
    AGG = A[G][:, G].toarray()
    if I.size == 0:
        return AGG
    AIG = A[I][:, G].toarray()
    lu = _splu_spd(A[I][:, I])
    X = lu.solve(AIG)
    Sd = AGG - A[G][:, I] @ X
    return 0.5 * (Sd + Sd.T)


def _schur_onto(Sfull, keep):
    """Schur complement of the symmetric matrix Sfull onto the index set keep."""
    n = Sfull.shape[0]
    rest = np.setdiff1d(np.arange(n), keep)
    if rest.size == 0:
        return Sfull[np.ix_(keep, keep)].copy()
    Snn = Sfull[np.ix_(rest, rest)]
    Sns = Sfull[np.ix_(rest, keep)]
    c = sla.cho_factor(Snn, lower=True)
    X = sla.cho_solve(c, Sns)
    R = Sfull[np.ix_(keep, keep)] - Sns.T @ X
    return 0.5 * (R + R.T)


class PairProblem:
    """Generalized eigenproblem of one face pair (i, j)."""

    def __init__(self, S, itf, cons, face_gi, Sd, reduced=True):
        gl = itf.globs[face_gi]
        i, j = gl["subs"]
        self.i, self.j, self.face_gi = i, j, face_gi
        gd = {s: S.gdof[s] for s in (i, j)}
        iface_g = {s: gd[s][itf.iface[s]] for s in (i, j)}
        shared_g = np.intersect1d(iface_g[i], iface_g[j])
        corner = np.zeros(S.n_glob, dtype=bool)
        corner[itf.corner_dofs] = True
        self.shared_corner = shared_g[corner[shared_g]]
        self.shared_nc = shared_g[~corner[shared_g]]          # where (I - E) acts
        # dofs kept on each side (global ids) and their interface positions
        side = {}
        for s in (i, j):
            X = shared_g if reduced else iface_g[s]
            posG = -np.ones(S.n_glob, dtype=np.int64)
            posG[iface_g[s]] = np.arange(iface_g[s].size)
            kp = posG[X]
            Sfull = Sd[s]
            side[s] = dict(X=X, num=Sfull[np.ix_(kp, kp)],
                           den=Sfull[np.ix_(kp, kp)] if not reduced else _schur_onto(Sfull, kp))
        # pair space: merged shared corners first, then side i dofs, side j dofs
        nc = self.shared_corner.size
        cidx = {g: k for k, g in enumerate(self.shared_corner)}
        col = {}
        nxt = nc
        for s in (i, j):
            c = np.empty(side[s]["X"].size, dtype=np.int64)
            for k, g in enumerate(side[s]["X"]):
                if g in cidx:
                    c[k] = cidx[g]
                else:
                    c[k] = nxt
                    nxt += 1
            col[s] = c
        n = nxt
        self.n = n
        self.col = col
        self.side = side

        def assemble(key):
            M = np.zeros((n, n))
            for s in (i, j):
                c = col[s]
                M[np.ix_(c, c)] += side[s][key]
            return M

        Snum = assemble("num")
        Sden = assemble("den")
        # I - E_ij on the pair space
        IE = np.zeros((n, n))
        dsum = {}
        wts = {}
        for s in (i, j):
            loc = -np.ones(S.n_glob, dtype=np.int64)
            loc[gd[s]] = np.arange(gd[s].size)
            wts[s] = itf.S.A[s].diagonal()[loc[self.shared_nc]]
        tot = wts[i] + wts[j]
        di, dj = wts[i] / tot, wts[j] / tot
        posX = {}
        for s in (i, j):
            m = {g: k for k, g in enumerate(side[s]["X"])}
            posX[s] = np.array([col[s][m[g]] for g in self.shared_nc], dtype=np.int64)
        a, b = posX[i], posX[j]
        # (I-E)w on side i: w_i - (di w_i + dj w_j) = dj (w_i - w_j)
        IE[a, a] += dj
        IE[a, b] -= dj
        IE[b, b] += di
        IE[b, a] -= di
        self.IE = IE
        # D^c_ij: rows of the globs shared by i and j
        rows = []
        for gi, g2 in enumerate(itf.globs):
            if i in g2["subs"] and j in g2["subs"]:
                G = cons.G[gi]
                if G.m == 0:
                    continue
                Rk = np.hstack([G.U, G.V])
                for k in range(G.m):
                    h = np.empty(G.n)
                    h[G.perm] = Rk[k]
                    row = np.zeros(n)
                    for s, sign in ((i, 1.0), (j, -1.0)):
                        m = {g: kk for kk, g in enumerate(side[s]["X"])}
                        for t, g in enumerate(g2["dofs"]):
                            row[col[s][m[g]]] += sign * h[t]
                    rows.append(row)
        D = np.array(rows) if rows else np.zeros((0, n))
        self.D = D
        if D.shape[0]:
            Pi = np.eye(n) - D.T @ np.linalg.solve(D @ D.T, D)
        else:
            Pi = np.eye(n)
        self.Pi = Pi
        self.C = Pi @ IE.T @ Snum @ IE @ Pi
        self.B = Pi @ Sden @ Pi
        self.Snum = Snum

    def solve(self, null_tol=1e-12):
        """All eigenpairs of C w = lambda B w in the factor space modulo
        null(B) (eq. (eig-nullspace)): null(B) is spanned by the eigenvectors
        of B whose eigenvalues are at most null_tol times the largest; the
        default 1e-12 keeps genuine small eigenvalues of a stiff pair (down to
        about 1e-11 of the largest at the 64^3 k-means size) out of the null
        space, where rounding leaves the rigid-body directions near 1e-14.
        Returns (lambdas ascending, W columns)."""
        ev, V = np.linalg.eigh(0.5 * (self.B + self.B.T))
        keep = ev > null_tol * ev.max()
        Vp = V[:, keep]
        Cp = Vp.T @ self.C @ Vp
        Bp = np.diag(ev[keep])
        lam, Y = sla.eigh(0.5 * (Cp + Cp.T), Bp)
        self.null_dim = int((~keep).sum())
        return lam, Vp @ Y

    def rows(self, W):
        """d = w^T Pi (I-E)^T S^c (I-E) Pi for each column w (eq. (d-def))."""
        return W.T @ self.C

    def face_part(self, d, itf):
        """Entries of d on substructure i's copy of the face glob dofs, in the
        glob's dof order."""
        gl = itf.globs[self.face_gi]
        m = {g: k for k, g in enumerate(self.side[self.i]["X"])}
        c = np.array([self.col[self.i][m[g]] for g in gl["dofs"]])
        return d[:, c]

    def edge_parts(self, d, itf):
        """[(edge glob index, entries of d on substructure i's copy of that
        edge's dofs in the glob's dof order)] for every edge glob shared by i
        and j (the edges of the face's closure), in glob order."""
        m = {g: k for k, g in enumerate(self.side[self.i]["X"])}
        out = []
        for gi, gl in enumerate(itf.globs):
            if gl["kind"] == "edge" and self.i in gl["subs"] and self.j in gl["subs"]:
                c = np.array([self.col[self.i][m[g]] for g in gl["dofs"]])
                out.append((gi, d[:, c]))
        return out

    def other_face_part(self, d, itf):
        gl = itf.globs[self.face_gi]
        m = {g: k for k, g in enumerate(self.side[self.j]["X"])}
        c = np.array([self.col[self.j][m[g]] for g in gl["dofs"]])
        return d[:, c]


def face_pair(S, itf, cons, fg, Sd, tau, reduced=True, count=None, edges=False):
    """Algorithm 1 on the face glob fg: the pair's eigenvalues (descending),
    the number selected, the largest unselected eigenvalue, and the new rows
    as [(glob index, row)] (face rows, then with edges=True the edge rows)."""
    pp = PairProblem(S, itf, cons, fg, Sd, reduced=reduced)
    lam, W = pp.solve()
    if count is None:
        sel = lam >= tau
    else:
        sel = np.zeros(lam.size, dtype=bool)
        sel[max(0, lam.size - count):] = True
    unsel = lam[~sel]
    out = []
    if sel.any():
        d = pp.rows(W[:, sel])[::-1]       # largest eigenvalue first
        c = pp.face_part(d, itf)
        out += [(fg, row) for row in c / np.abs(c).max(axis=1, keepdims=True)]
        if edges:
            scale = np.abs(d).max(axis=1)
            for gi, ce in pp.edge_parts(d, itf):
                for q in range(ce.shape[0]):
                    mx = np.abs(ce[q]).max()
                    if mx > EDGE_DROP * scale[q]:
                        out.append((gi, ce[q] / mx))
    return dict(lam=lam[::-1].copy(), k=int(sel.sum()),
                unsel_max=float(unsel.max()) if unsel.size else None, rows=out)


def adapt(S, itf, cons, tau, reduced=True, Sd=None, count=None, edges=False, mapper=map):
    """Algorithm 1: for every face pair select the eigenvectors with
    lambda >= tau (Sec. 7: eigenvalues greater or equal to tau were used), or
    the ``count`` largest when count is given (tau is then ignored).

    Returns dict(rows={glob: rows}, omega=indicator, k={face: count},
    lam={face: eigenvalues descending}).  rows holds the face rows and, with
    edges=True, the edge rows; on every glob they are ordered by face, then by
    eigenvalue (largest first).  ``mapper`` evaluates the independent pair
    problems (the built-in map by default; a process pool's map gives the same
    result)."""
    if Sd is None:
        Sd = {s: schur_dense(S, itf, s) for s in range(S.n_sub)}
    faces = list(itf.face_ids)
    res = list(mapper(lambda fg: face_pair(S, itf, cons, fg, Sd, tau, reduced, count, edges),
                      faces))
    rows, kcount, lams = {}, {}, {}
    omega = 0.0
    for fg, r in zip(faces, res):
        lams[fg] = r["lam"]
        kcount[fg] = r["k"]
        if r["unsel_max"] is not None:
            omega = max(omega, r["unsel_max"])
        for gi, row in r["rows"]:
            rows.setdefault(gi, []).append(row)
    rows = {g: np.array(r) for g, r in rows.items()}
    return dict(rows=rows, omega=omega, k=kcount, lam=lams)
