"""Oracle: averages and the generalized change of variables (Sec. 5).

For each glob g the constraint rows H^avg_g (weights over the glob's dofs, in
ascending global dof order, identical in every substructure sharing g) are
factored by QR with column pivoting, H^avg = Q [U V] K, and the inverse change
of variables is T = K^{-1} [U^{-1}  -U^{-1} V; 0  I]  (eq. (T)).  Rows whose
diagonal entry of U is negligible are dropped (Sec. 5, after eq. (T)).

Reading (the paper leaves the details open): the QR is LAPACK's DGEQP3 through SciPy, as in
the paper; rows with |U_kk| <= 1e-10 |U_11| are dropped.  Position
convention: the k-th new (explicit) variable of glob g is stored at the local
position of the dof K selects k-th; the other new variables are the unchanged
original dofs at their own positions.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

DROP_TOL = 1e-10


def unit_averages(glob, dpn):
    """One unit-weight (arithmetic) average per displacement component over
    the glob's dofs (Sec. 7: arithmetic averages; the worked example of Sec. 5
    uses unit weights)."""
    dofs = glob["dofs"]
    # component of each glob dof: dofs are node-major, component-minor, so the
    # component is recovered from the full-mesh dof id stored with the glob
    comp = glob["comp"]
    rows = []
    for c in range(dpn):
        sel = comp == c
        if sel.any():
            rows.append(sel.astype(np.float64))
    return np.array(rows) if rows else np.zeros((0, dofs.size))


class GlobTransform:
    """QR-CP of H^avg for one glob and the resulting T_g."""

    def __init__(self, H):
        H = np.atleast_2d(np.asarray(H, dtype=np.float64))
        m, n = H.shape
        self.n = n
        if m == 0:
            self.m = 0
            self.perm = np.arange(n)
            self.Tp = np.eye(n)
            self.T = np.eye(n)
            self.rows = H
            return
        Q, Rm, P = sla.qr(H, pivoting=True, mode="economic")
        d = np.abs(np.diag(Rm))
        keep = d > DROP_TOL * d[0]
        mk = int(np.count_nonzero(keep))
        # DGEQP3 orders |U_kk| non-increasingly: the kept rows are leading
        assert keep[:mk].all()
        U = Rm[:mk, :mk]
        V = Rm[:mk, mk:]
        Ui = sla.solve_triangular(U, np.eye(mk))
        Tp = np.eye(n)
        Tp[:mk, :mk] = Ui
        Tp[:mk, mk:] = -Ui @ V
        T = np.empty((n, n))
        T[np.ix_(P, P)] = Tp          # T[P[a], P[b]] = Tp[a, b]
        self.m = mk
        self.perm = P
        self.Tp = Tp
        self.T = T
        self.U, self.V, self.Q = U, V, Q
        self.rows = H
        self.dropped = int(m - mk)

    @property
    def explicit(self):
        """Glob-local indices holding the explicit (average) variables."""
        return self.perm[:self.m]


def glob_components(itf):
    """Attach the component index of each glob dof (needed for per-component
    averages)."""
    S = itf.S
    dpn = S.prob.dpn
    free = S.prob.free_dofs
    for gl in itf.globs:
        gl["comp"] = free[gl["dofs"]] % dpn


class Constraints:
    """H^avg and T_g for every glob; the block-diagonal T_i per substructure.

    mode: 'c' (corners only), 'ce' (+ edge averages), 'cef' (+ face averages),
    'all' (every glob dof constrained: H^avg = I, so the constrained space is
    the continuous one and BDDC becomes exact).
    extra_rows: dict glob index -> extra rows over that glob (the adaptive
    face rows, and the adaptive edge rows when they are kept), stacked after
    the averages.
    """

    def __init__(self, itf, mode="ce", extra_rows=None):
        self.itf = itf
        S = itf.S
        dpn = S.prob.dpn
        glob_components(itf)
        self.H = []
        for k, gl in enumerate(itf.globs):
            rows = []
            if mode == "all":
                rows.append(np.eye(gl["dofs"].size))
            if (gl["kind"] == "edge" and mode in ("ce", "cef")) or \
               (gl["kind"] == "face" and mode == "cef"):
                rows.append(unit_averages(gl, dpn))
            if extra_rows and k in extra_rows:
                rows.append(np.atleast_2d(extra_rows[k]))
            rows = [r for r in rows if r.size]
            self.H.append(np.vstack(rows) if rows else np.zeros((0, gl["dofs"].size)))
        self.G = [GlobTransform(H) for H in self.H]

    def Nc(self):
        """Number of rows of D: sum over globs of m_g (k_g - 1)."""
        return int(sum(g.m * (len(gl["subs"]) - 1) for g, gl in zip(self.G, self.itf.globs)))

    def T_i(self, i):
        """T_i (new -> original variables) on the local dofs of substructure i."""
        itf = self.itf
        n_i = itf.S.gdof[i].size
        T = sp.lil_matrix((n_i, n_i))
        T.setdiag(1.0)
        for gi, p in itf.pos[i].items():
            g = self.G[gi]
            if g.m == 0:
                continue
            T[np.ix_(p, p)] = g.T
        return T.tocsr()

    def explicit_positions(self, i):
        """List of (glob index, k, local position) of explicit variables of i."""
        out = []
        for gi, p in sorted(self.itf.pos[i].items()):
            g = self.G[gi]
            for k in range(g.m):
                out.append((gi, k, int(p[g.perm[k]])))
        return out
