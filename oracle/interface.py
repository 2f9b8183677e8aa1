"""Oracle: interface classification and the averaging operator E (Sec. 2).

Interface nodes are those in more than one substructure.  They are grouped by
the set of substructures that contain them: a class shared by exactly two
substructures is a face; a class shared by more than two is an edge, and an
edge with a single node is a corner (Sec. 2, definition of globs).

Readings where the paper is silent:
* corners also include the nodes of >2-substructure classes that lie on the
  domain boundary (this reproduces the 7 corners / 6 edges / 12 faces of the
  2x2x2 cube in the sparsity figure), and, for irregular partitions, face nodes
  added greedily until every face pair sees 1 (scalar) or 3 non-collinear
  (elasticity) corners in its closure (Assumptions 1 and 2);
* classification is done on the full mesh, then Dirichlet dofs are removed
  everywhere; globs left without dofs vanish;
* the weights of E are proportional to the diagonal of the substructure
  matrices (Sec. 7, numerical results), per dof.
"""
from __future__ import annotations

from collections import OrderedDict
import numpy as np
import scipy.sparse as sp


def boundary_nodes(hex8, n_nodes):
    """Nodes on the domain boundary: nodes of element faces owned by exactly
    one element."""
    fl = np.array([[0, 1, 2, 3], [4, 5, 6, 7], [0, 1, 5, 4],
                   [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]])
    faces = np.sort(hex8[:, fl].reshape(-1, 4), axis=1)
    uq, cnt = np.unique(faces, axis=0, return_counts=True)
    b = np.zeros(n_nodes, dtype=bool)
    b[uq[cnt == 1].ravel()] = True
    return b


def node_substructures(prob):
    ne = prob.n_elems
    inc = sp.csr_matrix((np.ones(8 * ne), (prob.hex8.ravel(), np.repeat(prob.elem_sub, 8))),
                        shape=(prob.n_nodes, prob.n_sub))
    inc.sum_duplicates()
    inc.sort_indices()
    return [tuple(inc.indices[inc.indptr[n]:inc.indptr[n + 1]].tolist())
            for n in range(prob.n_nodes)]


def _noncollinear_count(pts, tol=1e-12):
    """1 if >=1 point, 2 if >=2 distinct, 3 if three non-collinear exist."""
    if len(pts) == 0:
        return 0
    P = np.asarray(pts, dtype=float)
    d = P - P[0]
    if np.abs(d).max() < tol:
        return 1
    return 1 + min(2, np.linalg.matrix_rank(d, tol=1e-9))


class Interface:
    """Globs of a substructured mesh and the weights of E.

    Attributes
    ----------
    corners : list of node ids (ascending) that are corners with free dofs
    globs   : list of dicts {kind: 'edge'|'face', subs: tuple, nodes, dofs}
              (dofs = global free dofs of the glob, ascending)
    corner_dofs : global free dofs of all corners (ascending)
    interior[i], iface[i] : local dof indices of substructure i
    pos[i] : dict glob index -> local positions of that glob's dofs in i
    delta[i] : weights of E on the local dofs of i (interior: 1)
    """

    def __init__(self, S, augment_corners=True):
        prob = S.prob
        self.S = S
        dpn = prob.dpn
        ns = node_substructures(prob)
        self.node_subs = ns
        bnd = boundary_nodes(prob.hex8, prob.n_nodes)
        classes = OrderedDict()
        for n, key in enumerate(ns):
            if len(key) > 1:
                classes.setdefault(key, []).append(n)
        corner_nodes = []
        edges, faces = [], []
        for key in sorted(classes):
            nodes = classes[key]
            if len(key) == 2:
                faces.append((key, nodes))
            elif len(nodes) == 1:
                corner_nodes.append(nodes[0])
            else:
                on_b = [n for n in nodes if bnd[n]]
                rest = [n for n in nodes if not bnd[n]]
                corner_nodes += on_b
                if rest:
                    edges.append((key, rest))
        corner_set = set(corner_nodes)
        if augment_corners:
            faces, corner_set = self._augment(prob, ns, faces, corner_set)
        self.corner_nodes_all = sorted(corner_set)

        f2g = S.full2glob

        def dofs_of(nodes):
            d = (dpn * np.asarray(sorted(nodes), dtype=np.int64)[:, None]
                 + np.arange(dpn)[None, :]).ravel()
            g = f2g[d]
            return g[g >= 0]

        self.corners = [n for n in self.corner_nodes_all if dofs_of([n]).size > 0]
        self.corner_dofs = np.sort(np.concatenate([dofs_of([n]) for n in self.corners])) \
            if self.corners else np.zeros(0, dtype=np.int64)
        self.globs = []
        for kind, lst in (("edge", edges), ("face", faces)):
            for key, nodes in lst:
                nodes = sorted(n for n in nodes if n not in corner_set)
                if not nodes:
                    continue
                d = dofs_of(nodes)
                if d.size == 0:
                    continue
                self.globs.append(dict(kind=kind, subs=tuple(key), nodes=np.array(nodes),
                                       dofs=d))
        # local data
        n_glob = S.n_glob
        self.interior, self.iface, self.pos, self.delta = [], [], [], []
        dsum = np.zeros(n_glob)
        diags = [S.A[i].diagonal() for i in range(S.n_sub)]
        for i in range(S.n_sub):
            np.add.at(dsum, S.gdof[i], diags[i])
        mult = np.zeros(n_glob, dtype=np.int64)
        for i in range(S.n_sub):
            np.add.at(mult, S.gdof[i], 1)
        self.mult = mult
        for i in range(S.n_sub):
            g = S.gdof[i]
            self.interior.append(np.flatnonzero(mult[g] == 1))
            self.iface.append(np.flatnonzero(mult[g] > 1))
            self.delta.append(diags[i] / dsum[g])
            loc = -np.ones(n_glob, dtype=np.int64)
            loc[g] = np.arange(g.size)
            p = {}
            for gi, gl in enumerate(self.globs):
                if i in gl["subs"]:
                    p[gi] = loc[gl["dofs"]]
                    assert (p[gi] >= 0).all()
            self.pos.append(p)
        self.face_ids = [k for k, gl in enumerate(self.globs) if gl["kind"] == "face"]
        self.edge_ids = [k for k, gl in enumerate(self.globs) if gl["kind"] == "edge"]

    def _augment(self, prob, ns, faces, corner_set):
        """Greedy corner augmentation so that every face pair sees enough
        corners in the closure of its face (Assumption 2)."""
        need = 1 if prob.kind == 0 else 3
        xyz = prob.xyz
        # closure of a face pair: all nodes shared by both substructures
        shared = {}
        for n, s in enumerate(ns):
            if len(s) > 1:
                for a in range(len(s)):
                    for b in range(a + 1, len(s)):
                        shared.setdefault((s[a], s[b]), []).append(n)
        out = []
        for key, nodes in faces:
            cl = shared[key]
            cpts = [xyz[n] for n in cl if n in corner_set]
            cand = [n for n in nodes if n not in corner_set]
            if _noncollinear_count(cpts) >= need or not cand:
                out.append((key, nodes))
                continue
            cen = xyz[cand].mean(axis=0)
            while _noncollinear_count(cpts) < need and cand:
                # distances equal within 1e-9 (relative) count as ties, which
                # go to the lowest node id
                if not cpts:
                    d = ((xyz[cand] - cen) ** 2).sum(1)
                    ok = d <= d.min() * (1 + 1e-9) + 1e-300
                else:
                    C = np.array(cpts)
                    d = np.min(((xyz[cand][:, None, :] - C[None]) ** 2).sum(2), axis=1)
                    ok = d >= d.max() * (1 - 1e-9)
                k = int(np.flatnonzero(ok)[0])
                n = cand.pop(k)
                corner_set.add(n)
                cpts.append(xyz[n])
            out.append((key, [n for n in nodes if n not in corner_set]))
        return out, corner_set

    # ------------------------------------------------------------------
    def E(self):
        """Averaging operator E: W -> U as a sparse matrix (n_glob x sum n_i):
        (E w)(g) = sum_i delta_i(g) w_i(g)  (Sec. 2, eq. (E))."""
        S = self.S
        rows = np.concatenate(S.gdof)
        cols = np.arange(rows.size)
        vals = np.concatenate(self.delta)
        return sp.csr_matrix((vals, (rows, cols)), shape=(S.n_glob, rows.size))

    def counts(self):
        return dict(corners=len(self.corners),
                    edges=len(self.edge_ids), faces=len(self.face_ids))
