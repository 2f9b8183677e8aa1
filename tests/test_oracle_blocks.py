"""Pins of the oracle's block route of Algorithm 2 (``oracle.blocks``), the
form the full-size reference results are computed with: on meshes small
enough for the literal global form (``oracle.bddc.Algorithm2``, itself pinned
to the saddle-point system of Lemma 1 and the Pi-projected system), both give
the same preconditioned vector and the same PCG run.  The cases cover cube
and k-means partitions, scalar and elasticity problems, constraint sets c,
c+e, c+e+f and adaptive rows with edge rows kept."""
import numpy as np
import pytest

import meshgen
from oracle.fem import Substructures
from oracle.interface import Interface
from oracle.cov import Constraints
from oracle.bddc import Algorithm2
from oracle.blocks import Algorithm2Blocks, CoarseNumbering
from oracle.adapt import adapt
from oracle.solver import reduced_pcg

CASES = {
    "layers6_ce": (lambda: meshgen.small_elasticity_layers(6, 2, contrast=1e3), "ce"),
    "kmeans_elast_cef": (lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4, contrast=1e3), "cef"),
    "kmeans_poisson_c": (lambda: meshgen.small_kmeans(meshgen.POISSON, 10, 5), "c"),
    "poisson16_ce": (meshgen.poisson_16, "ce"),
}


def _setup(make, mode, extra=None):
    p = make()
    S = Substructures(p)
    itf = Interface(S)
    return p, S, itf, Constraints(itf, mode, extra)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", list(CASES))
def test_blocks_equal_literal_algorithm2(name):
    p, S, itf, cons = _setup(*CASES[name])
    a2 = Algorithm2(S, itf, cons)
    ab = Algorithm2Blocks(S, itf, cons)
    for seed in (0, 1):
        r = a2.harm.apply_T(meshgen.random_vector(S.n_glob, seed))
        # the k-means c+e+f case is the worst conditioned (1e-10 measured)
        assert rel(ab.apply(r), a2.apply(r)) < 1e-8


def test_coarse_numbering_counts_explicit_variables():
    """Coarse dofs = corner dofs + one per kept explicit average; every copy
    of a coarse dof is in a distinct substructure, and each explicit variable
    has as many copies as its glob has substructures."""
    p, S, itf, cons = _setup(*CASES["layers6_ce"])
    cn = CoarseNumbering(S, itf, cons)
    assert cn.n == itf.corner_dofs.size + sum(g.m for g in cons.G)
    copies = np.zeros(cn.n, dtype=np.int64)
    for i in range(S.n_sub):
        assert np.unique(cn.idx[i]).size == cn.idx[i].size
        np.add.at(copies, cn.idx[i], 1)
    for gi, (g, gl) in enumerate(zip(cons.G, itf.globs)):
        for k in range(g.m):
            assert copies[cn.n_corner + sum(x.m for x in cons.G[:gi]) + k] == len(gl["subs"])


def test_blocks_pcg_matches_global_with_adaptive_edge_rows():
    """Adaptive rows (tau = 5) with the edge rows kept: PCG with the block
    route takes the iterations of the literal form and reaches its solution."""
    p, S, itf, cons0 = _setup(lambda: meshgen.small_kmeans(meshgen.ELASTICITY, 8, 4,
                                                           contrast=1e3), "ce")
    ad = adapt(S, itf, cons0, 5.0, edges=True)
    cons = Constraints(itf, "ce", ad["rows"])
    K = S.assembled()
    a2 = Algorithm2(S, itf, cons)
    ab = Algorithm2Blocks(S, itf, cons, harm=a2.harm)
    g = reduced_pcg(itf, K, a2.harm, a2.apply, p.f)
    b = reduced_pcg(itf, K, a2.harm, ab.apply, p.f)
    assert g["converged"] and b["converged"]
    assert g["iters"] == b["iters"]
    assert abs(g["kappa"] - b["kappa"]) <= 1e-6 * g["kappa"]
    assert rel(b["u"], g["u"]) < 1e-10
