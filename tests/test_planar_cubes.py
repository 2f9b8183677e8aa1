"""The planar-cubes workload (Sec. 7, Table 9): k x k cubic substructures of
8^3 elasticity elements in one layer, corners only.

The generator is pinned by the table's sizes: the mesh of the k-th problem
has exactly the listed number of degrees of freedom (all nodes, the clamped
ones included) for 4 ... 64 substructures.  The oracle is checked on the
smallest problem: corners-only BDDC converges and its solution satisfies the
assembled system.  The material and the load are not stated in the paper, so
the iteration counts and condition numbers of the table are context only.
"""
import json
import os

import numpy as np

import meshgen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_planar_cubes_sizes_match_table9():
    t = json.load(open(os.path.join(GOLD, "table9_planar_cubes.json")))
    for k, n_sub, dofs in zip(range(2, 9), t["n_sub"], t["dofs"]):
        p = meshgen.planar_cubes(k)
        assert p.n_sub == n_sub == k * k
        assert p.n_nodes * p.dpn == dofs
        # every substructure is an 8^3 cube
        assert np.array_equal(np.bincount(p.elem_sub), np.full(n_sub, 512))
        # the load is a unit traction on the face x = k of area k
        assert abs(p.load.sum() + k) < 1e-12


def test_planar_cubes_oracle_corners_only():
    from oracle.solver import OracleBDDC
    p = meshgen.planar_cubes(2)
    o = OracleBDDC(p, "c")
    assert o.cons.Nc() == 0
    out = o.solve()
    assert out["converged"]
    r = np.linalg.norm(p.f - o.K @ out["u"]) / np.linalg.norm(p.f)
    assert r < 1e-6
    # more constraints can only help: c+e converges in fewer iterations
    assert OracleBDDC(p, "ce").solve()["iters"] < out["iters"]
