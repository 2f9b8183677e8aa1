"""Oracle: end-to-end BDDC-PCG driver (setup, optional adaptivity, solve)."""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse.linalg as spla

from .fem import Substructures
from .interface import Interface
from .cov import Constraints
from .bddc import Algorithm2
from .pcg import pcg


class OracleBDDC:
    def __init__(self, prob, mode="ce", extra_rows=None, augment_corners=True):
        t0 = time.perf_counter()
        self.prob = prob
        self.S = Substructures(prob)
        self.itf = Interface(self.S, augment_corners=augment_corners)
        self.t_setup = time.perf_counter() - t0
        self.mode = mode
        self.build(extra_rows)

    def build(self, extra_rows=None):
        t0 = time.perf_counter()
        self.cons = Constraints(self.itf, self.mode, extra_rows)
        self.M = Algorithm2(self.S, self.itf, self.cons)
        self.K = self.S.assembled()
        self.t_factor = time.perf_counter() - t0

    def apply(self, r):
        return self.M.apply(r)

    def solve(self, f=None, rtol=1e-8, maxit=1000):
        """PCG on the reduced problem with M_BDDC of Algorithm 2 (see
        ``reduced_pcg``)."""
        if f is None:
            f = self.prob.f
        out = reduced_pcg(self.itf, self.K, self.M.harm, self.M.apply, f, rtol, maxit)
        out["Nc"] = self.cons.Nc()
        return out


def reduced_pcg(itf, K, harm, M_apply, f, rtol=1e-8, maxit=1000):
    """PCG on the reduced problem (eq. (reduced-problem)).  Vectors are
    global, but every residual is kept exactly zero in the interiors, as the
    Remark after Lemma 1 states it is: the interior rows of R^T A R u are
    satisfied by the interior Dirichlet solves of the start and by the discrete
    harmonic search directions, so they are not iterated on.  K is the
    assembled R^T A R, harm the interior solves, M_apply the preconditioner."""
    t0 = time.perf_counter()
    interior = np.flatnonzero(itf.mult == 1)
    u0 = harm.interior_solve(f)
    fr = f.copy()
    fr[interior] = 0.0

    def Aop(v):
        q = K @ v
        q[interior] = 0.0
        return q

    out = pcg(Aop, fr, M_apply, u0, rtol=rtol, maxit=maxit)
    out["t_solve"] = time.perf_counter() - t0
    return out


def direct_solve(prob):
    """Direct sparse solve of R^T A R u = R^T f (eq. (assembled))."""
    S = Substructures(prob)
    K = S.assembled()
    return spla.splu(K.tocsc(), permc_spec="MMD_AT_PLUS_A").solve(prob.f)
