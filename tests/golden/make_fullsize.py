#!/usr/bin/env python3
"""Writes the oracle's reference results for the two full-size workloads.

    python tests/golden/make_fullsize.py elasticity48 [--workers N]
    python tests/golden/make_fullsize.py kmeans64 [--workers N]

Calls only ``oracle/`` (and the seeded generators in ``meshgen/``).  Each run
writes ``tests/golden/<name>.json`` (counts, adaptive selection, PCG figures,
row-span fingerprints, the oracle's wall times and core count) and
``tests/golden/<name>.npz`` (the solution u).

Workloads:
* elasticity48: 48^3 Q1 elasticity elements in 4 x 4 x 4 cubic
  substructures, layered E in {1, 1e6}, clamped at z = 0, gravity; corners
  and edge averages, then adaptive face rows at tau = 10 with the edge parts
  dropped (Remark after Proposition 1).
* kmeans64: 64^3 elements in 64 k-means substructures with 5% of the
  elements at E = 1e5; adaptive rows at tau = 10 with the edge parts kept as
  edge rows (Sec. 3 after Proposition 1).

Steps, all from the oracle:
1. dense Schur complements S_i of every substructure (worker processes);
2. Algorithm 1 on every face pair (worker processes): all eigenvalues, the
   selected rows, the indicator omega;
3. the constraints with the adaptive rows (QR-CP per glob, eq. (T));
4. Algorithm 2 by blocks (``oracle.blocks``): K_rr factors, Phi_i and S_pi^i
   (worker processes), the dense coarse Cholesky;
5. PCG on the reduced problem to 1e-8 (iterations, Lanczos kappa) and again
   to 1e-11, whose solution is stored as the reference u.

The oracle's wall time of steps 1-5 at 1e-8 (``oracle.step_s``, with the
worker count) and its CPU time summed over all processes
(``oracle.step_cpu_s``, about what one core would take) are recorded, with a
calibration task (one substructure's Schur complement on one thread) that
relates this host's speed to another's.

Every BLAS call runs on one thread and every worker task is independent, so
the files do not depend on the number of workers: the script reproduces them
bit for bit on the same host libraries.

Row-span fingerprint of face f (array ``face<f>`` of the .npz, faces
numbered in glob order): with v drawn from default_rng(glob index) (standard
normal over the face's dofs), the orthogonal projection of v onto the span
of the face's selected rows.  It differs between two row sets by about the
sine of their largest principal angle times |v|.  ``edge_rows`` maps an edge
index (edges numbered in glob order) to its number of adaptive rows.
"""
from __future__ import annotations

import os
import sys

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import argparse
import json
import multiprocessing as mp
import platform
import resource
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import meshgen                                              # noqa: E402
from oracle.fem import Substructures                        # noqa: E402
from oracle.interface import Interface                      # noqa: E402
from oracle.cov import Constraints                          # noqa: E402
from oracle.adapt import adapt, schur_dense                 # noqa: E402
from oracle.blocks import Algorithm2Blocks, CoarseNumbering, LocalBlocks  # noqa: E402
from oracle.bddc import HarmonicExtension                   # noqa: E402
from oracle.solver import reduced_pcg                       # noqa: E402

WORKLOADS = {
    "elasticity48": dict(make=meshgen.elasticity_layers_48, edges=False, tau=10.0),
    "kmeans64": dict(make=meshgen.elasticity_kmeans_64, edges=True, tau=10.0),
}
RTOL = 1e-8
RTOL_REF = 1e-11
MAXIT = 3000

_FN = None


def _call(x):
    return _FN(x)


def pmap(fn, items, workers):
    """Ordered map of fn over items in forked worker processes (fn and the
    data it closes over are inherited by the fork)."""
    global _FN
    items = list(items)
    if workers <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    _FN = fn
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_call, items, chunksize=1)
    _FN = None
    return out


def cpu_seconds():
    """User + system CPU time of this process and its finished workers."""
    a = resource.getrusage(resource.RUSAGE_SELF)
    b = resource.getrusage(resource.RUSAGE_CHILDREN)
    return a.ru_utime + a.ru_stime + b.ru_utime + b.ru_stime


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.machine()


def fingerprint(rows, seed):
    """Projection of a seeded standard normal vector onto span(rows)."""
    v = np.random.default_rng(seed).standard_normal(rows.shape[1])
    u, s, _ = np.linalg.svd(rows.T, full_matrices=False)
    q = u[:, s > 1e-10 * s[0]]
    return q @ (q.T @ v)


def run(name, workers):
    cfg = WORKLOADS[name]
    T = {}
    t0 = time.perf_counter()
    p = cfg["make"]()
    S = Substructures(p)
    itf = Interface(S)
    cons0 = Constraints(itf, "ce")
    T["setup_s"] = time.perf_counter() - t0
    print(f"{name}: setup {T['setup_s']:.1f} s, n_glob {p.n_glob}, Nc(c+e) {cons0.Nc()}", flush=True)
    # calibration task: one substructure's dense Schur complement on one
    # thread (the median interior size), to compare hosts
    cal = int(np.argsort([itf.interior[i].size for i in range(S.n_sub)])[S.n_sub // 2])
    t0 = time.perf_counter()
    schur_dense(S, itf, cal)
    cal_s = time.perf_counter() - t0
    print(f"  calibration: Schur complement of substructure {cal}: {cal_s:.2f} s", flush=True)

    # 1-2: Schur complements and Algorithm 1 on every face pair
    c0 = cpu_seconds()
    t0 = time.perf_counter()
    order = sorted(range(S.n_sub), key=lambda s: -itf.interior[s].size)
    sd = pmap(lambda s: schur_dense(S, itf, s), order, workers)
    Sd = dict(zip(order, sd))
    del sd
    T["schur_s"] = time.perf_counter() - t0
    print(f"  Schur complements {T['schur_s']:.1f} s", flush=True)
    t0 = time.perf_counter()
    ad = adapt(S, itf, cons0, cfg["tau"], Sd=Sd, edges=cfg["edges"],
               mapper=lambda fn, xs: pmap(fn, xs, workers))
    T["pairs_s"] = time.perf_counter() - t0
    del Sd
    print(f"  pair problems {T['pairs_s']:.1f} s, omega {ad['omega']:.6g}", flush=True)

    # 3-4: constraints with the adaptive rows, Algorithm 2 by blocks
    t0 = time.perf_counter()
    cons = Constraints(itf, "ce", extra_rows=ad["rows"])
    cn = CoarseNumbering(S, itf, cons)

    def coarse_blocks(i):
        lb = LocalBlocks(S.A[i], cons.T_i(i), cn.pos[i])
        return lb.Phi, lb.Spi

    order = sorted(range(S.n_sub), key=lambda s: -S.gdof[s].size)
    cb = dict(zip(order, pmap(coarse_blocks, order, workers)))
    local = [LocalBlocks(S.A[i], cons.T_i(i), cn.pos[i], coarse=cb.pop(i)) for i in range(S.n_sub)]
    harm = HarmonicExtension(S, itf)
    M = Algorithm2Blocks(S, itf, cons, local=local, harm=harm)
    K = S.assembled()
    T["factor_s"] = time.perf_counter() - t0
    print(f"  Algorithm 2 blocks {T['factor_s']:.1f} s, Nc {cons.Nc()}, coarse dofs {cn.n}",
          flush=True)

    # 5: PCG
    t0 = time.perf_counter()
    r8 = reduced_pcg(itf, K, harm, M.apply, p.f, rtol=RTOL, maxit=MAXIT)
    T["pcg_s"] = time.perf_counter() - t0
    step_cpu = cpu_seconds() - c0
    print(f"  PCG 1e-8: {r8['iters']} iterations, kappa {r8['kappa']:.6g}, {T['pcg_s']:.1f} s",
          flush=True)
    t0 = time.perf_counter()
    rr = reduced_pcg(itf, K, harm, M.apply, p.f, rtol=RTOL_REF, maxit=MAXIT)
    T["pcg_ref_s"] = time.perf_counter() - t0
    u = rr["u"]
    u0 = harm.interior_solve(p.f)
    r0 = float(np.linalg.norm(p.f - K @ u0))
    d8 = float(np.abs(r8["u"] - u).max() / np.abs(u).max())
    print(f"  PCG {RTOL_REF:g}: {rr['iters']} iterations; max|u_1e-8 - u| / max|u| = {d8:.3e}",
          flush=True)

    faces = []
    for f, gi in enumerate(itf.face_ids):
        lam = ad["lam"][gi]
        k = ad["k"][gi]
        ent = dict(face=f, glob=int(gi), subs=[int(s) for s in itf.globs[gi]["subs"]],
                   n_dofs=int(itf.globs[gi]["dofs"].size), k=int(k),
                   lam=[float(x) for x in lam[:k + 4]])
        faces.append(ent)
    fp = {}
    for f, gi in enumerate(itf.face_ids):
        if gi in ad["rows"]:
            fp[f"face{f}"] = fingerprint(np.array(ad["rows"][gi]), int(gi))
    edge_rows = {}
    for e, gi in enumerate(itf.edge_ids):
        if gi in ad["rows"]:
            edge_rows[str(e)] = int(len(ad["rows"][gi]))
    out = dict(
        workload=name, n_glob=int(p.n_glob), n_sub=int(p.n_sub), tau=cfg["tau"],
        edge_rows_kept=cfg["edges"],
        counts=dict(itf.counts()), nc_ce=int(cons0.Nc()), nc=int(cons.Nc()),
        n_coarse=int(cn.n), omega=float(ad["omega"]),
        n_selected=int(sum(ad["k"].values())), edge_rows=edge_rows,
        pcg=dict(rtol=RTOL, iters=int(r8["iters"]), kappa=float(r8["kappa"]),
                 lmin=float(r8["lmin"]), lmax=float(r8["lmax"]), relres=float(r8["relres"]),
                 converged=bool(r8["converged"])),
        pcg_ref=dict(rtol=RTOL_REF, iters=int(rr["iters"]), relres=float(rr["relres"]),
                     converged=bool(rr["converged"])),
        r0=r0, true_relres_ref=float(np.linalg.norm(p.f - K @ u) / r0),
        max_rel_diff_1e8_vs_ref=d8,
        faces=faces,
        oracle=dict(wall_s=T, workers=workers, blas_threads=1, nproc=os.cpu_count(),
                    step_s=T["schur_s"] + T["pairs_s"] + T["factor_s"] + T["pcg_s"],
                    step_cpu_s=step_cpu,
                    calibration=dict(task="schur_dense", substructure=cal, seconds=cal_s),
                    cpu=cpu_model(),
                    numpy=np.__version__),
    )
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), u=u, **fp)
    print(f"  wrote {name}.json / .npz", flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    a = ap.parse_args()
    run(a.workload, a.workers)


if __name__ == "__main__":
    main()
