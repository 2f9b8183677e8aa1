#!/usr/bin/env python3
"""Adaptive BDDC-PCG throughput on one MI355X.

Workload (default, --workload kmeans64): 3D linear elasticity (Q1
hexahedra, 3 dofs per node) on 64^3 elements split by seeded k-means into 64
uneven substructures; E = 1 with 5% of the elements (seeded) at E = 1e5,
nu = 0.3, clamped at z = 0, gravity load; corner and edge-average
constraints plus the adaptive constraints of the face-pair eigenproblems with
tau = 10 (Algorithm 1), the edge parts of the adaptive rows kept as edge rows
(Sec. 3 after Proposition 1); FP64; PCG to a relative residual of 1e-8.
--workload elasticity48: 48^3 elements in 4 x 4 x 4 cubic substructures of
12^3, Young's modulus 1 or 1e6 per horizontal layer (seeded), adaptive face
rows with the edge parts dropped.

One step is one pass of the whole hot path over the problem:
bddc_adapt(tau) (Dirichlet factors, Schur complements, face-pair
eigenproblems, constraint rows) -> bddc_factor (change of variables,
constrained factors, coarse problem) -> bddc_pcg_solve(f).  The problem
(substructure matrices, interface analysis) is set up and resident on the
device before the timed region, and so is the load vector.

The output is one JSON line.  `value` comes from the timed steps, run with
no instrumentation.  `roofline` describes the kernel with the largest summed
time over the same number of steps run again with every launch bracketed by
HIP events on the library's stream; `cpu_baseline` is the FP64 CPU oracle
(its full run on the same workload, scaled to this host by a calibration
task timed here).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TAU = 10.0
RTOL = 1e-8
WORKLOAD_C3 = "elasticity64_kmeans64_inclusions_adaptive_tau10_edge_rows_kept"
WORKLOAD_C2 = "elasticity48_4x4x4_layers_adaptive_tau10"
PEAK_FP64_MFMA = 78.6      # TFLOP/s, MI355X dense FP64 matrix
PEAK_HBM = 8000.0          # GB/s, MI355X HBM3E
# kernels whose work is a dense contraction on the matrix cores
MFMA_KERNELS = ("gemm_kernel", "chol_update_kernel", "chol_panel_kernel", "chol_diag_kernel",
                "chol_syrk_kernel", "trsm_update_kernel<fwd>", "trsm_update_kernel<bwd>",
                "trsm_diag_kernel<fwd>", "trsm_diag_kernel<bwd>", "trsm_gemm_kernel<fwd>",
                "trsm_gemm_kernel<bwd>")
KERNEL_SOURCE = {k: "paper_0910_5863_amd/csrc/dense.hip" for k in MFMA_KERNELS}
KERNEL_SOURCE.update({"trsv_kernel<lower>": "paper_0910_5863_amd/csrc/dense.hip",
                      "trsv_kernel<upper>": "paper_0910_5863_amd/csrc/dense.hip",
                      "mf_fwd_kernel": "paper_0910_5863_amd/csrc/multifrontal.hip",
                      "mf_bwd_kernel": "paper_0910_5863_amd/csrc/multifrontal.hip",
                      "mf_pull_kernel": "paper_0910_5863_amd/csrc/multifrontal.hip",
                      "gemv_t_kernel": "paper_0910_5863_amd/csrc/solver.hip",
                      "symv_kernel": "paper_0910_5863_amd/csrc/solver.hip",
                      "gemv_n_kernel": "paper_0910_5863_amd/csrc/solver.hip",
                      "lobpcg_kernel": "paper_0910_5863_amd/csrc/adapt.hip"})


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    # two untimed steps: with the GEMM tuner on, the step after the tuning
    # step is still about 0.1 s slower than the later ones (as the first
    # adaptive step after setup is without the tuner)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("kmeans64", "elasticity48"), default="kmeans64",
                    help="kmeans64 (default): 64^3 elasticity elements in 64 uneven k-means "
                         "substructures with stiff inclusions, adaptive edge rows kept; "
                         "elasticity48: 48^3 elements in 4x4x4 cubes with layered coefficients")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle sample (about 15 s)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default GEMM tile shapes (the tuner, on by default, "
                         "measures them during the warmup step)")
    ap.add_argument("--factor-precision", type=int, default=64, choices=(32, 64),
                    help="32: FP32 local factor L_rr and local triangular solves (outer PCG, "
                         "coarse problem and averaging stay FP64)")
    ap.add_argument("--per-substructure", action="store_true",
                    help="the unbatched baseline: every dense operation of adapt and factor "
                         "one launch sequence per entry (interior fronts one substructure at a "
                         "time, LOBPCG one face pair per launch), the PCG's Schur products and "
                         "local solves one substructure per launch")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the steps, run one plain device copy of this many MiB "
                         "(a known-size reference for hardware byte counters)")
    ap.add_argument("--serving", type=int, default=0, metavar="N",
                    help="instead of the step benchmark, serve the first N requests of the "
                         "seeded request stream (Poisson arrivals) and report latency")
    ap.add_argument("--serving-rate", type=float, default=8.0, help="arrivals per second")
    ap.add_argument("--serving-workers", type=int, default=4, help="requests in flight at once")
    ap.add_argument("--serving-precision", type=int, default=32, choices=(32, 64))
    ap.add_argument("--serving-problems", type=int, default=0, metavar="K",
                    help="> 0: the stream cycles over its first K problems, each request with "
                         "its own seeded load (a load-case stream on fixed geometries)")
    ap.add_argument("--serving-resident-gib", type=float, default=0.0,
                    help="> 0: keep factored contexts resident up to this many GiB, so that "
                         "requests on a problem already factored only solve")
    ap.add_argument("--variants", choices=("elasticity48", "kmeans64"), default=None,
                    help="instead of the step benchmark, solve the workload once per constraint "
                         "set (c, c+e, c+e+f, 3eigv, adaptive tau with and without edge rows) and "
                         "print one JSON line each: Nc, kappa, iterations, phase times")
    ap.add_argument("--tau-sweep", action="store_true",
                    help="instead of the step benchmark, the 64^3 k-means workload at tau = 2, "
                         "10, 100 with FP64 and FP32 local factors: one JSON line each with "
                         "iterations, kappa, phase times and the error against the FP64 oracle")
    ap.add_argument("--nrhs", type=int, default=0, metavar="K",
                    help="instead of the step benchmark, factor the workload once and solve K "
                         "loads (the mesh's load scaled entrywise by U(0.5, 2), seeded per load) "
                         "one call per load and as one call of K columns (block PCG, 8 columns "
                         "per block): one JSON line with both rates, per-kernel figures of one "
                         "preconditioner application with 1 and with 8 columns, and whether "
                         "every block column has the bits of its single solve")
    ap.add_argument("--planar-cubes", type=int, nargs=2, default=None, metavar=("KMIN", "KMAX"),
                    help="instead of the step benchmark, solve the planar-cubes series (k x k "
                         "substructures of 8^3 elasticity elements, corners only) for k in "
                         "KMIN..KMAX and print one JSON line each")
    return ap.parse_args()


# constraint sets of the variants table: (label, setup mode, adapt call, edges)
VARIANTS = [("c", "c", None, False), ("c+e", "ce", None, False), ("c+e+f", "cef", None, False),
            ("3eigv", "ce", ("count", 3), False), ("adaptive tau=10", "ce", ("tau", 10.0), False),
            ("adaptive tau=10, edge rows kept", "ce", ("tau", 10.0), True),
            ("adaptive tau=2", "ce", ("tau", 2.0), False),
            ("adaptive tau=2, edge rows kept", "ce", ("tau", 2.0), True)]


def variants(args):
    """The structure of the paper's Tables 1/3/5/7 on a synthetic workload:
    one solve per constraint set, with Nc, the Lanczos condition number
    estimate, iterations and phase times (setup, adapt, factor, PCG)."""
    import torch
    import meshgen
    from paper_0910_5863_amd import BDDC
    p = meshgen.elasticity_layers_48() if args.variants == "elasticity48" \
        else meshgen.elasticity_kmeans_64()
    f = torch.from_numpy(p.f).to("cuda:0")
    for label, mode, ad, edges in VARIANTS:
        b = BDDC(device=0)
        t0 = time.perf_counter()
        b.setup(p, mode, adaptive_edges=edges)
        t1 = time.perf_counter()
        ai = None
        if ad is not None:
            ai = b.adapt_count(ad[1]) if ad[0] == "count" else b.adapt(ad[1])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        b.factor()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        u, info = b.pcg_solve(f, rtol=RTOL, maxit=5000, raise_on_fail=False)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        nc = b.info().nc
        b.close()
        del b, u
        torch.cuda.empty_cache()
        print(json.dumps({
            "workload": p.name, "variant": label, "nc": int(nc),
            "omega": None if ai is None else float(ai.omega),
            "edge_rows": None if ai is None else int(ai.n_added_edge),
            "kappa": float(info[0].kappa), "iters": int(info[0].iters),
            "converged": bool(info[0].converged), "setup_s": t1 - t0, "adapt_s": t2 - t1,
            "factor_s": t3 - t2, "pcg_s": t4 - t3}), flush=True)


# the weak-scaling series of Table 9 (SGI Altix 4700, MUMPS, one processor per
# substructure): substructures, dofs, condition number, iterations, MUMPS
# analysis s, factorization s, PCG s; printed beside each result as context
TABLE9 = {2: (4, 7803, 28.3, 13, 0.2, 0.5, 0.8), 3: (9, 16875, 38.0, 26, 0.5, 0.4, 3.6),
          4: (16, 29403, 42.2, 36, 1, 0.8, 13), 5: (25, 45387, 44.4, 42, 15, 12, 613),
          6: (36, 64827, 45.7, 44, 14, 10, 524), 7: (49, 87723, 46.5, 46, 16, 12, 579),
          8: (64, 114075, 47.1, 47, 19, 14, 643)}


def planar_cubes(args):
    """Planar-cubes weak scaling on one GPU: k x k substructures of 8^3
    elasticity elements, corners only.  Setup (host analysis and upload),
    factor and PCG solve are timed; factor + solve run three times and the
    median is reported."""
    import numpy as np
    import torch
    import meshgen
    from paper_0910_5863_amd import BDDC
    for k in range(args.planar_cubes[0], args.planar_cubes[1] + 1):
        p = meshgen.planar_cubes(k)
        f = torch.from_numpy(p.f).to("cuda:0")
        b = BDDC(device=0)
        t0 = time.perf_counter()
        b.setup(p, "c")
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        tf, ts = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            b.factor()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            u, info = b.pcg_solve(f, rtol=RTOL, maxit=2000)
            torch.cuda.synchronize()
            tf.append(t1 - t0)
            ts.append(time.perf_counter() - t1)
        i = b.info()
        b.close()
        del b, u
        torch.cuda.empty_cache()
        it = int(info[0].iters)
        ctx = TABLE9.get(k)
        print(json.dumps({
            "workload": p.name, "k": k, "n_sub": int(p.n_sub), "dofs_all": int(p.n_nodes * 3),
            "n_glob": int(p.n_glob), "nc": int(i.nc), "n_coarse": int(i.n_coarse),
            "kappa": float(info[0].kappa), "iters": it, "setup_s": t_setup,
            "factor_s": float(np.median(tf)), "pcg_s": float(np.median(ts)),
            "ms_per_iteration": float(np.median(ts)) / max(it, 1) * 1e3,
            "paper_table9": None if ctx is None else dict(zip(
                ("n_sub", "dofs", "kappa", "iters", "analysis_s", "factorization_s", "pcg_s"), ctx)),
        }), flush=True)


def tau_sweep(args):
    """Precision and tau on the 64^3 k-means workload (edge rows kept): for
    tau in {2, 10, 100} and FP64 / FP32 local factors, a fresh context, one
    untimed adapt + factor + solve (GEMM tuning), then the timed one.  The
    error is max |u - u_oracle| / max |u_oracle| against the oracle's solution
    of the same system (tests/golden/kmeans64.npz; the solution does not
    depend on tau or on the preconditioner)."""
    import numpy as np
    import torch
    import meshgen
    from paper_0910_5863_amd import BDDC
    p = meshgen.elasticity_kmeans_64()
    uref = np.load(os.path.join(ROOT, "tests", "golden", "kmeans64.npz"))["u"]
    f = torch.from_numpy(p.f).to("cuda:0")
    for tau in (2.0, 10.0, 100.0):
        for prec in (64, 32):
            b = BDDC(device=0, autotune=True, factor_precision=prec)
            b.setup(p, "ce", adaptive_edges=True)
            for rep in range(2):
                t0 = time.perf_counter()
                ai = b.adapt(tau)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                b.factor()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                u, info = b.pcg_solve(f, rtol=RTOL, maxit=3000)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
            uu = u.cpu().numpy()[:, 0]
            i = b.info()
            b.close()
            del b, u
            torch.cuda.empty_cache()
            print(json.dumps({
                "workload": WORKLOAD_C3, "tau": tau, "factor_precision": prec, "nc": int(ai.nc),
                "omega": float(ai.omega), "iters": int(info[0].iters), "kappa": float(info[0].kappa),
                "true_relres": float(info[0].true_relres), "fp32_fallbacks": int(i.fp32_fallbacks),
                "max_rel_error_vs_oracle": float(np.abs(uu - uref).max() / np.abs(uref).max()),
                "adapt_s": t1 - t0, "factor_s": t2 - t1, "pcg_s": t3 - t2, "step_s": t3 - t0}),
                flush=True)


def serving(args):
    """Requests from the seeded stream (Poisson or elasticity cubes of
    16^3-48^3 elements in 8-64 substructures, layered contrast 1-1e6), each a
    full adapt(tau = 10) + factor + PCG solve, submitted at seeded Poisson
    arrival times to the request server; one JSON line with throughput and
    arrival-to-result latency percentiles."""
    import numpy as np
    import meshgen
    from paper_0910_5863_amd import Server
    K = args.serving_problems
    reqs = meshgen.serving_requests(max(args.serving, 512))[:(K if K > 0 else args.serving)]
    probs = [meshgen.request_problem(r) for r in reqs]  # generated before the clock starts
    if K > 0:
        # request i: problem i mod K, load scaled entrywise by U(0.5, 2) drawn from seed i
        loads = [probs[i % K].f * np.random.default_rng(i).uniform(0.5, 2.0, probs[i % K].f.shape)
                 for i in range(args.serving)]
        probs = [probs[i % K] for i in range(args.serving)]
    else:
        loads = [None] * len(probs)
    gaps = np.random.default_rng(7).exponential(1.0 / args.serving_rate, len(probs))
    srv = Server(max_active=args.serving_workers, factor_precision=args.serving_precision,
                 resident_bytes=args.serving_resident_gib * 2.0**30)
    t0 = time.perf_counter()
    ids = []
    for p, f, t in zip(probs, loads, np.cumsum(gaps)):
        delay = t0 + t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(p, 10.0, f=f))
    res = [srv.wait(i)[1] for i in ids]
    elapsed = time.perf_counter() - t0
    srv.close()
    failed = [r.error.decode() for r in res if r.state != 2]
    lat = np.array([r.done_s - r.submit_s for r in res])
    queue = np.array([r.start_s - r.submit_s for r in res])
    iters = np.array([r.pcg.iters for r in res])
    print(json.dumps({
        "metric": "serving: solves/s and arrival-to-result latency",
        "value": len(res) / elapsed, "unit": "solves/s", "n_gpus": 1,
        "requests": len(res), "failed": len(failed), "errors": failed[:3],
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "p50_queue_s": float(np.percentile(queue, 50)), "max_queue_s": float(queue.max()),
        "arrival_rate_per_s": args.serving_rate, "workers": args.serving_workers,
        "factor_precision": args.serving_precision, "pcg_iters_median": float(np.median(iters)),
        "reused": int(sum(r.reused for r in res)),
        "elapsed_s": elapsed, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": "serving_request_stream_seed5", "tau": 10.0, "rtol": 1e-8,
                   "problems": K if K > 0 else len(reqs),
                   "resident_gib": args.serving_resident_gib},
    }))


def multi_rhs(args):
    """K loads on one factored problem: one solve per call against one call
    with K columns (blocks of 8 solved by a lock-step block PCG, every factor
    read once per application for the block)."""
    import numpy as np
    import torch
    import meshgen
    from paper_0910_5863_amd import BDDC
    K = args.nrhs
    c3 = args.workload == "kmeans64"
    p = meshgen.elasticity_kmeans_64() if c3 else meshgen.elasticity_layers_48()
    b = BDDC(device=0, autotune=not args.no_autotune, factor_precision=args.factor_precision)
    b.setup(p, "ce", adaptive_edges=c3)
    b.adapt(TAU)
    b.factor()
    F = np.stack([p.f * np.random.default_rng(100 + j).uniform(0.5, 2.0, p.f.shape)
                  for j in range(K)], axis=1)
    Fd = torch.from_numpy(F).to("cuda:0")
    cols = [Fd[:, j].contiguous() for j in range(K)]
    b.pcg_solve(cols[0])  # warm: graphs of the single iteration
    b.pcg_solve(Fd[:, :min(K, 8)])  # and of the block widths used
    if K % 8:
        b.pcg_solve(Fd[:, :K % 8])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles = [b.pcg_solve(c) for c in cols]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    t0 = time.perf_counter()
    Ub, infos = b.pcg_solve(Fd)
    torch.cuda.synchronize()
    t_block = time.perf_counter() - t0
    Ub = Ub.cpu().numpy()
    same = all(np.array_equal(Ub[:, j], singles[j][0].cpu().numpy()[:, 0]) and
               infos[j].iters == singles[j][1][0].iters for j in range(K))
    # one preconditioner application with 1 and with 8 columns, every launch
    # timed with HIP events on the library's stream
    per = {}
    R = torch.from_numpy(np.stack([p.f] * 8, axis=1)).to("cuda:0")
    for m in (1, 8):
        b.apply(R[:, :m])
        torch.cuda.synchronize()
        b.set_timing(2)
        b.apply(R[:, :m])
        torch.cuda.synchronize()
        st = b.timing()
        b.set_timing(0)
        per[m] = {k: {"ms": v["ms"], "GB/s": v["bytes"] / (v["ms"] / 1e3) / 1e9 if v["ms"] > 0 else None,
                      "launches": v["launches"]}
                  for k, v in sorted(st.items(), key=lambda kv: -kv[1]["ms"])[:8]}
    it = [int(i.iters) for i in infos]
    print(json.dumps({
        "metric": "BDDC-PCG solves/s to 1e-8 rel. residual, K loads on one factored problem",
        "value": K / t_block, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "nrhs": K, "block_width": 8,
        "single_calls_solves_per_s": K / t_single, "speedup": t_single / t_block,
        "block_columns_bitwise_equal_to_single_solves": bool(same),
        "iters_min": min(it), "iters_max": max(it),
        "apply_kernels_1_column": per[1], "apply_kernels_8_columns": per[8],
        "dtype": "f64" if args.factor_precision == 64 else "f32+f64", "data": "synthetic",
        "config": {"workload": WORKLOAD_C3 if c3 else WORKLOAD_C2, "n_glob": int(p.n_glob),
                   "tau": TAU, "rtol": RTOL,
                   "loads": "f * U(0.5, 2) entrywise, seeds 100..100+K-1",
                   "timed": "pcg_solve only (adapt and factor once before)"},
    }), flush=True)
    b.close()


def source_sha(rel):
    with open(os.path.join(ROOT, rel), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(kernel, tag):
    """Per-launch HBM bytes of `kernel` from the committed counter summary
    (profiles/traffic_<kernel>_<tag>.txt: FETCH_SIZE + WRITE_SIZE per dispatch,
    scaled by a copy kernel of known size), or None when there is none or the
    kernel's source changed since the counters were taken."""
    safe = kernel.replace("<", "_").replace(">", "")
    path = os.path.join(ROOT, "profiles", f"traffic_{safe}_{tag}.txt")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCE:
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_sha(KERNEL_SOURCE[kernel]):
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(workload):
    """The FP64 CPU oracle on this workload.  The oracle's full run (Schur
    complements, every face-pair eigenproblem, Algorithm 2 by blocks, PCG to
    1e-8) on the whole mesh was timed when its reference results were written
    (tests/golden/<workload>.json: wall time with its worker processes, CPU
    time summed over them, and one calibration task).  Here, on this host, the
    calibration task alone is the sample: one substructure's dense Schur
    complement on one thread.  The ratio of the two calibration times scales
    the recorded full run to this host."""
    import meshgen
    from threadpoolctl import threadpool_limits
    from oracle.fem import Substructures
    from oracle.interface import Interface
    from oracle.adapt import schur_dense
    with open(os.path.join(ROOT, "tests", "golden", f"{workload}.json")) as fh:
        g = json.load(fh)
    o = g["oracle"]
    cal = o["calibration"]
    p = meshgen.elasticity_kmeans_64() if workload == "kmeans64" else meshgen.elasticity_layers_48()
    S = Substructures(p)
    itf = Interface(S)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        schur_dense(S, itf, cal["substructure"])
        t = time.perf_counter() - t0
    ratio = t / cal["seconds"]
    step = o["step_s"] * ratio
    return {"value": 1.0 / step, "unit": "solves/s", "cores": int(o["workers"]), "kind": "oracle",
            "sample": (f"calibration task on this host: the dense Schur complement of substructure "
                       f"{cal['substructure']} on one thread, {t:.2f} s against {cal['seconds']:.2f} s "
                       f"on the host of the oracle's full run ({o['cpu']}, {o['workers']} worker "
                       f"processes, one BLAS thread each); that run's step of {o['step_s']:.0f} s "
                       f"(adapt, factor, PCG to 1e-8 in {g['pcg']['iters']} iterations) is scaled "
                       f"by the ratio {ratio:.3f}"),
            "value_1core": 1.0 / (o["step_cpu_s"] * ratio),
            "sample_seconds": t}


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sharding the substructures across GPUs is designed, not implemented)",
              file=sys.stderr)
        sys.exit(2)
    if args.serving > 0:
        serving(args)
        return
    if args.variants or args.planar_cubes or args.tau_sweep or args.nrhs > 0:
        import torch
        if not torch.cuda.is_available():
            print("bench.py: no GPU visible", file=sys.stderr)
            sys.exit(1)
        if args.nrhs > 0:
            multi_rhs(args)
        elif args.tau_sweep:
            tau_sweep(args)
        elif args.variants:
            variants(args)
        else:
            planar_cubes(args)
        return
    import numpy as np
    import torch
    import meshgen
    from paper_0910_5863_amd import BDDC

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    c3 = args.workload == "kmeans64"
    p = meshgen.elasticity_kmeans_64() if c3 else meshgen.elasticity_layers_48()
    b = BDDC(device=0, autotune=not args.no_autotune, factor_precision=args.factor_precision,
             per_substructure_launches=args.per_substructure)
    b.setup(p, "ce", adaptive_edges=c3)
    f = torch.from_numpy(p.f).to("cuda:0")
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(phases):
        t0 = time.perf_counter()
        ai = b.adapt(TAU)
        t1 = time.perf_counter()
        b.factor()
        t2 = time.perf_counter()
        u, info = b.pcg_solve(f, rtol=RTOL, maxit=1000)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        if not info[0].converged:
            raise RuntimeError("PCG did not converge")
        if ai.unconverged:
            raise RuntimeError(f"{ai.unconverged} face-pair eigenproblems did not converge")
        phases.append((t1 - t0, t2 - t1, t3 - t2))
        return ai, info[0]

    warm = []
    for _ in range(args.warmup):
        step(warm)
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ai, pinfo = step(phases)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # per-kernel figures: the same steps again with every launch bracketed by
    # HIP events on the library's stream (PCG iterations then run launch by
    # launch instead of as graph replays, so this pass is not the one timed)
    b.set_timing(2)
    kphases = []
    for _ in range(args.steps):
        step(kphases)
    torch.cuda.synchronize()
    stats = b.timing()
    b.set_timing(0)

    # dominant kernel and its roofline
    name, st = max(stats.items(), key=lambda kv: kv[1]["ms"])
    avg_s = st["ms"] / st["launches"] / 1e3
    if name in MFMA_KERNELS:
        achieved = st["flops"] / st["launches"] / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_MFMA}
    else:
        achieved = st["bytes"] / st["launches"] / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM, "unit": "GB/s",
                "frac": achieved / PEAK_HBM}
    roof["traffic"] = measured_traffic(name, args.workload)
    roof["kernel"] = name
    roof["launches"] = st["launches"]
    roof["avg_launch_us"] = avg_s * 1e6
    roof["algorithmic_bytes_per_launch"] = st["bytes"] / st["launches"]
    roof["algorithmic_flops_per_launch"] = st["flops"] / st["launches"]
    top = sorted(stats.items(), key=lambda kv: -kv[1]["ms"])[:16]
    kernels = []
    for k, v in top:
        s_ = v["ms"] / 1e3
        kernels.append({"kernel": k, "ms_per_step": v["ms"] / args.steps, "launches_per_step":
                        v["launches"] / args.steps,
                        "TFLOP/s": v["flops"] / s_ / 1e12 if s_ > 0 else None,
                        "GB/s": v["bytes"] / s_ / 1e9 if s_ > 0 else None})

    ms_per_step = elapsed / args.steps * 1e3
    ph = np.array(phases)
    i = b.info()
    out = {
        "metric": "BDDC-PCG solves/s to 1e-8 rel. residual",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.factor_precision == 64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": (WORKLOAD_C3 if c3 else WORKLOAD_C2), "n_glob": int(p.n_glob),
                   "n_sub": int(p.n_sub), "tau": TAU, "rtol": RTOL,
                   "step": "adapt(tau) + factor + pcg_solve(f), problem set up and resident",
                   "gemm_autotune": not args.no_autotune,
                   "factor_precision": args.factor_precision,
                   "launches": "per_substructure" if args.per_substructure else "batched"},
        "roofline": roof,
        "phases_ms": {"adapt": float(ph[:, 0].mean() * 1e3), "factor": float(ph[:, 1].mean() * 1e3),
                      "pcg_solve": float(ph[:, 2].mean() * 1e3)},
        "resident_solves_per_s": float(1.0 / ph[:, 2].mean()),
        "pcg_iters": int(pinfo.iters),
        "kappa": float(pinfo.kappa),
        "omega": float(ai.omega),
        "nc": int(ai.nc),
        "factor_flops_executed": float(i.factor_flops),
        "device_gb": i.device_bytes / 1e9,
        "kernels": kernels,
        "cpu_baseline": None,
    }
    del b
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
