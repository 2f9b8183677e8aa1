"""Plain FP64 CPU oracle of adaptive BDDC (Mandel, Sousedik, Sistek, "Adaptive
BDDC in Three Dimensions").

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links anything under ``oracle/``; only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library: it has its own assembly, interface classification, change of
variables, preconditioner, PCG and eigen-solves, written from the paper in
NumPy/SciPy double precision, slow and literal on purpose.

Modules:
  fem         Q1 element matrices, substructure matrices A_i (Sec. 2)
  interface   faces / edges / corners, weights of the averaging E (Sec. 2, 7)
  cov         averages H^avg, QR with column pivoting, T_i (Sec. 5, eq. (T))
  bddc        Algorithm 2 with global sparse matrices; Lemma 1 and the
              Pi-projected system as cross-checks (Sec. 2, 4, 5)
  pcg         PCG on the reduced problem and the Lanczos condition estimate
  adapt       face-pair generalized eigenproblems, Algorithm 1 (Sec. 3)
"""
