// Adaptive face constraints on the device (Sec. 3, Algorithm 1).
#pragma once

#include <vector>

#include "host.h"
#include "solver.h"

namespace bddc {

struct AdaptState {
  std::vector<std::vector<double>> eigs;  // per face: computed eigenvalues, descending
};

struct AdaptResult {
  double omega = 0;
  int64_t n_added = 0, n_pairs = 0, iters = 0, unconverged = 0;
};

// Solves the face-pair eigenproblems with the current constraints, appends
// the selected rows to P.extra_rows / P.extra_k of every face.
AdaptResult run_adapt(Problem &P, Solver &S, AdaptState &st, double tau);

}  // namespace bddc
