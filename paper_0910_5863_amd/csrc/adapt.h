// Adaptive face constraints on the device (Sec. 3, Algorithm 1).
#pragma once

#include <vector>

#include "host.h"
#include "solver.h"

namespace bddc {

// One face pair (i, j) reduced to the jump space on the shared non-corner
// dofs (structure only; built from the setup data).
struct AdaptPair {
  int f = 0, gi = 0, sub[2] = {0, 0};
  std::vector<int> pos_s[2], pos_n[2];  // interface positions: shared, not shared
  std::vector<int> cidx;                // shared-list indices of the non-corner dofs
  std::vector<double> wi;               // renormalized weight of side i on every c dof
  std::vector<double> Q;                // rigid traces on s (n_s x nq, orthonormal columns)
  int nq = 0;
  double rho = 0;
  int d = 0;                            // dimension of the jump space
  std::vector<int> zptr, zrow;          // Z (n_c x d) by columns: rows and values
  std::vector<double> zval;
  std::vector<int> face_c;              // c-indices of the face glob dofs (glob order)
  std::vector<int> edge_gi;             // edge globs of the face's closure (ascending)
  std::vector<std::vector<int>> edge_c; // their c-indices (glob order)
};

struct AdaptState {
  std::vector<std::vector<double>> eigs;  // per face: computed eigenvalues, descending
  std::vector<AdaptPair> pairs;
  bool pairs_ready = false;
};

struct AdaptResult {
  double omega = 0;
  int64_t n_added = 0, n_added_edge = 0, n_pairs = 0, iters = 0, unconverged = 0;
};

// Solves the face-pair eigenproblems with the current constraints and
// appends the selected rows to P.extra_rows / P.extra_k of every face (and of
// the edges of its closure when P.adapt_edges).  count == 0 selects the
// eigenvalues >= tau; count > 0 the count dominant ones of every face.
AdaptResult run_adapt(Problem &P, Solver &S, AdaptState &st, double tau, int count = 0);

}  // namespace bddc
