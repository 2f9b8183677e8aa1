// Host-side data of the BDDC library: mesh-derived substructure matrices,
// interface globs, weights and the change of variables.  Built once per
// bddc_setup (and again after bddc_adapt for the constraints).
#pragma once

#include <algorithm>
#include <cstdint>
#include <exception>
#include <string>
#include <thread>
#include <vector>

namespace bddc {

struct MeshIn {
  int kind = 0;  // 0 scalar, 1 elasticity
  int dpn = 1;
  int64_t n_nodes = 0, n_elems = 0;
  std::vector<double> xyz;
  std::vector<int64_t> hex8;
  std::vector<double> coef;
  double nu = 0.3;
  std::vector<uint8_t> dirichlet;
  int n_sub = 0;
  std::vector<int32_t> elem_sub;
};

// Compressed sparse row matrix (local numbering of one substructure).
struct Csr {
  int n = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
};

enum GlobKind { GLOB_EDGE = 1, GLOB_FACE = 2 };

struct Glob {
  int kind = GLOB_EDGE;
  std::vector<int> subs;        // ascending
  std::vector<int64_t> nodes;   // ascending
  std::vector<int64_t> dofs;    // global free dofs, ascending
  std::vector<int> comp;        // component of each dof
};

// QR with column pivoting of a glob's constraint rows H (m x n):
// H = Q [U V] K.  The inverse change of variables T = K^T [U^-1 -U^-1 V; 0 I] K
// in glob-dof positions: the k-th explicit variable lives at glob index
// perm[k]; rows perm[0..m) of T are trow (m x n, row-major), the rest of T is
// the identity.  hrow (m x n) are the explicit variables as functionals of the
// original glob values: wbar[perm[k]] = hrow[k] . w.
struct GlobCov {
  int n = 0, m = 0, dropped = 0;
  std::vector<int> perm;
  std::vector<double> trow;
  std::vector<double> hrow;
};

// Substructure i: local dofs ordered interior first, then interface, each in
// ascending global order.
struct Sub {
  std::vector<int64_t> gdof;     // local -> global free dof
  int nI = 0, nG = 0;
  bool floating = true;          // no Dirichlet dof
  Csr A;                         // local stiffness (SPSD)
  std::vector<double> diag;      // diag(A) per local dof
  std::vector<double> delta;     // weights of E on the interface dofs (nG)
  // globs present in this substructure: glob id and the interface positions
  // (0..nG) of the glob's dofs in glob-dof order
  std::vector<int> glob_ids;
  std::vector<std::vector<int>> glob_pos;
  std::vector<int> corner_pos;   // interface positions of corner dofs
  std::vector<int64_t> corner_gdof;
};

struct Problem {
  MeshIn mesh;
  int64_t n_glob = 0;
  std::vector<int64_t> full2glob;     // n_nodes*dpn -> global free dof or -1
  std::vector<int64_t> glob2full;
  std::vector<Sub> subs;
  std::vector<Glob> globs;
  std::vector<int64_t> corner_nodes;  // ascending (with free dofs)
  std::vector<int64_t> corner_gdofs;  // ascending
  std::vector<int> face_ids, edge_ids;
  // constraints
  int mode = 1;
  double drop_tol = 1e-10;
  bool adapt_edges = false;                      // keep the edge parts of adaptive rows
  std::vector<std::vector<double>> extra_rows;   // per glob: adaptive rows (k x n)
  std::vector<int> extra_k;
  std::vector<GlobCov> cov;
};

// element matrices, substructure assembly (fem.cpp)
void element_matrix(const MeshIn &m, int64_t e, double *K /* (8dpn)^2 */);
void assemble_substructures(Problem &P);

// globs, corners, weights (interface.cpp)
void classify_interface(Problem &P, bool augment);
void compute_weights(Problem &P);

// f(i) for i in [0, n) on up to 16 host threads (i = t, t + nt, ...); the
// first exception a thread throws is rethrown after all have joined
template <class F>
void parallel_for(int n, F f) {
  int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
  nt = std::min(nt, n);
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::exception_ptr> err(nt);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      try {
        for (int i = t; i < n; i += nt) f(i);
      } catch (...) {
        err[t] = std::current_exception();
      }
    });
  for (auto &x : th) x.join();
  for (auto &e : err)
    if (e) std::rethrow_exception(e);
}

// change of variables (qrcp.cpp)
GlobCov qr_change_of_variables(const std::vector<double> &H, int m, int n, double drop_tol);
void build_constraints(Problem &P);
int64_t count_nc(const Problem &P);

}  // namespace bddc
