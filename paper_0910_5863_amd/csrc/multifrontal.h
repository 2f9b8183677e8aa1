// Multifrontal elimination of the substructure interiors.
//
// Every substructure's interior dofs are ordered by geometric nested
// dissection of its interior nodes (recursive bisection at the median
// coordinate of the longest extent; the separator is the side of the cut
// adjacent to the other side).  Each separator (or leaf set) is one front:
// p pivot dofs and the b boundary dofs the eliminated subtree couples to
// (separators of ancestors and interface dofs).  Eliminating the front's
// pivots leaves the b x b contribution block, which the parent front (or, at
// the top, the interface Schur complement) pulls in.  So the interface Schur
// complement S_i = A_GG - A_GI A_II^-1 A_IG of Sec. 2 is produced without a
// dense A_II factor, and the interior Dirichlet solves A_II^-1 of the
// harmonic extension (Sec. 2, (I - P)) run front by front.
//
// Storage per front: U = [F11 | F12] (p x f, column-major, ld p) becomes
// [L11 | L11^-1 F12] after the partial factorization; C (b x b, ld b, lower
// triangle) is the contribution block.  Fronts of the same depth over all
// substructures form one batch.
#pragma once

#include <cstdint>
#include <vector>

#include "dense.h"
#include "device.h"
#include "host.h"

namespace bddc {

struct MfFront {
  int sub = 0;
  int depth = 1;         // 1: child of the interface root
  int p = 0, b = 0;      // pivots, boundary; f = p + b
  int parent = -1;       // parent front, -1 for the interface root
  int64_t u_off = 0;     // p x f block in the U pool
  int64_t c_off = 0;     // b x b block in the C pool
  int64_t piv_off = 0;   // p entries in piv: interior stack indices
  int64_t bnd_off = 0;   // b entries in bnd: interior stack index, or -1 (interface)
  int64_t upd_off = 0;   // b entries of the solve's update pool
  int64_t pmap_off = 0;  // f_parent entries (n_G for the root): parent index -> own boundary index or -1
  int child_ptr = 0;     // children: child_ids[child_ptr .. child_ptr + n_child)
  int n_child = 0;
};

struct MfSymbolic {
  std::vector<MfFront> fronts;
  std::vector<int> child_ids;
  std::vector<int64_t> piv, bnd;   // stack indices (bnd: -1 for interface vars)
  std::vector<int> pmap;
  // top fronts (children of the interface root) per substructure
  std::vector<int> root_ptr, root_ids;
  // CSR entries of interior rows: destination in the U pool (-1: skip)
  std::vector<int64_t> asm_dst;
  int64_t u_size = 0, c_size = 0, upd_size = 0;
  int max_depth = 0;
  int max_p = 0, max_b = 0;
  double flops = 0;                // partial factorizations, all fronts
  double l_entries = 0;            // stored factor entries (sum p*p/2 + p*b)
  std::vector<std::vector<int>> levels;  // front ids per depth (index = depth)
};

// Nested dissection and front structure of every substructure's interior.
// offI: stack offset of each substructure's interior dofs.  Leaves hold at
// most leaf_nodes mesh nodes.
MfSymbolic mf_analyze(const Problem &P, const std::vector<int64_t> &offI, int leaf_nodes = 48);

// Device side: the symbolic structure, the factor pools and the batched
// factorization and solves.
class MfDevice {
 public:
  MfSymbolic sym;
  bool ready = false;
  // analysis and upload (the structure depends on the mesh and partition only)
  void setup(const Problem &P, const std::vector<int64_t> &offI, DevAlloc &A, hipStream_t st);
  void release(DevAlloc &A);
  // U, C <- partial factorizations of all fronts from the substructure CSR
  // values (val, in the stacked CSR order of the analysis); S (interface
  // Schur complements, per substructure n_G x n_G at offGG, holding A_GG) +=
  // the top contributions, lower triangle.  Throws on a non-positive pivot.
  void factor(hipStream_t st, const double *val, int64_t nnz, double *S, const int64_t *offGG,
              const int *nG, int max_nG, int nsub);
  // vI <- A_II^-1 vI on the stack of interiors, every substructure
  // interior solves in place, for m <= kMaxCols columns (column q at
  // vI + q ldI); upd / zp: work vectors of m upd_elems() and m zp_elems()
  // doubles (nullptr: the object's own).  A column gets the same bits for
  // every m.
  static constexpr int kMaxCols = 8;
  void solve(hipStream_t st, double *vI, double *upd = nullptr, double *zp = nullptr, int m = 1,
             int64_t ldI = 0);
  int64_t upd_elems() const { return upd_n_; }  // per column
  int64_t zp_elems() const { return zp_n_; }
  size_t bytes() const;

 private:
  DBuf d_fronts_, d_child_, d_piv_, d_bnd_, d_pmap_, d_asm_, d_root_ptr_, d_root_ids_;
  DBuf d_U_, d_C_, d_upd_, d_status_, d_level_ids_;
  std::vector<int64_t> level_off_;                 // into d_level_ids_ per depth
  std::vector<std::vector<MatDesc>> h_potrf_, h_trsm_;
  std::vector<std::vector<GemmDesc>> h_gemm_;
  std::vector<DBuf> d_potrf_, d_trsm_, d_gemm_;
  DBuf d_dinv_;                                    // inverses of the L11 diagonal blocks
  std::vector<DBuf> d_dinv_off_, d_dinv_toff_;     // per depth: for the potrf / trsm entries
  DBuf d_dinv_front_;                              // per front: offset of its inverses
  std::vector<int64_t> max_f_;                     // per depth: max p*f + b*b
  // per depth: block offsets of the extend-add launch over the depth's
  // fronts (each front its own blocks), host copy and device copy
  std::vector<std::vector<int64_t>> h_pull_off_;
  std::vector<DBuf> d_pull_off_;
  std::vector<int> max_pb_;                        // per depth: max p + b
  std::vector<int> max_p_, max_b_;                 // per depth: max p, max b
  DBuf d_zp_;                                      // solves: z of every front's pivots
  // per depth and substructure: [begin, end) of its fronts in the level list,
  // in the potrf entries and in the trsm / gemm entries (fronts of a depth
  // are ordered by substructure); used by the unbatched launches
  std::vector<std::vector<int>> lvl_lo_, pot_lo_, trs_lo_;
  int nsub_ = 0;
  int64_t nnz_ = 0;
  int64_t upd_n_ = 1, zp_n_ = 1;  // solve work per column
};

}  // namespace bddc
