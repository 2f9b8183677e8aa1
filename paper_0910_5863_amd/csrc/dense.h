// Batched dense linear algebra on gfx950 for the per-substructure factors:
// MFMA GEMM, left-looking blocked Cholesky, multi-right-hand-side triangular
// solves, and a flag-synchronized blocked triangular solve for few
// right-hand sides.  All matrices are column-major; every batch entry has its
// own sizes and leading dimensions.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace bddc {

constexpr int NB = 64;  // block size of the blocked factorizations and solves

// Per-launch timing.  When a LaunchTiming is installed for the calling
// thread, every kernel launch of the library is bracketed by events under its
// kernel name, with the algorithmic bytes and flops of that launch.
struct LaunchTiming {
  virtual void launch_begin(hipStream_t st, const char *kernel, double bytes, double flops) = 0;
  virtual void launch_end(hipStream_t st) = 0;
  // sets the work of the last timed launch (when it is known only afterwards)
  virtual void launch_amend(double bytes, double flops) = 0;
  virtual ~LaunchTiming() = default;
};
LaunchTiming *&launch_timing();  // the calling thread's slot (nullptr: off)

// GEMM tile autotuning.  When on for the calling thread, the first
// DenseOps::gemm call of each shape signature (element type, transposes,
// lower, batch size, largest M, N and K) times every tile shape whose result
// is bitwise the default one's, and that signature uses the fastest from
// then on (a table shared by the process).  Calls under stream capture use
// the table but never tune.
bool &autotune_enabled();   // the calling thread's switch (default off)

// Unbatched launches (the per-substructure baseline).  When on for the
// calling thread, every DenseOps call with more than one entry runs as one
// launch sequence per entry, the same operations entry by entry, and the GEMM
// tuner is not consulted.  Callers that batch by a coarser unit (the fronts
// of one substructure) switch it off around their calls (PerEntryOff).
bool &per_entry_launches();  // the calling thread's switch (default off)
struct PerEntryOff {
  bool saved;
  PerEntryOff() : saved(per_entry_launches()) { per_entry_launches() = false; }
  ~PerEntryOff() { per_entry_launches() = saved; }
};
int64_t autotune_entries();  // signatures tuned so far in this process

// The fused Cholesky.  When a workspace allocator is set for the calling
// thread (and per_entry_launches is off), DenseOps::potrf factors a batch of
// at most fused_max_tasks() tile tasks in one launch: the steps of the
// blocked factorization become tasks handed out by a ticket counter, each
// entry's tasks waiting on device-side counters of that entry only, so
// entries no longer wait for each other at every step and no launch gaps
// separate the steps.  Bitwise the same factor as one launch per step.  The
// plan and counters live in memory from the workspace for the duration of the
// call (which synchronizes the stream once).  Larger batches, or no
// workspace, run one launch per step: there the per-task start (ticket,
// decode, wait) costs more than the launch gaps it saves (measured at the
// 64^3 size: 64 K_rr of 2.6k-7.5k, 345k tasks, 64.4 ms fused against 57.0 ms
// per step; batches up to about 30k tasks are faster fused).
constexpr int64_t kFusedAutoTasks = 40000;
struct DevAlloc;
DevAlloc *&fused_workspace();  // the calling thread's slot (default nullptr)
int64_t &fused_max_tasks();    // the calling thread's limit (default kFusedAutoTasks)

struct LaunchScope {
  hipStream_t st;
  LaunchTiming *t;
  LaunchScope(hipStream_t s, const char *kernel, double bytes, double flops)
      : st(s), t(launch_timing()) {
    if (t) t->launch_begin(st, kernel, bytes, flops);
  }
  ~LaunchScope() {
    if (t) t->launch_end(st);
  }
  LaunchScope(const LaunchScope &) = delete;
  LaunchScope &operator=(const LaunchScope &) = delete;
};

// One batch entry: an n x n lower-triangular factor (or SPD matrix) at
// pool + a_off with leading dimension lda, and an n x nrhs right-hand side at
// pool + b_off with leading dimension ldb.
struct MatDesc {
  int64_t a_off;
  int64_t b_off;
  int n;
  int nrhs;
  int lda;
  int ldb;
};

// General batched GEMM descriptor: C = beta C + alpha op(A) op(B),
// op(A) is M x K, op(B) is K x N.
struct GemmDesc {
  int64_t a_off, b_off, c_off;
  int M, N, K;
  int lda, ldb, ldc;
};

template <class T>
struct DenseOps {
  // C = beta*C + alpha*op(A)*op(B) for every entry; lower != 0 computes only
  // tiles that intersect the lower triangle (i >= j).
  // h_desc (optional) is the host copy of the descriptors, used only to count
  // the launch's flops and bytes when per-launch timing is on.
  static hipError_t gemm(hipStream_t st, const T *A, const T *B, T *C, const GemmDesc *d_desc,
                         int batch, int maxM, int maxN, bool transA, bool transB, T alpha,
                         T beta, bool lower, const GemmDesc *h_desc = nullptr);
  // C[map(i), j] += (A B^T)[i, j] (map_rows) or C[i, map(j)] += (A B^T)[i, j]
  // for every entry (op(A) = A, op(B) = B^T), where map(x) =
  // map[map_off[e] + x]: a product added into scattered rows or columns of C
  // (every mapped row or column distinct within an entry).
  static hipError_t gemm_scatter(hipStream_t st, const T *A, const T *B, T *C,
                                 const GemmDesc *d_desc, const int *map, const int64_t *map_off,
                                 bool map_rows, int batch, int maxM, int maxN,
                                 const GemmDesc *h_desc = nullptr);
  // In-place lower Cholesky of every entry's A (n x n).  status[e] is set to
  // (column+1) of the first non-positive pivot (left untouched if none).  The
  // inverses of the NB x NB diagonal blocks of L are written to dinv: block
  // kb of entry e at dinv + dinv_off[e] + kb NB^2 (column-major, ld NB; size
  // from dinv_layout).
  static hipError_t potrf(hipStream_t st, T *pool, const MatDesc *d_desc, const MatDesc *h_desc,
                          int batch, int *status, T *dinv, const int64_t *dinv_off);
  // B <- L^{-1} B (forward) or L^{-T} B (backward), L the lower factor at a_off
  // with the inverses of its diagonal blocks in dinv (as written by potrf).
  static hipError_t trsm(hipStream_t st, T *pool_a, T *pool_b, const MatDesc *d_desc,
                         const MatDesc *h_desc, int batch, bool transpose, const T *dinv,
                         const int64_t *dinv_off);
};

// Copy the lower triangle onto the upper one (entries A at a_off, n x n).
// h_desc (optional): the host copy of the descriptors; with it only each
// entry's own tiles are launched.
template <class T>
hipError_t symmetrize_lower(hipStream_t st, T *pool, const MatDesc *d_desc, int batch, int maxn,
                            const MatDesc *h_desc = nullptr);

// Triangular solves with per-block completion flags (one launch per solve,
// all entries together): x <- L^{-1} x for a lower triangular L (upper =
// false) or x <- U^{-1} x for an upper triangular U (upper = true), both
// column-major at a_off with leading dimension lda; x at xpool + b_off, with
// m right-hand sides (1 <= m <= kTrsvMaxCols) at column stride ldx, which
// share every load of the factor.  A column gets the same bits for every m.
// L^{-T} x is the upper solve with U = L^T (transpose_batched).  work must
// hold 1 + sum over entries of ceil(n/NB) ints; it is cleared by the call.
// err receives 1 if a wait bound is exceeded.
constexpr int kTrsvMaxCols = 8;
struct TrsvPlan {
  int batch = 0;
  int total_blocks = 0;
  int *d_order_fwd = nullptr;  // (entry, block) pairs in dependency order
  int *d_order_bwd = nullptr;
  int *d_flag_off = nullptr;   // first flag of every entry
  double tri_elems = 0;        // sum over entries of n (n + 1) / 2 (for timing)
  double rows = 0;             // sum over entries of n
};

// dinv / dinv_off: inverses of the NB x NB diagonal blocks of L (diag_inverse;
// the same arrays serve the upper solve with U = L^T).
template <class T>
hipError_t trsv_blocked(hipStream_t st, const T *apool, T *xpool, const MatDesc *d_desc,
                        const TrsvPlan &plan, bool upper, const T *dinv, const int64_t *dinv_off,
                        int *work, int *err, int m = 1, int64_t ldx = 0);

// Offsets of the diagonal-block inverses of entries of sizes n (one NB x NB
// block per NB rows); returns the total number of elements.
inline int64_t dinv_layout(const MatDesc *h_desc, int batch, std::vector<int64_t> &off) {
  off.resize(batch);
  int64_t t = 0;
  for (int e = 0; e < batch; ++e) {
    off[e] = t;
    t += (int64_t)((h_desc[e].n + NB - 1) / NB) * NB * NB;
  }
  return t;
}

// Inverses of the NB x NB diagonal blocks of every entry's lower triangular
// factor (a_off, n, lda of d_desc): block kb of entry e at
// inv + inv_off[e] + kb NB^2, column-major with ld NB.
template <class T>
hipError_t diag_inverse(hipStream_t st, const T *pool, const MatDesc *d_desc, int batch, int maxn,
                        T *inv, const int64_t *inv_off);

// B <- A^T for every entry (n x n matrices: A at a_off, lda; B at b_off, ldb);
// h_desc (optional) as for symmetrize_lower
template <class T>
hipError_t transpose_batched(hipStream_t st, const T *apool, T *bpool, const MatDesc *d_desc,
                             int batch, int maxn, const MatDesc *h_desc = nullptr);

// Host: ticket orders for entries of sizes n (forward: block index upwards,
// backward: downwards, level by level across entries) and flag offsets.
void make_trsv_orders(const std::vector<int> &n, std::vector<int> &fwd, std::vector<int> &bwd,
                      std::vector<int> &flag_off, int &total);

}  // namespace bddc
