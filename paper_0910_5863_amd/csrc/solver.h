// Device solver of one BDDC problem (see solver.hip for the formulation).
#pragma once

#include <stdexcept>
#include <string>
#include <vector>

#include "device.h"
#include "host.h"
#include "multifrontal.h"

namespace bddc {

struct BddcError : std::runtime_error {
  int code;
  BddcError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};
struct ArgError : BddcError {
  explicit ArgError(const std::string &m) : BddcError(1, m) {}
};
struct StateError : BddcError {
  explicit StateError(const std::string &m) : BddcError(2, m) {}
};
struct OomError : BddcError {
  explicit OomError(const std::string &m) : BddcError(3, m) {}
};
struct NotSpdError : BddcError {
  explicit NotSpdError(const std::string &m) : BddcError(4, m) {}
};
struct SingularCoarseError : BddcError {
  explicit SingularCoarseError(const std::string &m) : BddcError(5, m) {}
};
struct NoConvergenceError : BddcError {
  explicit NoConvergenceError(const std::string &m) : BddcError(6, m) {}
};
struct CornersError : BddcError {
  explicit CornersError(const std::string &m) : BddcError(7, m) {}
};
struct DeviceError : BddcError {
  explicit DeviceError(const std::string &m) : BddcError(8, m) {}
};

struct PcgResult {
  int iters = 0;
  bool converged = false;
  double relres = 0, lmin = 0, lmax = 0, seconds = 0;
  double r0 = 0;              // ||r_0||: the reduced problem's initial residual
  double true_relres = 0;     // ||f - A u|| / ||r_0|| with the assembled A (CSR A_i)
  double residual_floor = 0;  // eps || |A| |u| || / ||r_0||: rounding scale of that product
  int refinements = 0;        // correction solves run because true_relres > rtol
  int refine_iters = 0;       // PCG iterations of those correction solves
  std::vector<double> alphas, betas;
  std::vector<double> history;  // ||r_k|| / ||r_0||, k = 0..iters
};

void lanczos_extremes(const std::vector<double> &a, const std::vector<double> &b, double &lmin,
                      double &lmax);

// Per-category kernel timing with HIP events on the solver's stream.  Each
// timed launch also records the algorithmic bytes and flops it must move /
// perform (from the operand sizes), so achieved rates can be derived.
struct KernelStat {
  double ms = 0, bytes = 0, flops = 0;
  int64_t launches = 0;
};

class Timer : public LaunchTiming {
 public:
  int mode = 0;  // 0: off, 1: phase categories (begin / end), 2: kernel launches
  std::vector<std::string> names;
  std::vector<KernelStat> stats;
  void begin(hipStream_t st, const char *name, double bytes, double flops);
  void end(hipStream_t st);
  void launch_begin(hipStream_t st, const char *kernel, double bytes, double flops) override;
  void launch_end(hipStream_t st) override;
  void launch_amend(double bytes, double flops) override;
  void collect();  // after a synchronization: resolve pending event pairs
  void reset();
  ~Timer();

 private:
  struct Pending {
    int idx;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int cur = -1;
  hipEvent_t cur_a = nullptr;
  double cur_bytes = 0, cur_flops = 0;
  hipEvent_t get_event();
  void record_begin(hipStream_t st, const char *name, double bytes, double flops);
  void record_end(hipStream_t st);
};

// Work vectors of one preconditioner application: by default the solver's
// own buffers (own_work); the allocation-free entry point carves them out of
// a static device array instead (carve_work).
struct ApplyWork {
  double *vI = nullptr, *vG = nullptr, *vG2 = nullptr, *gr = nullptr, *gz = nullptr;
  double *vR = nullptr, *vR2 = nullptr, *vP = nullptr, *vc = nullptr, *scr = nullptr;
  float *vR32 = nullptr;
  double *mf_upd = nullptr, *mf_zp = nullptr;
  int *trsv_work = nullptr, *err = nullptr;
  int cols = 1;  // right-hand sides the vectors hold (each stack at its own length per column)
};

class Solver {
 public:
  // right-hand sides solved together (block PCG, multi-column applies)
  static constexpr int kMaxRhs = 8;
  static_assert(kMaxRhs <= kTrsvMaxCols && kMaxRhs <= MfDevice::kMaxCols, "block width");
  static constexpr int kMaxIt = 5000;

  DevAlloc alloc;
  hipStream_t stream = nullptr;
  Layout L;
  bool factored = false;
  double factor_seconds = 0, factor_flops = 0;
  std::vector<double> last_history;
  Timer timer;
  int verbose = 0;
  // 32: the constrained local factor K_rr = L L^T is stored in FP32 and the
  // preconditioner's local triangular solves run in FP32; the factorization,
  // the coarse basis and coarse matrix, and everything else stay FP64
  int factor_precision = 64;

  ~Solver();
  void build(const Problem &P, hipStream_t st, bool keep_interior = false);
  void factor();
  void factor_schur();
  void factor_local_fp32(int *status);
  int fp32_fallbacks = 0;  // substructures whose FP32 local factor fell back to FP64
  std::vector<int64_t> h_dinv_rr_off;
  void check_status(bool all);
  bool schur_ready = false;
  bool struct_ready = false;  // mesh / partition part of the layout is current
  void apply_global(const double *r, double *z);
  void apply_global(const double *r, double *z, const ApplyWork &w);
  // m <= w.cols columns at strides ldr, ldz (each factor read once for all)
  void apply_global(const double *r, int64_t ldr, double *z, int64_t ldz, int m, const ApplyWork &w);
  ApplyWork own_work();
  // bytes of a work set for apply_global (segments 256-byte aligned) and the
  // set laid out from base (device memory of at least work_bytes())
  size_t work_bytes() const;
  ApplyWork carve_work(void *base) const;
  PcgResult pcg(const double *f, double *u, double rtol, int maxit);
  // m <= kMaxRhs right-hand sides in one block PCG (f, u at strides ldf,
  // ldu), then the true-residual check and corrections per column
  std::vector<PcgResult> pcg_block(const double *f, int64_t ldf, double *u, int64_t ldu, int m,
                                   double rtol, int maxit);
  // one block PCG solve on the explicit Schur operator (pcg_block adds the
  // true-residual check and the correction solves); abs_tol[c] > 0 replaces
  // rtol[c] by abs_tol[c] / ||r_0||
  std::vector<PcgResult> pcg_once(const double *f, int64_t ldf, double *u, int64_t ldu, int m,
                                  const double *rtol, int maxit, const double *abs_tol);
  // rt = f - A u over all free dofs with the substructure matrices A_i;
  // returns ||rt|| and, in *floor, eps || |A| |u| ||
  double true_residual(const double *f, const double *u, double *rt, double *floor);
  static constexpr int kMaxRefine = 3;
  void free_all();

  // bytes streamed per PCG-internal preconditioner application and per
  // iteration (one right-hand side), counted from the stored operands
  double apply_bytes() const;
  double iter_bytes() const;

  // internals (public for the adaptive module)
  // (m: columns of a block, each vector stack at its own length per column)
  void apply_gamma(const double *r, double *z, int m = 1);
  void apply_gamma_condensed(const double *r, const double *vG_cond, double *z, const ApplyWork &w,
                             int m = 1);
  void apply_local(double *b, double *z, const ApplyWork &w, int m = 1);
  void apply_T_vec(double *x, double *scr, int m = 1);
  void apply_Tt_vec(double *b, double *scr, int m = 1);
  void schur_gamma(const double *p, double *q, int m = 1);
  void harmonic_extension(const double *zg, double *z, int64_t ldz, const ApplyWork &w, int m = 1);
  void interior_solve(double *vI, const ApplyWork *w = nullptr, int m = 1);
  void dot(const double *a, const double *b, int64_t n, double *out, int m = 1, int64_t lda = 0,
           int64_t ldb = 0);
  void scatter_gamma(const double *zg, double *z, int64_t ldz, int m = 1);
  void scatter_interior(const double *vI, double *z, int64_t ldz, int m = 1);
  void scatter64(const double *src, int64_t lds, const int64_t *idx, int64_t n, double *dst,
                 int64_t ldd, int m = 1);
  void trsv(const TrsvPlan &plan, const DBuf &A, const DBuf &desc, const DBuf &dinv,
            const DBuf &dinv_off, double *x, bool upper, const ApplyWork &w, int m = 1,
            int64_t ldx = 0);
  void trsv32(const TrsvPlan &plan, const DBuf &A, const DBuf &desc, const DBuf &dinv,
              const DBuf &dinv_off, float *x, bool upper, const ApplyWork &w, int m = 1,
              int64_t ldx = 0);
  void release(DBuf &b);
  std::vector<DBuf *> all_buffers();
  std::vector<DBuf *> struct_buffers();
  std::vector<DBuf *> cons_buffers();
  void build_structure(const Problem &P, hipStream_t st);

  int64_t n_rows = 0, nnz = 0;
  double bytes_S = 0, bytes_Lrr_tri = 0;
  double bytes_S_sym = 0, symv_parts = 0;  // symmetric Schur product: panel bytes, partial sums
  int n_gx = 0;
  TrsvPlan plan_rr, plan_c;
  std::vector<MatDesc> h_descRR, h_descGG, h_descC;
  std::vector<GemmDesc> h_spi;
  MfDevice mf;  // interior elimination (multifrontal)

  DBuf d_row_sub, d_row_loc, d_rowptr, d_col, d_val, d_nI, d_nG, d_nr, d_np;
  DBuf d_offI, d_offG, d_offR, d_offP, d_offGG, d_offRR, d_offRP, d_offPP;
  DBuf d_S, d_W, d_Lrr, d_Urr, d_Phi, d_Spi, d_Lc, d_Uc, d_descRRT;
  DBuf d_dinv_rr, d_dinv_rr_off, d_dinv_c, d_dinv_c_off;
  DBuf d_Lrr32, d_Urr32, d_dinv_rr32, d_vR32;  // FP32 local factor (factor_precision 32)
  DBuf d_Phi32, d_rscale;  // FP32 coarse-basis work block; diag(K_rr)^-1/2 per remaining dof
  DBuf d_PhiF, d_krrphi_desc;  // FP64 copy of the FP32 basis; K_rr Phi product descriptors
  std::vector<GemmDesc> h_krrphi;
  int64_t dinv_rr_elems = 0;
  DBuf d_descRR, d_descC, d_spi_desc, d_descGG, d_descRRvec,
      d_descCvec;
  DBuf d_gx, d_gx_ptr, d_trow, d_pos, d_wmat, d_gk_glob, d_gk_k, d_scr;
  int64_t scrS_elems = 0;
  int64_t scr_elems = 1;  // T / T^T vector scratch per column
  // the two passes of T^T S T as scatter products: descriptors (column
  // pass, row pass), local glob positions and their offsets per record
  DBuf d_xf_cols, d_xf_rows, d_xf_map, d_xf_map_off;
  std::vector<GemmDesc> h_xf_cols, h_xf_rows;
  int xf_max_ng = 0;
  int n_gk = 0;
  DBuf d_ridx, d_ridx_off, d_pidx, d_pidx_off, d_rabs, d_pabs, d_pcid, d_sub_cids;
  // block offsets of the flat gathers of K_rr, K_r,pi and K_pi,pi (host and device)
  std::vector<int64_t> h_gb_rr, h_gb_rp, h_gb_pp;
  DBuf d_gb_rr, d_gb_rp, d_gb_pp;
  DBuf d_c_ptr, d_c_sub, d_c_loc, d_c_copies;
  DBuf d_ifc_gamma, d_ifc_delta, d_gamma_ptr, d_gamma_copies, d_gamma_gdof, d_int_gdof, d_ifc_gdof;
  DBuf d_trsv_rr_fwd, d_trsv_rr_bwd, d_trsv_rr_off;
  DBuf d_trsv_c_fwd, d_trsv_c_bwd, d_trsv_c_off, d_work_i, d_status;
  DBuf d_vG, d_vG2, d_vR, d_vR2, d_vP, d_vI, d_vI2, d_vc;
  DBuf d_gam_r, d_gam_z, d_gam_p, d_gam_q, d_gam_x, d_sc, d_part, d_alphas, d_betas;
  DBuf d_true_r, d_true_d;  // global vectors: true residual and correction
  DBuf d_abs_I, d_abs_G;    // |A_i| |u_i| on the local stacks (rounding scale)
  DBuf d_symv_part, d_symv_off;  // partial products of the symmetric Schur operator
  DBuf d_pcg_ctl, d_pcg_hist;  // PCG control words (stop, iterations, converged, maxit), history
  // one PCG iteration captured as a graph (rebuilt after every build); the
  // stream it is captured on, two events and pinned words for the lookahead
  hipGraphExec_t pcg_exec[kMaxRhs + 1] = {};  // per block width
  hipStream_t cap_stream = nullptr;
  hipEvent_t pcg_ev[2] = {nullptr, nullptr};
  int *pcg_pin = nullptr;
  bool use_graphs = true;
  // unbatched baseline: the PCG's Schur products and local triangular solves
  // one substructure at a time (the dense operations follow the calling
  // thread's per_entry_launches switch)
  bool per_sub_launches = false;
  std::vector<TrsvPlan> sub_plans;  // per substructure (per_sub_launches)
  std::vector<DBuf> sub_plan_bufs;
  void pcg_iteration(int m);
  void drop_pcg_graph();
};

}  // namespace bddc
