// C ABI of the BDDC library (include/bddc.h): argument checks, the call-order
// state machine and error reporting around the host setup and device solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>

#include "ctx.h"

using namespace bddc;

extern "C" {

bddc_status bddc_create(const bddc_options *opt, bddc_ctx **out) {
  if (!out) return BDDC_ERR_ARG;
  *out = nullptr;
  auto c = std::make_unique<bddc_ctx>();
  if (opt) c->opt = *opt;
  if (c->opt.factor_precision == 0) c->opt.factor_precision = 64;
  if (c->opt.factor_precision != 64 && c->opt.factor_precision != 32) return BDDC_ERR_ARG;
  if (c->opt.chol_launch < 0 || c->opt.chol_launch > 2) return BDDC_ERR_ARG;
  if (c->opt.device < 0) {  // host-only context: analysis without a GPU
    c->S = std::make_unique<Solver>();
    *out = c.release();
    return BDDC_OK;
  }
  bddc_status st = guarded(c.get(), [&] {
    int n = 0;
    check_hip(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (c->opt.device < 0 || c->opt.device >= n) throw ArgError("no such HIP device");
    check_hip(hipSetDevice(c->opt.device), "hipSetDevice");
    if (c->opt.hip_stream) {
      c->stream = (hipStream_t)c->opt.hip_stream;
    } else {
      check_hip(hipStreamCreate(&c->stream), "hipStreamCreate");
      c->own_stream = true;
    }
    c->S = std::make_unique<Solver>();
    c->S->alloc.alloc = c->opt.alloc;
    c->S->alloc.free = c->opt.free;
    c->S->alloc.user = c->opt.alloc_user;
    c->S->verbose = c->opt.verbose;
    c->S->factor_precision = c->opt.factor_precision;
    c->S->per_sub_launches = c->opt.per_substructure_launches != 0;
  });
  if (st != BDDC_OK) return st;
  *out = c.release();
  return BDDC_OK;
}

bddc_status bddc_setup(bddc_ctx *c, const bddc_mesh *mesh, const bddc_partition *part,
                       const bddc_constraints *cons) {
  if (!c) return BDDC_ERR_ARG;
  if (!mesh || !part || !cons) return fail(c, BDDC_ERR_ARG, "null argument");
  if (!mesh->xyz || !mesh->hex8 || !mesh->coef || !mesh->dirichlet || !part->elem_sub)
    return fail(c, BDDC_ERR_ARG, "null mesh or partition array");
  if (mesh->kind != 0 && mesh->kind != 1) return fail(c, BDDC_ERR_ARG, "kind must be 0 or 1");
  if (mesh->n_nodes <= 0 || mesh->n_elems <= 0 || part->n_sub <= 0)
    return fail(c, BDDC_ERR_ARG, "empty mesh or partition");
  if (cons->mode < 0 || cons->mode > 3) return fail(c, BDDC_ERR_ARG, "constraint mode in 0..3");
  return guarded(c, [&] {
    if (c->opt.device >= 0) check_hip(hipSetDevice(c->opt.device), "hipSetDevice");
    Problem &P = c->P;
    P = Problem();
    MeshIn &m = P.mesh;
    m.kind = mesh->kind;
    m.dpn = mesh->kind == 0 ? 1 : 3;
    m.n_nodes = mesh->n_nodes;
    m.n_elems = mesh->n_elems;
    m.xyz.assign(mesh->xyz, mesh->xyz + 3 * mesh->n_nodes);
    m.hex8.assign(mesh->hex8, mesh->hex8 + 8 * mesh->n_elems);
    m.coef.assign(mesh->coef, mesh->coef + mesh->n_elems);
    m.nu = mesh->nu;
    m.dirichlet.assign(mesh->dirichlet, mesh->dirichlet + m.dpn * mesh->n_nodes);
    m.n_sub = part->n_sub;
    m.elem_sub.assign(part->elem_sub, part->elem_sub + mesh->n_elems);
    for (int64_t v : m.hex8)
      if (v < 0 || v >= m.n_nodes) throw ArgError("hex8 node id out of range");
    std::vector<int> cnt(m.n_sub, 0);
    for (int32_t s : m.elem_sub) {
      if (s < 0 || s >= m.n_sub) throw ArgError("elem_sub out of range");
      cnt[s]++;
    }
    for (int s = 0; s < m.n_sub; ++s)
      if (!cnt[s]) throw ArgError("substructure " + std::to_string(s) + " has no element");
    if (m.kind == 1 && !(m.nu > -1.0 && m.nu < 0.5)) throw ArgError("nu must lie in (-1, 0.5)");
    P.full2glob.assign(m.n_nodes * m.dpn, -1);
    int64_t ng = 0;
    for (int64_t d = 0; d < m.n_nodes * m.dpn; ++d)
      if (!m.dirichlet[d]) {
        P.full2glob[d] = ng++;
        P.glob2full.push_back(d);
      }
    P.n_glob = ng;
    P.mode = cons->mode;
    P.drop_tol = cons->qr_drop_tol > 0 ? cons->qr_drop_tol : 1e-10;
    P.adapt_edges = cons->adaptive_edges != 0;
    assemble_substructures(P);
    classify_interface(P, cons->augment_corners != 0);
    compute_weights(P);
    build_constraints(P);
    c->adapt = AdaptState();
    if (c->opt.device >= 0) c->S->build(P, c->stream);
    c->state = 1;
  });
}

bddc_status bddc_factor(bddc_ctx *c) {
  if (c && c->opt.device < 0) return fail(c, BDDC_ERR_STATE, "host-only context (device < 0)");
  if (!c) return BDDC_ERR_ARG;
  if (c->state < 1) return fail(c, BDDC_ERR_STATE, "bddc_factor before bddc_setup");
  return guarded(c, [&] {
    check_hip(hipSetDevice(c->opt.device), "hipSetDevice");
    c->state = 1;
    c->S->factor();
    c->state = 2;
  });
}

bddc_status bddc_apply(bddc_ctx *c, int nrhs, const double *r, int64_t ldr, double *z,
                       int64_t ldz) {
  if (!c) return BDDC_ERR_ARG;
  if (c->state < 2) return fail(c, BDDC_ERR_STATE, "bddc_apply before bddc_factor");
  if (nrhs < 0 || (nrhs > 0 && (!r || !z))) return fail(c, BDDC_ERR_ARG, "bad vectors");
  if (ldr < c->P.n_glob || ldz < c->P.n_glob) return fail(c, BDDC_ERR_ARG, "leading dimension < n_glob");
  return guarded(c, [&] {
    check_hip(hipSetDevice(c->opt.device), "hipSetDevice");
    // blocks of up to Solver::kMaxRhs columns, each reading the factors once
    const ApplyWork w = c->S->own_work();
    for (int q0 = 0; q0 < nrhs; q0 += Solver::kMaxRhs) {
      const int m = std::min(Solver::kMaxRhs, nrhs - q0);
      c->S->apply_global(r + q0 * ldr, ldr, z + q0 * ldz, ldz, m, w);
    }
    check_hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  });
}

bddc_status bddc_pcg_solve(bddc_ctx *c, int nrhs, const double *f, int64_t ldf, double *u,
                           int64_t ldu, const bddc_pcg_params *prm, bddc_pcg_info *info) {
  if (!c) return BDDC_ERR_ARG;
  if (c->state < 2) return fail(c, BDDC_ERR_STATE, "bddc_pcg_solve before bddc_factor");
  if (nrhs < 0 || (nrhs > 0 && (!f || !u))) return fail(c, BDDC_ERR_ARG, "bad vectors");
  if (ldf < c->P.n_glob || ldu < c->P.n_glob) return fail(c, BDDC_ERR_ARG, "leading dimension < n_glob");
  const double rtol = (prm && prm->rtol > 0) ? prm->rtol : 1e-8;
  const int maxit = (prm && prm->maxit > 0) ? prm->maxit : 1000;
  bool all_conv = true;
  bddc_status st = guarded(c, [&] {
    check_hip(hipSetDevice(c->opt.device), "hipSetDevice");
    // blocks of up to Solver::kMaxRhs columns solved in lock step
    std::vector<PcgResult> all;
    for (int q0 = 0; q0 < nrhs; q0 += Solver::kMaxRhs) {
      const int m = std::min(Solver::kMaxRhs, nrhs - q0);
      std::vector<PcgResult> b = c->S->pcg_block(f + q0 * ldf, ldf, u + q0 * ldu, ldu, m, rtol, maxit);
      all.insert(all.end(), b.begin(), b.end());
    }
    for (int q = 0; q < nrhs; ++q) {
      const PcgResult &res = all[q];
      if (info) {
        bddc_pcg_info &o = info[q];
        o.iters = res.iters;
        o.converged = res.converged;
        o.relres = res.relres;
        o.lmin = res.lmin;
        o.lmax = res.lmax;
        o.kappa = res.lmax / res.lmin;
        o.seconds = res.seconds;
        o.true_relres = res.true_relres;
        o.refinements = res.refinements;
        o.refine_iters = res.refine_iters;
        o.residual_floor = res.residual_floor;
      }
      all_conv &= res.converged;
    }
    check_hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  });
  if (st != BDDC_OK) return st;
  if (!all_conv) return fail(c, BDDC_ERR_NO_CONVERGENCE, "PCG did not reach the tolerance");
  return BDDC_OK;
}

static bddc_status adapt_impl(bddc_ctx *c, double tau, int count, bddc_adapt_info *info) {
  return guarded(c, [&] {
    check_hip(hipSetDevice(c->opt.device), "hipSetDevice");
    auto t0 = std::chrono::steady_clock::now();
    // adaptive rows of an earlier call are replaced, not added to
    bool had_rows = false;
    for (int k : c->P.extra_k) had_rows |= k > 0;
    if (had_rows) {
      for (auto &r : c->P.extra_rows) r.clear();
      for (int &k : c->P.extra_k) k = 0;
      build_constraints(c->P);
    }
    AdaptResult res = run_adapt(c->P, *c->S, c->adapt, tau, count);
    auto ta = std::chrono::steady_clock::now();
    build_constraints(c->P);
    auto tb = std::chrono::steady_clock::now();
    c->S->build(c->P, c->stream, /*keep_interior=*/true);
    if (c->opt.verbose) {
      auto tc = std::chrono::steady_clock::now();
      std::fprintf(stderr, "[bddc adapt] constraints (host QR) %.3f s, solver rebuild %.3f s\n",
                   std::chrono::duration<double>(tb - ta).count(),
                   std::chrono::duration<double>(tc - tb).count());
    }
    c->state = 1;
    if (info) {
      info->omega = res.omega;
      info->nc = count_nc(c->P);
      info->n_added = res.n_added;
      info->n_pairs = res.n_pairs;
      info->lobpcg_iters = res.iters;
      info->unconverged = res.unconverged;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      info->n_added_edge = res.n_added_edge;
    }
  });
}

bddc_status bddc_adapt(bddc_ctx *c, double tau, bddc_adapt_info *info) {
  if (c && c->opt.device < 0) return fail(c, BDDC_ERR_STATE, "host-only context (device < 0)");
  if (!c) return BDDC_ERR_ARG;
  if (c->state < 1) return fail(c, BDDC_ERR_STATE, "bddc_adapt before bddc_setup");
  if (!(tau > 0)) return fail(c, BDDC_ERR_ARG, "tau must be positive");
  return adapt_impl(c, tau, 0, info);
}

bddc_status bddc_adapt_count(bddc_ctx *c, int rows_per_face, bddc_adapt_info *info) {
  if (c && c->opt.device < 0) return fail(c, BDDC_ERR_STATE, "host-only context (device < 0)");
  if (!c) return BDDC_ERR_ARG;
  if (c->state < 1) return fail(c, BDDC_ERR_STATE, "bddc_adapt_count before bddc_setup");
  if (rows_per_face < 1) return fail(c, BDDC_ERR_ARG, "rows_per_face must be >= 1");
  return adapt_impl(c, HUGE_VAL, rows_per_face, info);
}

bddc_status bddc_get_info(const bddc_ctx *c, bddc_info *o) {
  if (!c || !o) return BDDC_ERR_ARG;
  std::memset(o, 0, sizeof(*o));
  if (c->state < 1) return BDDC_ERR_STATE;
  const Problem &P = c->P;
  const Layout &L = c->S->L;
  if (c->opt.device < 0) {
    o->n_glob = P.n_glob;
    o->n_sub = (int64_t)P.subs.size();
    o->n_corners = (int64_t)P.corner_nodes.size();
    o->n_edges = (int64_t)P.edge_ids.size();
    o->n_faces = (int64_t)P.face_ids.size();
    o->nc = count_nc(P);
    for (const Sub &S : P.subs) {
      o->n_iface_total += S.nG;
      o->max_interior = std::max<int64_t>(o->max_interior, S.nI);
      o->max_iface = std::max<int64_t>(o->max_iface, S.nG);
    }
    return BDDC_OK;
  }
  o->n_glob = P.n_glob;
  o->n_sub = (int64_t)P.subs.size();
  o->n_corners = (int64_t)P.corner_nodes.size();
  o->n_edges = (int64_t)P.edge_ids.size();
  o->n_faces = (int64_t)P.face_ids.size();
  o->nc = count_nc(P);
  o->n_coarse = L.n_coarse;
  o->n_iface_total = L.sumG;
  o->max_interior = L.max_nI;
  o->max_iface = L.max_nG;
  o->factor_flops = c->S->factor_flops;
  o->factor_seconds = c->S->factor_seconds;
  o->apply_bytes = c->S->apply_bytes();
  o->pcg_iter_bytes = c->S->iter_bytes();
  o->device_bytes = c->S->alloc.held;
  o->autotune_entries = autotune_entries();
  o->fp32_fallbacks = c->S ? c->S->fp32_fallbacks : 0;
  return BDDC_OK;
}

bddc_status bddc_get_face_rows(const bddc_ctx *c, int64_t f, int64_t max_rows, double *out,
                               int64_t *dofs, int64_t *rows, int64_t *n_dofs, int32_t *subs) {
  if (!c || !rows || !n_dofs) return BDDC_ERR_ARG;
  if (c->state < 1) return BDDC_ERR_STATE;
  const Problem &P = c->P;
  if (f < 0 || f >= (int64_t)P.face_ids.size()) return BDDC_ERR_ARG;
  const int gi = P.face_ids[f];
  const Glob &g = P.globs[gi];
  const int n = (int)g.dofs.size();
  const int k = (gi < (int)P.extra_k.size()) ? P.extra_k[gi] : 0;
  *rows = k;
  *n_dofs = n;
  if (subs) subs[0] = g.subs[0], subs[1] = g.subs[1];
  if (dofs)
    for (int t = 0; t < n; ++t) dofs[t] = g.dofs[t];
  if (out)
    for (int64_t r = 0; r < std::min<int64_t>(k, max_rows); ++r)
      for (int t = 0; t < n; ++t) out[r * n + t] = P.extra_rows[gi][(size_t)r * n + t];
  return BDDC_OK;
}

bddc_status bddc_get_edge_rows(const bddc_ctx *c, int64_t e, int64_t max_rows, double *out,
                               int64_t *dofs, int64_t *rows, int64_t *n_dofs) {
  if (!c || !rows || !n_dofs) return BDDC_ERR_ARG;
  if (c->state < 1) return BDDC_ERR_STATE;
  const Problem &P = c->P;
  if (e < 0 || e >= (int64_t)P.edge_ids.size()) return BDDC_ERR_ARG;
  const int gi = P.edge_ids[e];
  const Glob &g = P.globs[gi];
  const int n = (int)g.dofs.size();
  const int k = (gi < (int)P.extra_k.size()) ? P.extra_k[gi] : 0;
  *rows = k;
  *n_dofs = n;
  if (dofs)
    for (int t = 0; t < n; ++t) dofs[t] = g.dofs[t];
  if (out)
    for (int64_t r = 0; r < std::min<int64_t>(k, max_rows); ++r)
      for (int t = 0; t < n; ++t) out[r * n + t] = P.extra_rows[gi][(size_t)r * n + t];
  return BDDC_OK;
}

bddc_status bddc_get_face_eigs(const bddc_ctx *c, int64_t f, int64_t max, double *out,
                               int64_t *count) {
  if (!c || !count) return BDDC_ERR_ARG;
  if (c->state < 1) return BDDC_ERR_STATE;
  if (f < 0 || f >= (int64_t)c->P.face_ids.size()) return BDDC_ERR_ARG;
  const auto &ev = c->adapt.eigs;
  if (f >= (int64_t)ev.size()) {
    *count = 0;
    return BDDC_OK;
  }
  *count = (int64_t)ev[f].size();
  if (out)
    for (int64_t i = 0; i < std::min<int64_t>(*count, max); ++i) out[i] = ev[f][i];
  return BDDC_OK;
}

bddc_status bddc_pcg_history(const bddc_ctx *c, int64_t max, double *out, int64_t *count) {
  if (!c || !count) return BDDC_ERR_ARG;
  if (c->state < 2) return BDDC_ERR_STATE;
  const auto &h = c->S->last_history;
  *count = (int64_t)h.size();
  if (out)
    for (int64_t i = 0; i < std::min<int64_t>(*count, max); ++i) out[i] = h[i];
  return BDDC_OK;
}

bddc_status bddc_get_substructure(const bddc_ctx *c, int32_t s, int64_t *n, int64_t *n_interior,
                                  int64_t *nnz, int64_t *gdof, int64_t *rowptr, int32_t *col,
                                  double *val, double *weights) {
  if (!c || !n || !n_interior || !nnz) return BDDC_ERR_ARG;
  if (c->state < 1) return BDDC_ERR_STATE;
  if (s < 0 || s >= (int32_t)c->P.subs.size()) return BDDC_ERR_ARG;
  const Sub &S = c->P.subs[s];
  *n = S.nI + S.nG;
  *n_interior = S.nI;
  *nnz = (int64_t)S.A.val.size();
  if (gdof)
    for (int64_t i = 0; i < *n; ++i) gdof[i] = S.gdof[i];
  if (rowptr)
    for (int64_t i = 0; i <= *n; ++i) rowptr[i] = S.A.ptr[i];
  if (col)
    for (int64_t k = 0; k < *nnz; ++k) col[k] = S.A.col[k];
  if (val)
    for (int64_t k = 0; k < *nnz; ++k) val[k] = S.A.val[k];
  if (weights)
    for (int t = 0; t < S.nG; ++t) weights[t] = S.delta[t];
  return BDDC_OK;
}

bddc_status bddc_set_timing(bddc_ctx *c, int on) {
  if (!c) return BDDC_ERR_ARG;
  if (c->opt.device < 0) return fail(c, BDDC_ERR_STATE, "host-only context (device < 0)");
  return guarded(c, [&] {
    if (on < 0 || on > 2) throw ArgError("timing mode must be 0, 1 or 2");
    c->S->timer.reset();
    c->S->timer.mode = on;
  });
}

bddc_status bddc_get_timing(const bddc_ctx *c, int max, bddc_kernel_stat *out, int *count) {
  if (!c || !count) return BDDC_ERR_ARG;
  if (!c->S) return BDDC_ERR_STATE;
  Timer &t = c->S->timer;
  try {
    t.collect();
  } catch (const std::exception &) {
    return BDDC_ERR_DEVICE;
  }
  *count = (int)t.names.size();
  if (out)
    for (int i = 0; i < std::min(max, *count); ++i) {
      std::memset(out[i].name, 0, sizeof(out[i].name));
      std::strncpy(out[i].name, t.names[i].c_str(), sizeof(out[i].name) - 1);
      out[i].ms = t.stats[i].ms;
      out[i].launches = t.stats[i].launches;
      out[i].bytes = t.stats[i].bytes;
      out[i].flops = t.stats[i].flops;
    }
  return BDDC_OK;
}

const char *bddc_last_error(const bddc_ctx *c) { return c ? c->err.c_str() : "null context"; }

void bddc_destroy(bddc_ctx *c) {
  if (!c) return;
  if (c->opt.device < 0) {
    delete c;
    return;
  }
  (void)hipSetDevice(c->opt.device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->S.reset();
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
