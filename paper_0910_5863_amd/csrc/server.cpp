// Request server (bddc_server_*): continuous admission of independent solves
// by device-memory footprint, one worker thread and one non-blocking stream
// per request in flight, stream-ordered allocations (hipMallocAsync /
// hipFreeAsync) so that no allocation or release synchronizes the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bddc.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  // copies of the inputs
  bddc_mesh mesh{};
  std::vector<double> xyz, coef, f;
  std::vector<int64_t> hex8;
  std::vector<uint8_t> dirichlet;
  std::vector<int32_t> elem_sub;
  int32_t n_sub = 0;
  bddc_constraints cons{};
  bddc_pcg_params params{};
  double tau = 0;
  int64_t n_glob = 0;
  // results
  bddc_request_info info{};
  std::vector<double> u;
};

// Footprint estimate from the mesh and partition (see bddc_server_submit).
double footprint(const Request &r) {
  const int dpn = r.mesh.kind == 0 ? 1 : 3;
  const int64_t nn = r.mesh.n_nodes;
  // substructures touching each node
  std::vector<std::pair<int64_t, int32_t>> ns;
  ns.reserve((size_t)r.mesh.n_elems * 8);
  for (int64_t e = 0; e < r.mesh.n_elems; ++e)
    for (int k = 0; k < 8; ++k) ns.emplace_back(r.hex8[8 * e + k], r.elem_sub[e]);
  std::sort(ns.begin(), ns.end());
  ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
  std::vector<double> nG(r.n_sub, 0.0), nI(r.n_sub, 0.0);
  for (size_t i = 0; i < ns.size();) {
    size_t j = i;
    while (j < ns.size() && ns[j].first == ns[i].first) ++j;
    const int64_t node = ns[i].first;
    int free_dofs = 0;
    if (node >= 0 && node < nn)
      for (int c = 0; c < dpn; ++c) free_dofs += r.dirichlet[dpn * node + c] ? 0 : 1;
    for (size_t k = i; k < j; ++k) {
      const int32_t s = ns[k].second;
      if (s < 0 || s >= r.n_sub) continue;
      (j - i > 1 ? nG : nI)[s] += free_dofs;
    }
    i = j;
  }
  double b = 0;
  for (int s = 0; s < r.n_sub; ++s) {
    const double g = nG[s], n = nG[s] + nI[s];
    b += 8.0 * (6.0 + (r.tau > 0 ? 6.0 : 0.0)) * g * g;
    b += 8.0 * 2.0 * 81.0 * dpn * n;  // CSR values and indices
    b += 8.0 * 16.0 * n;              // vectors and index maps
  }
  return 1.15 * b + 64.0 * (1 << 20);
}

void *async_alloc(size_t bytes, void *user) {
  void *p = nullptr;
  if (hipMallocAsync(&p, bytes, (hipStream_t)user) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void async_free(void *p, void *user) { (void)hipFreeAsync(p, (hipStream_t)user); }

}  // namespace

struct bddc_server {
  bddc_server_options opt{};
  Clock::time_point t0;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  double reserved = 0;
  int running = 0;
  int64_t next_id = 0;
  bool stopping = false;
  std::vector<std::thread> workers;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // the head of the queue fits beside the requests in flight (or runs alone)
  bool head_fits() const {
    if (queue.empty()) return false;
    return running == 0 || reserved + queue.front()->info.footprint_bytes <= opt.hbm_budget_bytes;
  }

  // runs request r; results go to out and u (published by the caller under
  // the lock, so that queries never read a record being written)
  void process(const Request &r, bddc_request_info &out, std::vector<double> &u, hipStream_t st);
  void worker();
};

void bddc_server::process(const Request &r, bddc_request_info &info, std::vector<double> &u,
                          hipStream_t st) {
  bddc_options o{};
  o.device = opt.device;
  o.hip_stream = st;
  o.factor_precision = opt.factor_precision;
  o.alloc = async_alloc;
  o.free = async_free;
  o.alloc_user = st;
  bddc_ctx *c = nullptr;
  double *fd = nullptr, *ud = nullptr;
  auto fail = [&](bddc_status s, const char *what) {
    info.status = s;
    std::snprintf(info.error, sizeof info.error, "%s: %s", what,
                  c ? bddc_last_error(c) : "context creation");
  };
  bddc_status s = bddc_create(&o, &c);
  if (s != BDDC_OK) {
    fail(s, "create");
    return;
  }
  bddc_partition part{r.n_sub, r.elem_sub.data()};
  s = bddc_setup(c, &r.mesh, &part, &r.cons);
  bddc_info inf{};
  if (s == BDDC_OK) s = bddc_get_info(c, &inf);
  if (s != BDDC_OK) {
    fail(s, "setup");
  } else if (inf.n_glob != r.n_glob) {
    info.status = BDDC_ERR_ARG;
    std::snprintf(info.error, sizeof info.error, "load has %lld entries, the mesh %lld dofs",
                  (long long)r.n_glob, (long long)inf.n_glob);
  } else {
    info.nc = inf.nc;
    if (r.tau > 0) {
      bddc_adapt_info ai{};
      s = bddc_adapt(c, r.tau, &ai);
      if (s != BDDC_OK) fail(s, "adapt");
      info.omega = ai.omega;
      info.nc = ai.nc;
    }
    if (s == BDDC_OK && (s = bddc_factor(c)) != BDDC_OK) fail(s, "factor");
    if (s == BDDC_OK) {
      const size_t nb = sizeof(double) * (size_t)r.n_glob;
      fd = (double *)async_alloc(nb, st);
      ud = (double *)async_alloc(nb, st);
      if (!fd || !ud || hipMemcpyAsync(fd, r.f.data(), nb, hipMemcpyHostToDevice, st) != hipSuccess) {
        info.status = BDDC_ERR_OOM;
        std::snprintf(info.error, sizeof info.error, "load / solution buffers");
      } else if ((s = bddc_pcg_solve(c, 1, fd, r.n_glob, ud, r.n_glob, &r.params, &info.pcg)) !=
                 BDDC_OK) {
        fail(s, "pcg");
      } else {
        u.resize(r.n_glob);
        if (hipMemcpyAsync(u.data(), ud, nb, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
          info.status = BDDC_ERR_DEVICE;
          std::snprintf(info.error, sizeof info.error, "copy of the solution");
        }
      }
    }
  }
  if (fd) async_free(fd, st);
  if (ud) async_free(ud, st);
  bddc_destroy(c);
  (void)hipStreamSynchronize(st);
}

void bddc_server::worker() {
  (void)hipSetDevice(opt.device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(m);
      cv_work.wait(lk, [&] { return head_fits() || (stopping && queue.empty()); });
      if (queue.empty()) break;
      r = queue.front();
      queue.pop_front();
      reserved += r->info.footprint_bytes;
      running++;
      r->info.state = 1;
      r->info.start_s = now();
    }
    cv_work.notify_all();  // the new head may fit beside this one
    bddc_request_info res;
    std::vector<double> u;
    {
      std::lock_guard<std::mutex> lk(m);
      res = r->info;
    }
    if (have_stream) {
      process(*r, res, u, st);
    } else {
      res.status = BDDC_ERR_DEVICE;
      std::snprintf(res.error, sizeof res.error, "stream creation failed");
    }
    {
      std::lock_guard<std::mutex> lk(m);
      r->info = res;
      r->u.swap(u);
      reserved -= r->info.footprint_bytes;
      running--;
      r->info.done_s = now();
      r->info.state = r->info.status == BDDC_OK ? 2 : 3;
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
  if (have_stream) (void)hipStreamDestroy(st);
}

extern "C" {

bddc_status bddc_server_create(const bddc_server_options *opt, bddc_server **out) {
  if (!out) return BDDC_ERR_ARG;
  *out = nullptr;
  auto S = std::make_unique<bddc_server>();
  if (opt) S->opt = *opt;
  if (S->opt.factor_precision == 0) S->opt.factor_precision = 64;
  if (S->opt.factor_precision != 64 && S->opt.factor_precision != 32) return BDDC_ERR_ARG;
  if (S->opt.max_active <= 0) S->opt.max_active = 4;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || S->opt.device < 0 || S->opt.device >= n)
    return BDDC_ERR_ARG;
  if (hipSetDevice(S->opt.device) != hipSuccess) return BDDC_ERR_DEVICE;
  if (S->opt.hbm_budget_bytes <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return BDDC_ERR_DEVICE;
    S->opt.hbm_budget_bytes = 0.8 * (double)fr;
  }
  // keep freed blocks in the stream-ordered pool up to the budget instead of
  // returning them to the driver at every synchronization
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, S->opt.device) == hipSuccess) {
    uint64_t thr = (uint64_t)S->opt.hbm_budget_bytes;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  S->t0 = Clock::now();
  bddc_server *raw = S.get();
  for (int w = 0; w < S->opt.max_active; ++w) S->workers.emplace_back([raw] { raw->worker(); });
  *out = S.release();
  return BDDC_OK;
}

bddc_status bddc_server_submit(bddc_server *srv, const bddc_mesh *mesh, const bddc_partition *part,
                               const bddc_constraints *cons, double tau, const double *f,
                               int64_t n_glob, const bddc_pcg_params *params, int64_t *id) {
  if (!srv || !mesh || !part || !cons || !f || !id || n_glob <= 0) return BDDC_ERR_ARG;
  if (!mesh->xyz || !mesh->hex8 || !mesh->coef || !mesh->dirichlet || !part->elem_sub ||
      mesh->n_nodes <= 0 || mesh->n_elems <= 0 || part->n_sub <= 0 ||
      (mesh->kind != 0 && mesh->kind != 1))
    return BDDC_ERR_ARG;
  auto r = std::make_unique<Request>();
  const int dpn = mesh->kind == 0 ? 1 : 3;
  r->xyz.assign(mesh->xyz, mesh->xyz + 3 * mesh->n_nodes);
  r->hex8.assign(mesh->hex8, mesh->hex8 + 8 * mesh->n_elems);
  r->coef.assign(mesh->coef, mesh->coef + mesh->n_elems);
  r->dirichlet.assign(mesh->dirichlet, mesh->dirichlet + dpn * mesh->n_nodes);
  r->elem_sub.assign(part->elem_sub, part->elem_sub + mesh->n_elems);
  r->f.assign(f, f + n_glob);
  r->mesh = *mesh;
  r->mesh.xyz = r->xyz.data();
  r->mesh.hex8 = r->hex8.data();
  r->mesh.coef = r->coef.data();
  r->mesh.dirichlet = r->dirichlet.data();
  r->n_sub = part->n_sub;
  r->cons = *cons;
  if (params) r->params = *params;
  r->tau = tau;
  r->n_glob = n_glob;
  r->info.footprint_bytes = footprint(*r);
  r->info.n_glob = n_glob;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    r->id = r->info.id = srv->next_id++;
    r->info.submit_s = srv->now();
    *id = r->id;
    srv->queue.push_back(r.get());
    srv->reqs.emplace(r->id, std::move(r));
  }
  srv->cv_work.notify_all();
  return BDDC_OK;
}

bddc_status bddc_server_query(bddc_server *srv, int64_t id, bddc_request_info *info) {
  if (!srv) return BDDC_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->m);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end()) return BDDC_ERR_ARG;
  if (info) *info = it->second->info;
  return BDDC_OK;
}

bddc_status bddc_server_wait(bddc_server *srv, int64_t id, double *u, bddc_request_info *info) {
  if (!srv) return BDDC_ERR_ARG;
  std::unique_lock<std::mutex> lk(srv->m);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end()) return BDDC_ERR_ARG;
  Request *r = it->second.get();
  srv->cv_done.wait(lk, [&] { return r->info.state >= 2; });
  if (info) *info = r->info;
  if (u && r->info.state == 2) std::memcpy(u, r->u.data(), sizeof(double) * r->u.size());
  return BDDC_OK;
}

bddc_status bddc_server_release(bddc_server *srv, int64_t id) {
  if (!srv) return BDDC_ERR_ARG;
  std::lock_guard<std::mutex> lk(srv->m);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end() || it->second->info.state < 2) return BDDC_ERR_STATE;
  srv->reqs.erase(it);
  return BDDC_OK;
}

void bddc_server_destroy(bddc_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  for (std::thread &t : srv->workers) t.join();
  delete srv;
}

}  // extern "C"
