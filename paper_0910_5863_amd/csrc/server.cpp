// Request server (bddc_server_*): continuous admission of independent solves
// by device-memory footprint, one worker thread and one non-blocking stream
// per request in flight, stream-ordered allocations (hipMallocAsync /
// hipFreeAsync) so that no allocation or release synchronizes the device.
// With resident factors on, the factored context of a problem stays on the
// device after its request (on a stream of its own); later requests on the
// same problem skip setup, adaptation and factorization, queued ones are
// taken together and solved as blocks (one block PCG for up to kBlockRhs
// loads, reading each factor once per application for all of them), and
// idle contexts are evicted least recently used first when the budget needs
// their memory.
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
  uint64_t key = 0;  // fingerprint of the problem (everything but the load)
  // resident match, resolved once per resident context: the serial of the
  // matching one (0: none known) and the largest serial already compared
  uint64_t match = 0, checked_upto = 0;
  // results
  bddc_request_info info{};
  std::vector<double> u;
};

// FNV-1a over the bytes of the problem (mesh, partition, constraints, tau)
uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

uint64_t problem_key(const Request &r) {
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, &r.mesh.kind, sizeof r.mesh.kind);
  h = fnv(h, &r.mesh.nu, sizeof r.mesh.nu);
  h = fnv(h, r.xyz.data(), sizeof(double) * r.xyz.size());
  h = fnv(h, r.hex8.data(), sizeof(int64_t) * r.hex8.size());
  h = fnv(h, r.coef.data(), sizeof(double) * r.coef.size());
  h = fnv(h, r.dirichlet.data(), r.dirichlet.size());
  h = fnv(h, r.elem_sub.data(), sizeof(int32_t) * r.elem_sub.size());
  h = fnv(h, &r.n_sub, sizeof r.n_sub);
  h = fnv(h, &r.cons.mode, sizeof r.cons.mode);
  h = fnv(h, &r.cons.augment_corners, sizeof r.cons.augment_corners);
  h = fnv(h, &r.cons.qr_drop_tol, sizeof r.cons.qr_drop_tol);
  h = fnv(h, &r.cons.adaptive_edges, sizeof r.cons.adaptive_edges);
  h = fnv(h, &r.tau, sizeof r.tau);
  return h;
}

// the same problem (the fingerprint only selects the candidates)
bool same_problem(const Request &a, const Request &b) {
  return a.key == b.key && a.n_glob == b.n_glob && a.mesh.kind == b.mesh.kind &&
         a.mesh.nu == b.mesh.nu &&
         a.xyz == b.xyz && a.hex8 == b.hex8 && a.coef == b.coef && a.dirichlet == b.dirichlet &&
         a.elem_sub == b.elem_sub && a.n_sub == b.n_sub && a.cons.mode == b.cons.mode &&
         a.cons.augment_corners == b.cons.augment_corners &&
         a.cons.qr_drop_tol == b.cons.qr_drop_tol && a.cons.adaptive_edges == b.cons.adaptive_edges &&
         a.tau == b.tau;
}

// A factored context kept on the device for its problem.
struct Resident {
  uint64_t serial = 0;             // unique per resident context, increasing
  std::unique_ptr<Request> proto;  // a copy of the problem's inputs (the load unused)
  bddc_ctx *ctx = nullptr;
  hipStream_t st = nullptr;
  double footprint = 0;
  bool busy = true;   // a worker builds or uses it
  uint64_t last_used = 0;
  double omega = 0;
  int64_t nc = 0;
};

constexpr int kMaxTaken = 16;  // queued requests on one resident problem taken at once
constexpr int kBlockRhs = 8;   // loads per block PCG (the library's block width)

bool same_params(const Request &a, const Request &b) {
  return a.params.rtol == b.params.rtol && a.params.maxit == b.params.maxit;
}

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
  double reserved = 0;   // footprints of the requests in flight and the resident contexts
  int running = 0;
  int64_t next_id = 0;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::vector<std::unique_ptr<Resident>> resident;
  uint64_t use_clock = 0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  bool keep_resident() const { return opt.resident_bytes > 0; }

  uint64_t resident_serial = 0;

  // the resident context of r's problem, or null.  The byte-wise comparison
  // of the problem runs once per (request, resident context) pair: its
  // outcome is kept in the request (match, checked_upto), so the wake-ups of
  // the workers, under the lock, only compare serials.
  Resident *find_resident(Request &r) const {
    if (r.match) {
      for (auto &e : resident)
        if (e->serial == r.match) return e.get();
      r.match = 0;  // evicted
    }
    uint64_t upto = r.checked_upto;
    Resident *hit = nullptr;
    for (auto &e : resident) {
      if (e->serial <= r.checked_upto) continue;
      upto = std::max(upto, e->serial);
      if (!hit && e->proto->key == r.key && same_problem(*e->proto, r)) hit = e.get();
    }
    r.checked_upto = upto;
    if (hit) r.match = hit->serial;
    return hit;
  }
  double idle_resident_bytes() const {
    double b = 0;
    for (auto &e : resident)
      if (!e->busy) b += e->footprint;
    return b;
  }

  // the head of the queue can start: its problem is resident and idle, or it
  // fits beside the requests in flight once idle resident contexts are
  // evicted (or runs alone); a head whose problem is resident but busy waits
  bool head_admissible() const {
    if (queue.empty()) return false;
    Request &h = *queue.front();
    if (Resident *e = find_resident(h)) return !e->busy;
    return running == 0 ||
           reserved - idle_resident_bytes() + h.info.footprint_bytes <= opt.hbm_budget_bytes;
  }

  // removes idle resident contexts, least recently used first, while
  // pred(bytes removed so far) holds.  They are destroyed by the caller
  // outside the lock; their footprints stay in `reserved` until then
  // (release_destroyed), so admission never counts memory not yet freed.
  template <class Pred>
  void evict_while(Pred pred, std::vector<std::unique_ptr<Resident>> &out) {
    double freed = 0;
    while (pred(freed)) {
      int v = -1;
      for (int i = 0; i < (int)resident.size(); ++i)
        if (!resident[i]->busy && (v < 0 || resident[i]->last_used < resident[v]->last_used)) v = i;
      if (v < 0) return;
      freed += resident[v]->footprint;
      out.push_back(std::move(resident[v]));
      resident.erase(resident.begin() + v);
    }
  }
  // destroys removed resident contexts, then returns their footprints
  void release_destroyed(std::vector<std::unique_ptr<Resident>> &v);

  // builds a context for r's problem on stream st (setup, adapt, factor);
  // null on failure, with info.status and info.error set
  bddc_ctx *build(const Request &r, bddc_request_info &info, hipStream_t st);
  // solves the loads of rs (same PCG parameters, at most kBlockRhs) as one
  // block on a factored context; results go to infos and us (published by
  // the caller under the lock, so that queries never read a record being
  // written)
  void solve(bddc_ctx *c, const std::vector<Request *> &rs, std::vector<bddc_request_info *> &infos,
             std::vector<std::vector<double> *> &us, hipStream_t st);
  void worker();
};

void destroy_resident(std::vector<std::unique_ptr<Resident>> &v) {
  for (auto &e : v) {
    if (e->ctx) bddc_destroy(e->ctx);
    if (e->st) {
      (void)hipStreamSynchronize(e->st);
      (void)hipStreamDestroy(e->st);
    }
  }
  v.clear();
}

void bddc_server::release_destroyed(std::vector<std::unique_ptr<Resident>> &v) {
  if (v.empty()) return;
  double b = 0;
  for (auto &e : v) b += e->footprint;
  destroy_resident(v);
  {
    std::lock_guard<std::mutex> lk(m);
    reserved -= b;
  }
  cv_work.notify_all();
}

bddc_ctx *bddc_server::build(const Request &r, bddc_request_info &info, hipStream_t st) {
  bddc_options o{};
  o.device = opt.device;
  o.hip_stream = st;
  o.factor_precision = opt.factor_precision;
  o.alloc = async_alloc;
  o.free = async_free;
  o.alloc_user = st;
  bddc_ctx *c = nullptr;
  auto fail = [&](bddc_status s, const char *what) {
    info.status = s;
    std::snprintf(info.error, sizeof info.error, "%s: %s", what,
                  c ? bddc_last_error(c) : "context creation");
  };
  bddc_status s = bddc_create(&o, &c);
  if (s != BDDC_OK) {
    fail(s, "create");
    return nullptr;
  }
  bddc_partition part{r.n_sub, r.elem_sub.data()};
  s = bddc_setup(c, &r.mesh, &part, &r.cons);
  bddc_info inf{};
  if (s == BDDC_OK) s = bddc_get_info(c, &inf);
  if (s != BDDC_OK) {
    fail(s, "setup");
  } else if (inf.n_glob != r.n_glob) {
    s = BDDC_ERR_ARG;
    info.status = s;
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
  }
  if (s != BDDC_OK) {
    bddc_destroy(c);
    (void)hipStreamSynchronize(st);
    return nullptr;
  }
  return c;
}

void bddc_server::solve(bddc_ctx *c, const std::vector<Request *> &rs,
                        std::vector<bddc_request_info *> &infos,
                        std::vector<std::vector<double> *> &us, hipStream_t st) {
  const int m = (int)rs.size();
  const int64_t n = rs[0]->n_glob;
  const size_t nb = sizeof(double) * (size_t)n * m;
  double *fd = (double *)async_alloc(nb, st), *ud = (double *)async_alloc(nb, st);
  auto fail_all = [&](int status, const char *msg) {
    for (bddc_request_info *i : infos) {
      i->status = status;
      std::snprintf(i->error, sizeof i->error, "%s", msg);
    }
  };
  bool copied = fd && ud;
  for (int q = 0; q < m && copied; ++q)
    copied = hipMemcpyAsync(fd + q * n, rs[q]->f.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                            st) == hipSuccess;
  if (!copied) {
    fail_all(BDDC_ERR_OOM, "load / solution buffers");
  } else {
    std::vector<bddc_pcg_info> pinfo(m);
    const bddc_status s = bddc_pcg_solve(c, m, fd, n, ud, n, &rs[0]->params, pinfo.data());
    if (s != BDDC_OK && s != BDDC_ERR_NO_CONVERGENCE) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "pcg: %s", bddc_last_error(c));
      fail_all(s, msg);
    } else {
      bool ok = true;
      for (int q = 0; q < m && ok; ++q) {
        us[q]->resize(n);
        ok = hipMemcpyAsync(us[q]->data(), ud + q * n, sizeof(double) * n, hipMemcpyDeviceToHost,
                            st) == hipSuccess;
      }
      if (ok) ok = hipStreamSynchronize(st) == hipSuccess;
      if (!ok) fail_all(BDDC_ERR_DEVICE, "copy of the solution");
      for (int q = 0; q < m && ok; ++q) {
        infos[q]->pcg = pinfo[q];
        infos[q]->batch = m;
        if (!pinfo[q].converged) {
          infos[q]->status = BDDC_ERR_NO_CONVERGENCE;
          std::snprintf(infos[q]->error, sizeof infos[q]->error,
                        "pcg: PCG did not reach the tolerance");
        }
      }
    }
  }
  if (fd) async_free(fd, st);
  if (ud) async_free(ud, st);
  (void)hipStreamSynchronize(st);
}

void bddc_server::worker() {
  (void)hipSetDevice(opt.device);
  hipStream_t wst = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&wst, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    std::vector<Request *> batch;
    Resident *res = nullptr;
    bool fresh = true;  // the context is built for this batch
    std::vector<std::unique_ptr<Resident>> victims;
    {
      std::unique_lock<std::mutex> lk(m);
      cv_work.wait(lk, [&] { return head_admissible() || (stopping && queue.empty()); });
      if (queue.empty()) break;
      Request *h = queue.front();
      res = find_resident(*h);
      if (res) {
        // resident and idle: take the queued requests on this problem
        res->busy = true;
        fresh = false;
        for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < kMaxTaken;) {
          if (find_resident(**it) == res) {
            batch.push_back(*it);
            it = queue.erase(it);
          } else {
            ++it;
          }
        }
      } else {
        queue.pop_front();
        batch.push_back(h);
        const double fp = h->info.footprint_bytes;
        evict_while([&](double freed) { return reserved - freed + fp > opt.hbm_budget_bytes; },
                    victims);
        reserved += fp;
        if (keep_resident()) {
          // registered now, so requests on the same problem wait for it
          // instead of factoring it again
          auto e = std::make_unique<Resident>();
          e->serial = ++resident_serial;
          e->proto = std::make_unique<Request>(*h);
          e->proto->f.clear();
          e->proto->mesh.xyz = e->proto->xyz.data();  // its own copies
          e->proto->mesh.hex8 = e->proto->hex8.data();
          e->proto->mesh.coef = e->proto->coef.data();
          e->proto->mesh.dirichlet = e->proto->dirichlet.data();
          e->footprint = fp;
          res = e.get();
          resident.push_back(std::move(e));
        }
      }
      running++;
      for (Request *r : batch) {
        r->info.state = 1;
        r->info.start_s = now();
      }
    }
    cv_work.notify_all();  // the new head may be admissible too
    release_destroyed(victims);
    std::vector<bddc_request_info> out(batch.size());
    std::vector<std::vector<double>> us(batch.size());
    {
      std::lock_guard<std::mutex> lk(m);
      for (size_t i = 0; i < batch.size(); ++i) out[i] = batch[i]->info;
    }
    bddc_ctx *c = res ? res->ctx : nullptr;
    hipStream_t st = (res && !fresh) ? res->st : wst;
    bool ok = true;
    if (fresh) {
      // a resident context gets a stream of its own (any worker may use it later)
      bool stream_ok = have_stream;
      if (res) {
        stream_ok = hipStreamCreateWithFlags(&res->st, hipStreamNonBlocking) == hipSuccess;
        if (!stream_ok) res->st = nullptr;
        st = res->st;
      }
      if (!stream_ok) {
        out[0].status = BDDC_ERR_DEVICE;
        std::snprintf(out[0].error, sizeof out[0].error, "stream creation failed");
        ok = false;
      } else {
        c = build(*batch[0], out[0], st);
        ok = c != nullptr;
        if (ok && res) {
          res->ctx = c;
          res->omega = out[0].omega;
          res->nc = out[0].nc;
        }
      }
    }
    // the taken requests in blocks of equal PCG parameters (arrival order
    // within each), each block published as soon as it is solved
    std::vector<char> published(batch.size(), 0);
    if (ok) {
      std::vector<size_t> order(batch.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        const bddc_pcg_params &x = batch[a]->params, &y = batch[b]->params;
        return x.rtol != y.rtol ? x.rtol < y.rtol : x.maxit < y.maxit;
      });
      for (size_t i0 = 0; i0 < order.size();) {
        size_t i1 = i0 + 1;
        while (i1 < order.size() && (int)(i1 - i0) < kBlockRhs &&
               same_params(*batch[order[i1]], *batch[order[i0]]))
          ++i1;
        std::vector<Request *> rs;
        std::vector<bddc_request_info *> infos;
        std::vector<std::vector<double> *> uv;
        for (size_t k = i0; k < i1; ++k) {
          const size_t i = order[k];
          if (!fresh) {
            out[i].omega = res->omega;
            out[i].nc = res->nc;
            out[i].reused = 1;
          }
          rs.push_back(batch[i]);
          infos.push_back(&out[i]);
          uv.push_back(&us[i]);
        }
        solve(c, rs, infos, uv, st);
        {
          std::lock_guard<std::mutex> lk(m);
          for (size_t k = i0; k < i1; ++k) {
            const size_t i = order[k];
            Request *r = batch[i];
            r->info = out[i];
            r->u.swap(us[i]);
            r->info.done_s = now();
            r->info.state = r->info.status == BDDC_OK ? 2 : 3;
            published[i] = 1;
          }
        }
        cv_done.notify_all();
        i0 = i1;
      }
    }
    // a context of its own is freed before its footprint is returned
    if (!res && c) {
      bddc_destroy(c);
      (void)hipStreamSynchronize(st);
    }
    std::vector<std::unique_ptr<Resident>> dropped;
    {
      std::lock_guard<std::mutex> lk(m);
      for (size_t i = 0; i < batch.size(); ++i) {
        if (published[i]) continue;
        Request *r = batch[i];
        r->info = out[i];
        if (!ok && i > 0) {
          r->info.status = out[0].status;
          std::memcpy(r->info.error, out[0].error, sizeof r->info.error);
        }
        r->u.swap(us[i]);
        r->info.done_s = now();
        r->info.state = r->info.status == BDDC_OK ? 2 : 3;
      }
      running--;
      if (res) {
        if (ok) {
          res->busy = false;
          res->last_used = ++use_clock;
          // keep the idle contexts within their own limit
          evict_while([&](double freed) { return idle_resident_bytes() > opt.resident_bytes; },
                      dropped);
        } else {
          for (size_t i = 0; i < resident.size(); ++i)
            if (resident[i].get() == res) {
              dropped.push_back(std::move(resident[i]));
              resident.erase(resident.begin() + i);
              break;
            }
        }
      } else {
        reserved -= batch[0]->info.footprint_bytes;
      }
    }
    cv_done.notify_all();
    release_destroyed(dropped);
    cv_work.notify_all();
  }
  if (have_stream) (void)hipStreamDestroy(wst);
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
  // a request that alone exceeds the admission budget could never start
  if (r->info.footprint_bytes > srv->opt.hbm_budget_bytes) return BDDC_ERR_OOM;
  r->info.n_glob = n_glob;
  r->key = problem_key(*r);
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
  destroy_resident(srv->resident);
  delete srv;
}

}  // extern "C"
