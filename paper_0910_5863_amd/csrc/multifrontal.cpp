// Symbolic multifrontal analysis: nested dissection of each substructure's
// interior and the front structure (see multifrontal.h).
#include "multifrontal.h"

#include <algorithm>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace bddc {

namespace {

// One substructure's analysis in local numbering (local dof ids 0..n, the
// interior ones below nI).
struct LocalFront {
  std::vector<int> piv, bnd;  // local dof ids, ascending
  std::vector<int> children;  // local front ids
  int parent = -1, depth = 1;
};

struct LocalResult {
  std::vector<LocalFront> fronts;  // post-order: children before parents
  std::vector<int> top;            // children of the interface root
  std::vector<int> asm_front;      // per CSR entry: front of the entry, -1: skip
  std::vector<int64_t> asm_idx;    // index inside the front's U block
};

struct Tree {
  std::vector<std::vector<int>> nodes;  // pivot nodes per tree vertex
  std::vector<std::vector<int>> kids;
};

class Dissector {
 public:
  Dissector(const std::vector<double> &xyz, const std::vector<std::vector<int>> &adj, int leaf)
      : xyz_(xyz), adj_(adj), leaf_(leaf), stamp_(adj.size(), 0) {}

  // returns the tree vertex of V's subtree (vertices are appended in post-order)
  int build(std::vector<int> V, Tree &T) {
    if ((int)V.size() > leaf_) {
      // axes by decreasing extent
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int v : V)
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], xyz_[3 * v + a]);
          hi[a] = std::max(hi[a], xyz_[3 * v + a]);
        }
      int order[3] = {0, 1, 2};
      std::stable_sort(order, order + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
      for (int oi = 0; oi < 3; ++oi) {
        const int a = order[oi];
        if (!(hi[a] > lo[a])) break;
        std::vector<int> S = V;
        std::sort(S.begin(), S.end(), [&](int x, int y) {
          const double cx = xyz_[3 * x + a], cy = xyz_[3 * y + a];
          return cx < cy || (cx == cy && x < y);
        });
        const double c = xyz_[3 * S[S.size() / 2] + a];
        std::vector<int> L, R;
        for (int v : V) (xyz_[3 * v + a] < c ? L : R).push_back(v);
        if (L.empty() || R.empty()) continue;
        ++cur_;
        for (int v : L) stamp_[v] = cur_;
        std::vector<int> sep, rest;
        for (int v : R) {
          bool touches = false;
          for (int w : adj_[v])
            if (stamp_[w] == cur_) {
              touches = true;
              break;
            }
          (touches ? sep : rest).push_back(v);
        }
        std::vector<int> kids;
        kids.push_back(build(std::move(L), T));
        if (!rest.empty()) kids.push_back(build(std::move(rest), T));
        T.nodes.push_back(std::move(sep));
        T.kids.push_back(std::move(kids));
        return (int)T.nodes.size() - 1;
      }
    }
    T.nodes.push_back(std::move(V));
    T.kids.push_back({});
    return (int)T.nodes.size() - 1;
  }

 private:
  const std::vector<double> &xyz_;
  const std::vector<std::vector<int>> &adj_;
  int leaf_;
  std::vector<int> stamp_;
  int cur_ = 0;
};

LocalResult analyze_sub(const Problem &P, int s, int leaf) {
  const Sub &S = P.subs[s];
  const Csr &A = S.A;
  const int n = A.n, nI = S.nI, dpn = P.mesh.dpn;
  LocalResult res;
  res.asm_front.assign(A.col.size(), -1);
  res.asm_idx.assign(A.col.size(), -1);
  if (nI == 0) return res;
  // interior nodes
  std::vector<int64_t> node_of(nI);
  for (int u = 0; u < nI; ++u) node_of[u] = P.glob2full[S.gdof[u]] / dpn;
  std::vector<int64_t> un(node_of);
  std::sort(un.begin(), un.end());
  un.erase(std::unique(un.begin(), un.end()), un.end());
  const int nn = (int)un.size();
  std::vector<int> lnode(nI);
  for (int u = 0; u < nI; ++u)
    lnode[u] = (int)(std::lower_bound(un.begin(), un.end(), node_of[u]) - un.begin());
  std::vector<std::vector<int>> dofs(nn), adj(nn);
  for (int u = 0; u < nI; ++u) dofs[lnode[u]].push_back(u);
  for (int u = 0; u < nI; ++u)
    for (int k = A.ptr[u]; k < A.ptr[u + 1]; ++k) {
      const int w = A.col[k];
      if (w < nI && lnode[w] != lnode[u]) adj[lnode[u]].push_back(lnode[w]);
    }
  for (auto &a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  std::vector<double> xyz(3 * (size_t)nn);
  for (int v = 0; v < nn; ++v)
    for (int a = 0; a < 3; ++a) xyz[3 * v + a] = P.mesh.xyz[3 * un[v] + a];
  // dissection
  Tree T;
  Dissector D(xyz, adj, leaf);
  std::vector<int> all(nn);
  std::iota(all.begin(), all.end(), 0);
  const int top = D.build(std::move(all), T);
  const int nf = (int)T.nodes.size();
  res.fronts.resize(nf);
  res.top = {top};
  // fronts in post-order: pivots, boundary (vars adjacent to the subtree and
  // not eliminated in it)
  std::vector<char> elim(n, 0);
  std::vector<int> mark(n, -1), fpos(n, -1);
  for (int t = 0; t < nf; ++t) {
    LocalFront &F = res.fronts[t];
    for (int v : T.nodes[t]) F.piv.insert(F.piv.end(), dofs[v].begin(), dofs[v].end());
    std::sort(F.piv.begin(), F.piv.end());
    F.children = T.kids[t];
    for (int u : F.piv) mark[u] = t;  // pivots are not boundary
    auto add = [&](int w) {
      if (mark[w] != t && !elim[w]) {
        mark[w] = t;
        F.bnd.push_back(w);
      }
    };
    for (int u : F.piv)
      for (int k = A.ptr[u]; k < A.ptr[u + 1]; ++k) add(A.col[k]);
    for (int c : F.children) {
      res.fronts[c].parent = t;
      for (int w : res.fronts[c].bnd) add(w);
    }
    std::sort(F.bnd.begin(), F.bnd.end());
    // assembly of the pivot rows: (u, w) goes to U[pos_u, pos_w] when w is
    // a variable of this front (otherwise it was eliminated below and the
    // descendant assembled (w, u))
    const int p = (int)F.piv.size();
    for (int i = 0; i < p; ++i) fpos[F.piv[i]] = i;
    for (size_t j = 0; j < F.bnd.size(); ++j) fpos[F.bnd[j]] = p + (int)j;
    for (int i = 0; i < p; ++i) {
      const int u = F.piv[i];
      for (int k = A.ptr[u]; k < A.ptr[u + 1]; ++k) {
        const int w = A.col[k];
        if (elim[w]) continue;
        res.asm_front[k] = t;
        res.asm_idx[k] = i + (int64_t)fpos[w] * p;
      }
    }
    for (int u : F.piv) elim[u] = 1;
  }
  for (int u = 0; u < nI; ++u)
    if (!elim[u]) throw std::runtime_error("nested dissection: an interior dof is not a pivot");
  // depths
  for (int t = nf - 1; t >= 0; --t) {
    LocalFront &F = res.fronts[t];
    F.depth = F.parent < 0 ? 1 : res.fronts[F.parent].depth + 1;
  }
  return res;
}

}  // namespace

MfSymbolic mf_analyze(const Problem &P, const std::vector<int64_t> &offI, int leaf_nodes) {
  const int ns = (int)P.subs.size();
  std::vector<LocalResult> loc(ns);
  {
    const int nt = std::max(1, std::min<int>(ns, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    std::vector<std::string> err(nt);
    for (int w = 0; w < nt; ++w)
      th.emplace_back([&, w] {
        try {
          for (int s = w; s < ns; s += nt) loc[s] = analyze_sub(P, s, leaf_nodes);
        } catch (const std::exception &e) {
          err[w] = e.what();
        }
      });
    for (auto &t : th) t.join();
    for (auto &e : err)
      if (!e.empty()) throw std::runtime_error(e);
  }
  MfSymbolic M;
  M.root_ptr.assign(ns + 1, 0);
  std::vector<int> base(ns);
  int64_t nnz_total = 0;
  for (int s = 0; s < ns; ++s) nnz_total += (int64_t)P.subs[s].A.col.size();
  M.asm_dst.assign(nnz_total, -1);
  int64_t nnz_off = 0;
  for (int s = 0; s < ns; ++s) {
    const Sub &S = P.subs[s];
    const LocalResult &R = loc[s];
    base[s] = (int)M.fronts.size();
    for (size_t t = 0; t < R.fronts.size(); ++t) {
      const LocalFront &L = R.fronts[t];
      MfFront F;
      F.sub = s;
      F.depth = L.depth;
      F.p = (int)L.piv.size();
      F.b = (int)L.bnd.size();
      F.parent = L.parent < 0 ? -1 : base[s] + L.parent;
      F.u_off = M.u_size;
      F.c_off = M.c_size;
      F.piv_off = (int64_t)M.piv.size();
      F.bnd_off = (int64_t)M.bnd.size();
      F.upd_off = M.upd_size;
      const int64_t f = F.p + F.b;
      M.u_size += (int64_t)F.p * f;
      M.c_size += (int64_t)F.b * F.b;
      M.upd_size += F.b;
      for (int u : L.piv) M.piv.push_back(offI[s] + u);
      for (int w : L.bnd) M.bnd.push_back(w < S.nI ? offI[s] + w : -1);
      F.child_ptr = (int)M.child_ids.size();
      F.n_child = (int)L.children.size();
      for (int c : L.children) M.child_ids.push_back(base[s] + c);
      M.max_depth = std::max(M.max_depth, F.depth);
      M.max_p = std::max(M.max_p, F.p);
      M.max_b = std::max(M.max_b, F.b);
      const double p = F.p, b = F.b;
      M.flops += p * p * p / 3 + p * p * b + p * b * b;
      M.l_entries += 0.5 * p * (p + 1) + p * b;
      M.fronts.push_back(F);
    }
    for (int t : R.top) M.root_ids.push_back(base[s] + t);
    M.root_ptr[s + 1] = (int)M.root_ids.size();
    for (size_t k = 0; k < R.asm_front.size(); ++k)
      if (R.asm_front[k] >= 0)
        M.asm_dst[nnz_off + k] = M.fronts[base[s] + R.asm_front[k]].u_off + R.asm_idx[k];
    nnz_off += (int64_t)S.A.col.size();
  }
  // pull maps: for every front, the parent's variables (pivots, then
  // boundary; the interface positions for the root) -> own boundary index
  std::vector<int> pos;
  for (int s = 0; s < ns; ++s) {
    const Sub &S = P.subs[s];
    const LocalResult &R = loc[s];
    pos.assign(S.A.n, -1);
    for (size_t t = 0; t < R.fronts.size(); ++t) {
      const LocalFront &L = R.fronts[t];
      MfFront &F = M.fronts[base[s] + t];
      for (size_t j = 0; j < L.bnd.size(); ++j) pos[L.bnd[j]] = (int)j;
      F.pmap_off = (int64_t)M.pmap.size();
      if (L.parent < 0) {
        for (int j = 0; j < S.nG; ++j) M.pmap.push_back(pos[S.nI + j]);
      } else {
        const LocalFront &Pa = R.fronts[L.parent];
        for (int v : Pa.piv) M.pmap.push_back(pos[v]);
        for (int v : Pa.bnd) M.pmap.push_back(pos[v]);
      }
      for (int w : L.bnd) pos[w] = -1;
    }
  }
  M.levels.assign(M.max_depth + 1, {});
  for (size_t t = 0; t < M.fronts.size(); ++t) M.levels[M.fronts[t].depth].push_back((int)t);
  return M;
}

}  // namespace bddc
