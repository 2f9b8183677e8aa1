// Interface classification into faces, edges and corners (Sec. 2: a face holds
// the nodes shared by exactly one pair of substructures, an edge the nodes
// shared by the same set of more than two, a corner is a one-node edge), and
// the weights of the averaging operator E (proportional to the diagonal of
// the substructure matrices, Sec. 7).
//
// Where the paper is silent: nodes of >2-substructure classes lying on the
// domain boundary are corners too; for irregular partitions face nodes are
// promoted to corners greedily until every face pair sees 1 (scalar) or 3
// non-collinear (elasticity) corners (Assumptions 1 and 2).  Classification
// is done on the full mesh; Dirichlet dofs are removed afterwards and globs
// without free dofs vanish.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <set>
#include <unordered_map>

#include "host.h"
#include "solver.h"

namespace bddc {

namespace {

struct ArrHash {
  size_t operator()(const std::array<int64_t, 4> &a) const {
    size_t h = 1469598103934665603ull;
    for (int64_t v : a) h = (h ^ (size_t)v) * 1099511628211ull;
    return h;
  }
};

std::vector<uint8_t> boundary_nodes(const MeshIn &m) {
  static const int fl[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4},
                               {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
  std::unordered_map<std::array<int64_t, 4>, int, ArrHash> cnt;
  cnt.reserve(m.n_elems * 4);
  for (int64_t e = 0; e < m.n_elems; ++e)
    for (int f = 0; f < 6; ++f) {
      std::array<int64_t, 4> k;
      for (int a = 0; a < 4; ++a) k[a] = m.hex8[8 * e + fl[f][a]];
      std::sort(k.begin(), k.end());
      cnt[k]++;
    }
  std::vector<uint8_t> b(m.n_nodes, 0);
  for (auto &kv : cnt)
    if (kv.second == 1)
      for (int64_t n : kv.first) b[n] = 1;
  return b;
}

// 0 (none), 1 (one point), 2 (collinear), 3 (three non-collinear points)
int noncollinear_count(const std::vector<std::array<double, 3>> &p) {
  if (p.empty()) return 0;
  double far = 0;
  size_t k1 = 0;
  for (size_t k = 1; k < p.size(); ++k) {
    double d = 0;
    for (int c = 0; c < 3; ++c) d = std::max(d, std::fabs(p[k][c] - p[0][c]));
    if (d > far) far = d, k1 = k;
  }
  if (far < 1e-12) return 1;
  double u[3] = {p[k1][0] - p[0][0], p[k1][1] - p[0][1], p[k1][2] - p[0][2]};
  double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (size_t k = 1; k < p.size(); ++k) {
    double v[3] = {p[k][0] - p[0][0], p[k][1] - p[0][1], p[k][2] - p[0][2]};
    double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
           cz = u[0] * v[1] - u[1] * v[0];
    double vn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (std::sqrt(cx * cx + cy * cy + cz * cz) > 1e-9 * un * std::max(vn, 1e-300)) return 3;
  }
  return 2;
}

}  // namespace

void classify_interface(Problem &P, bool augment) {
  const MeshIn &m = P.mesh;
  const int dpn = m.dpn;
  // substructures of every node
  std::vector<std::vector<int>> ns(m.n_nodes);
  for (int64_t e = 0; e < m.n_elems; ++e)
    for (int a = 0; a < 8; ++a) {
      auto &v = ns[m.hex8[8 * e + a]];
      int s = m.elem_sub[e];
      if (std::find(v.begin(), v.end(), s) == v.end()) v.push_back(s);
    }
  for (auto &v : ns) std::sort(v.begin(), v.end());
  auto bnd = boundary_nodes(m);

  std::map<std::vector<int>, std::vector<int64_t>> classes;
  for (int64_t n = 0; n < m.n_nodes; ++n)
    if (ns[n].size() > 1) classes[ns[n]].push_back(n);

  std::set<int64_t> corner;
  std::vector<std::pair<std::vector<int>, std::vector<int64_t>>> edges, faces;
  for (auto &kv : classes) {
    const auto &key = kv.first;
    const auto &nodes = kv.second;
    if (key.size() == 2) {
      faces.push_back(kv);
    } else if (nodes.size() == 1) {
      corner.insert(nodes[0]);
    } else {
      std::vector<int64_t> rest;
      for (int64_t n : nodes) {
        if (bnd[n])
          corner.insert(n);
        else
          rest.push_back(n);
      }
      if (!rest.empty()) edges.push_back({key, rest});
    }
  }

  const int need = m.kind == 0 ? 1 : 3;
  std::map<std::pair<int, int>, std::vector<int64_t>> shared;
  for (int64_t n = 0; n < m.n_nodes; ++n) {
    const auto &s = ns[n];
    if (s.size() < 2) continue;
    for (size_t a = 0; a < s.size(); ++a)
      for (size_t b = a + 1; b < s.size(); ++b) shared[{s[a], s[b]}].push_back(n);
  }
  auto pt = [&](int64_t n) {
    return std::array<double, 3>{m.xyz[3 * n], m.xyz[3 * n + 1], m.xyz[3 * n + 2]};
  };
  if (!augment) {
    // Assumption 2 (Sec. 3): the corners shared by two adjacent substructures
    // must remove their relative rigid body motions: at least one corner
    // (scalar) or three non-collinear corners (elasticity) in the closure of
    // the pair's face, unless neither substructure floats (both carry
    // Dirichlet dofs, so the pair has no rigid motion).  Without the corner
    // augmentation a partition that breaks it is rejected here.
    std::vector<char> fixed(m.n_sub, 0);
    for (int64_t e = 0; e < m.n_elems; ++e)
      for (int a = 0; a < 8 && !fixed[m.elem_sub[e]]; ++a)
        for (int c = 0; c < dpn; ++c)
          if (m.dirichlet[dpn * m.hex8[8 * e + a] + c]) fixed[m.elem_sub[e]] = 1;
    for (auto &f : faces) {
      const int i = f.first[0], j = f.first[1];
      if (fixed[i] && fixed[j]) continue;
      std::vector<std::array<double, 3>> cpts;
      for (int64_t n : shared[{i, j}])
        if (corner.count(n)) cpts.push_back(pt(n));
      const int have = noncollinear_count(cpts);
      if (have < need)
        throw CornersError("face pair (" + std::to_string(i) + ", " + std::to_string(j) +
                           ") sees " + std::to_string(have) + " independent corner(s), " +
                           std::to_string(need) + " needed (Assumption 2); set augment_corners");
    }
  }
  if (augment) {
    for (auto &f : faces) {
      const auto &cl = shared[{f.first[0], f.first[1]}];
      std::vector<std::array<double, 3>> cpts;
      for (int64_t n : cl)
        if (corner.count(n)) cpts.push_back(pt(n));
      std::vector<int64_t> cand;
      for (int64_t n : f.second)
        if (!corner.count(n)) cand.push_back(n);
      if (noncollinear_count(cpts) >= need || cand.empty()) continue;
      double cen[3] = {0, 0, 0};
      for (int64_t n : cand)
        for (int c = 0; c < 3; ++c) cen[c] += m.xyz[3 * n + c];
      for (int c = 0; c < 3; ++c) cen[c] /= (double)cand.size();
      while (noncollinear_count(cpts) < need && !cand.empty()) {
        std::vector<double> dist(cand.size());
        for (size_t k = 0; k < cand.size(); ++k) {
          const int64_t n = cand[k];
          double d;
          if (cpts.empty()) {
            d = 0;
            for (int c = 0; c < 3; ++c) {
              double t = m.xyz[3 * n + c] - cen[c];
              d += t * t;
            }
          } else {
            d = INFINITY;
            for (auto &q : cpts) {
              double dd = 0;
              for (int c = 0; c < 3; ++c) {
                double t = m.xyz[3 * n + c] - q[c];
                dd += t * t;
              }
              d = std::min(d, dd);
            }
          }
          dist[k] = d;
        }
        // nearest the centroid (no corner yet) or farthest from the corners;
        // distances equal within 1e-9 relative are ties, won by the lowest id
        size_t best = 0;
        if (cpts.empty()) {
          double dm = *std::min_element(dist.begin(), dist.end());
          while (!(dist[best] <= dm * (1 + 1e-9) + 1e-300)) ++best;
        } else {
          double dm = *std::max_element(dist.begin(), dist.end());
          while (!(dist[best] >= dm * (1 - 1e-9))) ++best;
        }
        int64_t n = cand[best];
        cand.erase(cand.begin() + best);
        corner.insert(n);
        cpts.push_back(pt(n));
      }
    }
  }

  auto free_dofs = [&](const std::vector<int64_t> &nodes, std::vector<int64_t> &d,
                       std::vector<int> &comp) {
    for (int64_t n : nodes)
      for (int c = 0; c < dpn; ++c) {
        int64_t g = P.full2glob[dpn * n + c];
        if (g >= 0) d.push_back(g), comp.push_back(c);
      }
  };
  P.corner_nodes.clear();
  P.corner_gdofs.clear();
  for (int64_t n : corner) {
    std::vector<int64_t> d;
    std::vector<int> c;
    free_dofs({n}, d, c);
    if (d.empty()) continue;
    P.corner_nodes.push_back(n);
    P.corner_gdofs.insert(P.corner_gdofs.end(), d.begin(), d.end());
  }
  std::sort(P.corner_gdofs.begin(), P.corner_gdofs.end());
  P.globs.clear();
  P.face_ids.clear();
  P.edge_ids.clear();
  for (int kind : {GLOB_EDGE, GLOB_FACE}) {
    auto &lst = kind == GLOB_EDGE ? edges : faces;
    for (auto &kv : lst) {
      std::vector<int64_t> nodes;
      for (int64_t n : kv.second)
        if (!corner.count(n)) nodes.push_back(n);
      if (nodes.empty()) continue;
      Glob g;
      g.kind = kind;
      g.subs = kv.first;
      g.nodes = nodes;
      free_dofs(nodes, g.dofs, g.comp);
      if (g.dofs.empty()) continue;
      (kind == GLOB_EDGE ? P.edge_ids : P.face_ids).push_back((int)P.globs.size());
      P.globs.push_back(std::move(g));
    }
  }
  // glob and corner positions inside every substructure's interface
  for (auto &S : P.subs) {
    S.glob_ids.clear();
    S.glob_pos.clear();
    S.corner_pos.clear();
    S.corner_gdof.clear();
  }
  for (int gi = 0; gi < (int)P.globs.size(); ++gi) {
    const Glob &g = P.globs[gi];
    for (int s : g.subs) {
      Sub &S = P.subs[s];
      auto b = S.gdof.begin() + S.nI, e = S.gdof.end();
      std::vector<int> pos(g.dofs.size());
      for (size_t t = 0; t < g.dofs.size(); ++t) {
        auto it = std::lower_bound(b, e, g.dofs[t]);
        pos[t] = (int)(it - b);
      }
      S.glob_ids.push_back(gi);
      S.glob_pos.push_back(std::move(pos));
    }
  }
  for (auto &S : P.subs) {
    auto b = S.gdof.begin() + S.nI, e = S.gdof.end();
    for (int64_t g : P.corner_gdofs) {
      auto it = std::lower_bound(b, e, g);
      if (it != e && *it == g) {
        S.corner_pos.push_back((int)(it - b));
        S.corner_gdof.push_back(g);
      }
    }
  }
}

void compute_weights(Problem &P) {
  std::vector<double> dsum(P.n_glob, 0.0);
  for (auto &S : P.subs)
    for (int l = 0; l < S.nI + S.nG; ++l) dsum[S.gdof[l]] += S.diag[l];
  for (auto &S : P.subs) {
    S.delta.resize(S.nG);
    for (int t = 0; t < S.nG; ++t) S.delta[t] = S.diag[S.nI + t] / dsum[S.gdof[S.nI + t]];
  }
}

}  // namespace bddc
