// Q1 hexahedral element matrices and the substructure matrices A_i (Sec. 2,
// eq. (block-operators): A_i is the subassembly of element matrices of the
// elements of substructure i only).
#include <algorithm>
#include <cmath>
#include <thread>

#include "host.h"

namespace bddc {

namespace {

const double kRef[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                           {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

void inv3(const double J[3][3], double Ji[3][3], double &det) {
  det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double id = 1.0 / det;
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
}

}  // namespace

// Element stiffness by the 2x2x2 Gauss rule; K is (8 dpn) x (8 dpn) row-major.
void element_matrix(const MeshIn &m, int64_t e, double *K) {
  const int dpn = m.dpn;
  const int nd = 8 * dpn;
  std::fill(K, K + nd * nd, 0.0);
  double X[8][3];
  for (int a = 0; a < 8; ++a)
    for (int d = 0; d < 3; ++d) X[a][d] = m.xyz[3 * m.hex8[8 * e + a] + d];
  const double g = 1.0 / std::sqrt(3.0);
  const double coef = m.coef[e];
  double lam = 0, mu = 0;
  if (m.kind == 1) {
    const double nu = m.nu;
    lam = coef * nu / ((1 + nu) * (1 - 2 * nu));
    mu = coef / (2 * (1 + nu));
  }
  for (int q = 0; q < 8; ++q) {
    const double p[3] = {(q & 1) ? g : -g, (q & 2) ? g : -g, (q & 4) ? g : -g};
    double dr[8][3];
    for (int a = 0; a < 8; ++a) {
      const double xa = kRef[a][0], ya = kRef[a][1], za = kRef[a][2];
      dr[a][0] = xa * (1 + ya * p[1]) * (1 + za * p[2]) * 0.125;
      dr[a][1] = ya * (1 + xa * p[0]) * (1 + za * p[2]) * 0.125;
      dr[a][2] = za * (1 + xa * p[0]) * (1 + ya * p[1]) * 0.125;
    }
    double J[3][3] = {{0}};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int a = 0; a < 8; ++a) J[i][j] += dr[a][i] * X[a][j];
    double Ji[3][3], det;
    inv3(J, Ji, det);
    double G[8][3];  // physical gradients
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 3; ++i)
        G[a][i] = Ji[i][0] * dr[a][0] + Ji[i][1] * dr[a][1] + Ji[i][2] * dr[a][2];
    if (m.kind == 0) {
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b)
          K[a * nd + b] += coef * det * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
    } else {
      // K_ab(i,j) = lam dNa_i dNb_j + mu dNa_j dNb_i + mu delta_ij (dNa . dNb)
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
          const double dot = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
              double v = lam * G[a][i] * G[b][j] + mu * G[a][j] * G[b][i];
              if (i == j) v += mu * dot;
              K[(3 * a + i) * nd + 3 * b + j] += det * v;
            }
        }
    }
  }
}

// Builds, for every substructure: local dof numbering (interior first, then
// interface, each ascending in global order), the CSR matrix A_i and diag.
// Requires P.full2glob and the node multiplicities (computed here).
void assemble_substructures(Problem &P) {
  const MeshIn &m = P.mesh;
  const int dpn = m.dpn;
  const int nd = 8 * dpn;
  // elements and node multiplicity per substructure
  std::vector<std::vector<int64_t>> elems(m.n_sub);
  for (int64_t e = 0; e < m.n_elems; ++e) elems[m.elem_sub[e]].push_back(e);
  std::vector<std::vector<int64_t>> sub_nodes(m.n_sub);
  parallel_for(m.n_sub, [&](int s) {
    auto &v = sub_nodes[s];
    for (int64_t e : elems[s])
      for (int a = 0; a < 8; ++a) v.push_back(m.hex8[8 * e + a]);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  });
  std::vector<int> mult(m.n_nodes, 0);
  for (int s = 0; s < m.n_sub; ++s)
    for (int64_t n : sub_nodes[s]) mult[n]++;

  P.subs.assign(m.n_sub, Sub());
  parallel_for(m.n_sub, [&](int s) {
    Sub &S = P.subs[s];
    const auto &nodes = sub_nodes[s];
    std::vector<int64_t> intr, itf;
    bool has_dir = false;
    for (int64_t n : nodes)
      for (int c = 0; c < dpn; ++c) {
        int64_t g = P.full2glob[dpn * n + c];
        if (g < 0) {
          has_dir = true;
          continue;
        }
        (mult[n] > 1 ? itf : intr).push_back(g);
      }
    S.floating = !has_dir;
    S.nI = (int)intr.size();
    S.nG = (int)itf.size();
    S.gdof = intr;
    S.gdof.insert(S.gdof.end(), itf.begin(), itf.end());
    const int n = S.nI + S.nG;
    // global dof -> local via binary search over the two sorted halves
    auto local_of = [&](int64_t g, int64_t node) -> int {
      if (mult[node] > 1) {
        auto it = std::lower_bound(itf.begin(), itf.end(), g);
        return S.nI + (int)(it - itf.begin());
      }
      auto it = std::lower_bound(intr.begin(), intr.end(), g);
      return (int)(it - intr.begin());
    };
    // pattern: for each local row the set of local columns
    std::vector<std::vector<int>> cols(n);
    std::vector<int> ld(nd);
    for (int64_t e : elems[s]) {
      for (int a = 0; a < 8; ++a) {
        int64_t node = m.hex8[8 * e + a];
        for (int c = 0; c < dpn; ++c) {
          int64_t g = P.full2glob[dpn * node + c];
          ld[a * dpn + c] = g < 0 ? -1 : local_of(g, node);
        }
      }
      for (int i = 0; i < nd; ++i) {
        if (ld[i] < 0) continue;
        for (int j = 0; j < nd; ++j)
          if (ld[j] >= 0) cols[ld[i]].push_back(ld[j]);
      }
    }
    Csr &A = S.A;
    A.n = n;
    A.ptr.assign(n + 1, 0);
    for (int r = 0; r < n; ++r) {
      auto &c = cols[r];
      std::sort(c.begin(), c.end());
      c.erase(std::unique(c.begin(), c.end()), c.end());
      A.ptr[r + 1] = A.ptr[r] + (int)c.size();
    }
    A.col.resize(A.ptr[n]);
    for (int r = 0; r < n; ++r) std::copy(cols[r].begin(), cols[r].end(), A.col.begin() + A.ptr[r]);
    A.val.assign(A.ptr[n], 0.0);
    std::vector<double> Ke(nd * nd);
    for (int64_t e : elems[s]) {
      element_matrix(m, e, Ke.data());
      for (int a = 0; a < 8; ++a) {
        int64_t node = m.hex8[8 * e + a];
        for (int c = 0; c < dpn; ++c) {
          int64_t g = P.full2glob[dpn * node + c];
          ld[a * dpn + c] = g < 0 ? -1 : local_of(g, node);
        }
      }
      for (int i = 0; i < nd; ++i) {
        const int r = ld[i];
        if (r < 0) continue;
        const int *cb = A.col.data() + A.ptr[r];
        const int *ce = A.col.data() + A.ptr[r + 1];
        for (int j = 0; j < nd; ++j) {
          if (ld[j] < 0) continue;
          const int *pos = std::lower_bound(cb, ce, ld[j]);
          A.val[pos - A.col.data()] += Ke[i * nd + j];
        }
      }
    }
    S.diag.assign(n, 0.0);
    for (int r = 0; r < n; ++r)
      for (int k = A.ptr[r]; k < A.ptr[r + 1]; ++k)
        if (A.col[k] == r) S.diag[r] = A.val[k];
  });
}

}  // namespace bddc
