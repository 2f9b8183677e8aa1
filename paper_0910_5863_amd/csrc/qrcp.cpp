// Generalized change of variables (Sec. 5): Householder QR with column
// pivoting of each glob's constraint rows, H = Q [U V] K, and the inverse
// change of variables T = K^-1 [U^-1  -U^-1 V; 0  I] (eq. (T)).  Rows whose
// |U_kk| is negligible against |U_11| are dropped as numerically redundant.
#include <algorithm>
#include <cmath>

#include "host.h"

namespace bddc {

// H: m x n row-major.  Pivot: the trailing column of largest 2-norm, first
// one on ties.  A reflector is the identity when the part of the column
// below the diagonal is already zero (so a single unit-weight average gives
// U = [1], K = I, the worked example of Sec. 5).
GlobCov qr_change_of_variables(const std::vector<double> &H, int m, int n, double drop_tol) {
  GlobCov c;
  c.n = n;
  c.perm.resize(n);
  for (int j = 0; j < n; ++j) c.perm[j] = j;
  if (m == 0 || n == 0) {
    c.m = 0;
    return c;
  }
  // column-major working copy
  std::vector<double> A((size_t)m * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)j * m + i] = H[(size_t)i * n + j];
  const int kmax = std::min(m, n);
  std::vector<double> v(m);
  for (int k = 0; k < kmax; ++k) {
    int piv = k;
    double best = -1;
    for (int j = k; j < n; ++j) {
      double s = 0;
      for (int i = k; i < m; ++i) s += A[(size_t)j * m + i] * A[(size_t)j * m + i];
      if (s > best) best = s, piv = j;
    }
    if (piv != k) {
      for (int i = 0; i < m; ++i) std::swap(A[(size_t)k * m + i], A[(size_t)piv * m + i]);
      std::swap(c.perm[k], c.perm[piv]);
    }
    double *x = &A[(size_t)k * m];
    double alpha = x[k];
    double xn = 0;
    for (int i = k + 1; i < m; ++i) xn += x[i] * x[i];
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;  // identity reflector
    double beta = -std::copysign(std::hypot(alpha, xn), alpha);
    double tau = (beta - alpha) / beta;
    double scal = 1.0 / (alpha - beta);
    v[k] = 1.0;
    for (int i = k + 1; i < m; ++i) v[i] = x[i] * scal;
    x[k] = beta;
    for (int i = k + 1; i < m; ++i) x[i] = 0.0;
    for (int j = k + 1; j < n; ++j) {
      double *y = &A[(size_t)j * m];
      double s = 0;
      for (int i = k; i < m; ++i) s += v[i] * y[i];
      s *= tau;
      for (int i = k; i < m; ++i) y[i] -= s * v[i];
    }
  }
  // R = upper part; keep leading rows with |R_kk| > tol |R_00|
  const double r00 = std::fabs(A[0]);
  int mk = 0;
  while (mk < kmax && std::fabs(A[(size_t)mk * m + mk]) > drop_tol * r00) ++mk;
  c.m = mk;
  c.dropped = m - mk;
  // Tp = [U^-1, -U^-1 V] (mk x n) in pivoted column order, by back substitution
  // of U X = [I, -V]
  std::vector<double> X((size_t)mk * n, 0.0);  // row-major mk x n
  for (int col = 0; col < n; ++col) {
    // rhs column
    for (int i = mk - 1; i >= 0; --i) {
      double r = (col < mk) ? (col == i ? 1.0 : 0.0) : -A[(size_t)col * m + i];
      for (int t = i + 1; t < mk; ++t) r -= A[(size_t)t * m + i] * X[(size_t)t * n + col];
      X[(size_t)i * n + col] = r / A[(size_t)i * m + i];
    }
  }
  c.trow.assign((size_t)mk * n, 0.0);
  c.hrow.assign((size_t)mk * n, 0.0);
  for (int k = 0; k < mk; ++k)
    for (int b = 0; b < n; ++b) {
      c.trow[(size_t)k * n + c.perm[b]] = X[(size_t)k * n + b];
      c.hrow[(size_t)k * n + c.perm[b]] = (b >= k) ? A[(size_t)b * m + k] : 0.0;
    }
  return c;
}

void build_constraints(Problem &P) {
  const int dpn = P.mesh.dpn;
  P.cov.assign(P.globs.size(), GlobCov());
  if (P.extra_rows.size() != P.globs.size()) {
    P.extra_rows.assign(P.globs.size(), {});
    P.extra_k.assign(P.globs.size(), 0);
  }
  // globs are independent: one QR-CP each, on the host threads
  parallel_for((int)P.globs.size(), [&](int gi) {
    const Glob &g = P.globs[gi];
    const int n = (int)g.dofs.size();
    std::vector<double> H;
    int m = 0;
    if (P.mode == 3) {
      H.assign((size_t)n * n, 0.0);
      for (int t = 0; t < n; ++t) H[(size_t)t * n + t] = 1.0;
      m = n;
    } else if ((g.kind == GLOB_EDGE && P.mode >= 1) || (g.kind == GLOB_FACE && P.mode >= 2)) {
      // one unit-weight average per displacement component
      for (int c = 0; c < dpn; ++c) {
        bool any = false;
        for (int t = 0; t < n; ++t) any |= g.comp[t] == c;
        if (!any) continue;
        size_t off = H.size();
        H.resize(off + n, 0.0);
        for (int t = 0; t < n; ++t)
          if (g.comp[t] == c) H[off + t] = 1.0;
        ++m;
      }
    }
    if (P.extra_k[gi] > 0) {
      H.insert(H.end(), P.extra_rows[gi].begin(), P.extra_rows[gi].end());
      m += P.extra_k[gi];
    }
    P.cov[gi] = qr_change_of_variables(H, m, n, P.drop_tol);
  });
}

int64_t count_nc(const Problem &P) {
  int64_t nc = 0;
  for (size_t gi = 0; gi < P.globs.size(); ++gi)
    nc += (int64_t)P.cov[gi].m * ((int64_t)P.globs[gi].subs.size() - 1);
  return nc;
}

}  // namespace bddc
