// Adaptive face constraints on the device (Sec. 3, Algorithm 1).
//
// For a face shared by substructures i and j the generalized eigenproblem of
// eq. (eig-matrix) is reduced exactly, before any iteration:
//
// * (I - E_ij) w depends only on the jump J = w_i - w_j on the shared
//   non-corner dofs: side i receives delta_j J, side j receives -delta_i J
//   (weights renormalized over {i, j}).  The numerator is J^T M J with
//   M = D_j S_i[s,s] D_j + D_i S_j[s,s] D_i (Schur complements, original
//   basis, shared dofs s), since (I - P) extends these values harmonically
//   with zero on the rest of each interface.
// * The denominator, minimized over everything that does not change J (the
//   interface dofs of either side that are not shared, and the common part
//   w_j), is J^T B_J J with the parallel sum B_J = Sh_i - Sh_i (Sh_i + Sh_j)^+ Sh_i
//   of the Schur complements Sh_a of S_a onto s.  By the minimax principle
//   (Lemma on Courant-Fisher-Weyl) the nonzero eigenvalues and the rows
//   d = w^T C are unchanged.  The pseudo-inverse of Sh_i + Sh_j acts on
//   the range of Sh_i; when both substructures float, its null space is the
//   rigid-body traces R on s and a rank-|R| term rho R R^T makes it regular.
// * Corner dofs have J = 0; the constraints of the globs shared by i and j
//   (D^c_ij) are J-space conditions h.J = 0, so J = Z y with Z the columns of
//   the globs' change of variables T that are not explicit averages.
//
// The pair problem becomes  (Z^T M Z) y = lambda (Z^T B_J Z) y; with
// Z^T B_J Z = L L^T it is the standard problem C' x = lambda x,
// C' = L^-1 Z^T M Z L^-T, whose dominant eigenpairs are found by batched
// LOBPCG (one work-group per face, Rayleigh-Ritz in LDS by Jacobi rotations).
// The rows are d = Pi_G M J with J = Z L^-T x; the face part of d, projected
// onto the null space of the face's own existing constraints, is the new
// constraint row (edge parts are dropped, Remark after Proposition 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "adapt.h"
#include "dense.h"

namespace bddc {

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));             \
  } while (0)

namespace {

constexpr int TPB = 256;
constexpr int LOB_MAXB = 48;  // basis columns in the Rayleigh-Ritz step (3 x block)

inline unsigned nblocks(int64_t n, int tpb = TPB) {
  return (unsigned)std::max<int64_t>(1, (n + tpb - 1) / tpb);
}

// dst[e] (rows x cols, ld = rows) = src_sub[ridx, cidx] of the source matrix
__global__ void gather_rc_kernel(const double *src, const int64_t *src_off, const int *lds,
                                 double *dst, const int64_t *dst_off, const int *ridx,
                                 const int64_t *ridx_off, const int *nrow, const int *cidx,
                                 const int64_t *cidx_off, const int *ncol) {
  const int e = blockIdx.y;
  const int64_t nr = nrow[e], nc = ncol[e];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr * nc) return;
  const int a = (int)(i % nr), b = (int)(i / nr);
  const int ra = ridx[ridx_off[e] + a], cb = cidx[cidx_off[e] + b];
  dst[dst_off[e] + i] = src[src_off[e] + ra + (int64_t)cb * lds[e]];
}

// Ssum = Sh_i + Sh_j + rho Q Q^T ; Xb = Sh_i  (per pair, n x n, ld n)
__global__ void pair_sum_kernel(const double *Sh, const int64_t *off_i, const int64_t *off_j,
                                const int *ns, double *Ssum, double *Xb, double *BJ,
                                const int64_t *off_p, const double *Q, const int64_t *q_off,
                                const int *nq, const double *rho) {
  const int e = blockIdx.y;
  const int64_t n = ns[e];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * n) return;
  const int r = (int)(i % n), c = (int)(i / n);
  const double si = Sh[off_i[e] + i];
  double v = si + Sh[off_j[e] + i];
  for (int k = 0; k < nq[e]; ++k) v += rho[e] * Q[q_off[e] + r + k * n] * Q[q_off[e] + c + k * n];
  Ssum[off_p[e] + i] = v;
  Xb[off_p[e] + i] = si;
  BJ[off_p[e] + i] = si;
}

// compact c x c blocks: M = Dj Si Dj + Di Sj Di, BJ = (Sh_i - Sh_i X)[c,c]
__global__ void pair_restrict_kernel(const double *Sss, const int64_t *off_si,
                                     const int64_t *off_sj, const double *BJfull,
                                     const int64_t *off_p, const int *ns, const int *cidx,
                                     const int64_t *c_off, const int *nc, const double *wi,
                                     double *M, double *BJ, const int64_t *off_c) {
  const int e = blockIdx.y;
  const int64_t m = nc[e], n = ns[e];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * m) return;
  const int a = (int)(i % m), b = (int)(i / m);
  const int ra = cidx[c_off[e] + a], rb = cidx[c_off[e] + b];
  const double dia = wi[c_off[e] + a], dib = wi[c_off[e] + b];
  const double dja = 1.0 - dia, djb = 1.0 - dib;
  const int64_t src = ra + (int64_t)rb * n;
  M[off_c[e] + i] = dja * Sss[off_si[e] + src] * djb + dia * Sss[off_sj[e] + src] * dib;
  BJ[off_c[e] + i] = BJfull[off_p[e] + src];
}

__global__ void transpose_kernel(const double *src, double *dst, const int64_t *off,
                                 const int *n) {
  const int e = blockIdx.y;
  const int64_t m = n[e];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * m) return;
  const int r = (int)(i % m), c = (int)(i / m);
  dst[off[e] + c + (int64_t)r * m] = src[off[e] + i];
}

// ---------------------------------------------------------------------------
// batched LOBPCG: dominant eigenpairs of a symmetric d x d matrix per entry

struct LobDesc {
  int64_t a_off;    // d x d matrix (ld d)
  int64_t v_off;    // 6 blocks of d x s: X, AX, W, AW, P, AP (ld d)
  int64_t t_off;    // 2 blocks of d x s scratch
  int d, s;
  int need;         // number of leading eigenpairs that must converge (>= 1)
  double tau;       // threshold: pairs with theta >= tau are needed, plus one below
};

struct LobOut {
  int iters;
  int converged;
  int nconv;
};

// y = sum_k x[k] over the work-group
__device__ double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// Symmetric eigen-decomposition of the n x n matrix H (LDS, ld LOB_MAXB+1) by
// parallel cyclic Jacobi (round-robin pairing): H <- diag, V <- eigenvectors.
__device__ void jacobi_eig(double (*H)[LOB_MAXB + 1], double (*V)[LOB_MAXB + 1], int n,
                           int *perm, double *cs, double *sn, double *red) {
  const int tid = threadIdx.x;
  for (int i = tid; i < n * n; i += blockDim.x) V[i % n][i / n] = (i % n == i / n) ? 1.0 : 0.0;
  const int m = (n + 1) / 2 * 2;  // even number of players (a dummy when n is odd)
  for (int i = tid; i < m; i += blockDim.x) perm[i] = i;
  __syncthreads();
  for (int sweep = 0; sweep < 20; ++sweep) {
    double off = 0, tot = 0;
    for (int i = tid; i < n * n; i += blockDim.x) {
      const double h = H[i % n][i / n];
      tot += h * h;
      if (i % n != i / n) off += h * h;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (off <= 1e-30 * tot || tot == 0) break;
    for (int step = 0; step < m - 1; ++step) {
      // pairs (perm[k], perm[m-1-k]), k < m/2
      for (int k = tid; k < m / 2; k += blockDim.x) {
        int p = perm[k], q = perm[m - 1 - k];
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        double c = 1, s = 0;
        if (q < n && H[p][q] != 0.0) {
          const double theta = (H[q][q] - H[p][p]) / (2 * H[p][q]);
          const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1));
          c = 1 / sqrt(t * t + 1);
          s = t * c;
        }
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // rows: H <- J^T H
      for (int i = tid; i < (m / 2) * n; i += blockDim.x) {
        const int k = i % (m / 2), col = i / (m / 2);
        int p = perm[k], q = perm[m - 1 - k];
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        if (q >= n) continue;
        const double c = cs[k], s = sn[k];
        const double hp = H[p][col], hq = H[q][col];
        H[p][col] = c * hp - s * hq;
        H[q][col] = s * hp + c * hq;
      }
      __syncthreads();
      // columns: H <- H J, V <- V J
      for (int i = tid; i < (m / 2) * n; i += blockDim.x) {
        const int k = i % (m / 2), row = i / (m / 2);
        int p = perm[k], q = perm[m - 1 - k];
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        if (q >= n) continue;
        const double c = cs[k], s = sn[k];
        const double hp = H[row][p], hq = H[row][q];
        H[row][p] = c * hp - s * hq;
        H[row][q] = s * hp + c * hq;
        const double vp = V[row][p], vq = V[row][q];
        V[row][p] = c * vp - s * vq;
        V[row][q] = s * vp + c * vq;
      }
      __syncthreads();
      // rotate the round-robin schedule (player 0 fixed)
      if (tid == 0) {
        const int last = perm[m - 1];
        for (int k = m - 1; k > 1; --k) perm[k] = perm[k - 1];
        perm[1] = last;
      }
      __syncthreads();
    }
  }
}

// One work-group per entry.  Basis blocks live in global memory; Gram and
// projected matrices (at most 48 x 48) in LDS.
__global__ __launch_bounds__(256) void lobpcg_kernel(double *pool, const LobDesc *desc,
                                                     LobOut *out, int maxit, double tol,
                                                     double tol_ind) {
  __shared__ double G[LOB_MAXB][LOB_MAXB + 1];
  __shared__ double H[LOB_MAXB][LOB_MAXB + 1];
  __shared__ double Q[LOB_MAXB][LOB_MAXB + 1];
  __shared__ double Y[LOB_MAXB][LOB_MAXB + 1];
  __shared__ double theta[LOB_MAXB], gsc[LOB_MAXB], res[LOB_MAXB];
  __shared__ double cs[LOB_MAXB], sn[LOB_MAXB], red[8];
  __shared__ int perm[LOB_MAXB + 2];
  __shared__ int s_nb, s_keep, s_done;
  const LobDesc D = desc[blockIdx.x];
  const int d = D.d, s = D.s, tid = threadIdx.x;
  const double *A = pool + D.a_off;
  double *X = pool + D.v_off, *AX = X + (int64_t)d * s, *W = AX + (int64_t)d * s;
  double *AW = W + (int64_t)d * s, *P = AW + (int64_t)d * s, *AP = P + (int64_t)d * s;
  double *T1 = pool + D.t_off, *T2 = T1 + (int64_t)d * s;
  // blocks of the basis: 0 = X, 1 = W, 2 = P
  auto blk = [&](int b) -> double * { return b == 0 ? X : (b == 1 ? W : P); };
  auto ablk = [&](int b) -> double * { return b == 0 ? AX : (b == 1 ? AW : AP); };
  // AX = A X (X holds the initial block)
  auto matblock = [&](const double *in, double *o) {
    for (int i = tid; i < d * s; i += blockDim.x) {
      const int r = i % d, q = i / d;
      double acc = 0;
      for (int c = 0; c < d; ++c) acc += A[r + (int64_t)c * d] * in[c + (int64_t)q * d];
      o[i] = acc;
    }
  };
  int it = 0, nconv = 0, have_p = 0;
  bool done = false;
  // Rayleigh-Ritz on [X] first to get theta and an orthonormal X
  for (it = 0; it <= maxit; ++it) {
    const int nb = (it == 0) ? 1 : (have_p ? 3 : 2);
    if (it == 0) {
      matblock(X, AX);
      __syncthreads();
    } else {
      // W = AX - X theta (residuals), norms
      for (int i = tid; i < d * s; i += blockDim.x) {
        const int q = i / d;
        W[i] = AX[i] - X[i] * theta[q];
      }
      __syncthreads();
      for (int q = 0; q < s; ++q) {
        double acc = 0;
        for (int r = tid; r < d; r += blockDim.x) acc += W[r + (int64_t)q * d] * W[r + (int64_t)q * d];
        acc = block_sum(acc, red);
        if (tid == 0) res[q] = sqrt(acc);
      }
      __syncthreads();
      // convergence of the leading pairs that matter: those >= tau and the
      // first one below (or the 'need' leading ones)
      // the pairs with theta >= tau must converge to tol; the first one
      // below tau only sets the indicator and converges to tol_ind
      if (tid == 0) {
        int k = 0, ok = 1;
        for (k = 0; k < s; ++k) {
          const bool selected = theta[k] >= D.tau;
          const bool needed = (k < D.need) || (k == 0) || (theta[k - 1] >= D.tau);
          if (!needed) break;
          const double t = selected ? tol : tol_ind;
          if (res[k] > t * fmax(fabs(theta[k]), 1.0)) ok = 0;
        }
        nconv = k;
        s_done = ok;
      }
      __syncthreads();
      if (s_done || it == maxit) {
        done = s_done;
        break;
      }
      // unit columns in W and P keep the Gram matrix free of scale disparity
      // as the residuals shrink (otherwise the g^-1/2 basis loses accuracy)
      for (int q = 0; q < s; ++q) {
        double pn = 0;
        if (have_p)
          for (int r = tid; r < d; r += blockDim.x) pn += P[r + (int64_t)q * d] * P[r + (int64_t)q * d];
        pn = block_sum(pn, red);
        if (tid == 0) gsc[q] = (have_p && pn > 0) ? 1.0 / sqrt(pn) : 1.0;
      }
      __syncthreads();
      for (int i = tid; i < d * s; i += blockDim.x) {
        const int q = i / d;
        if (res[q] > 0) W[i] /= res[q];
        if (have_p) {
          P[i] *= gsc[q];
          AP[i] *= gsc[q];
        }
      }
      __syncthreads();
      matblock(W, AW);
      __syncthreads();
    }
    // Gram G = V^T V and H = V^T A V over the nb blocks
    const int n = nb * s;
    for (int i = tid; i < n * n; i += blockDim.x) {
      const int a = i % n, b = i / n;
      if (a > b) continue;
      const double *va = blk(a / s) + (int64_t)(a % s) * d;
      const double *vb = blk(b / s) + (int64_t)(b % s) * d;
      const double *ab = ablk(b / s) + (int64_t)(b % s) * d;
      double g = 0, h = 0;
      for (int r = 0; r < d; ++r) {
        g += va[r] * vb[r];
        h += va[r] * ab[r];
      }
      G[a][b] = G[b][a] = g;
      H[a][b] = h;
      H[b][a] = h;
    }
    __syncthreads();
    // symmetrize H (A V computed in rounding, V^T A V slightly asymmetric)
    for (int i = tid; i < n * n; i += blockDim.x) {
      const int a = i % n, b = i / n;
      if (a < b) {
        const double m = 0.5 * (H[a][b] + H[b][a]);
        H[a][b] = H[b][a] = m;
      }
    }
    __syncthreads();
    // G = Q diag(g) Q^T; keep g > 1e-13 g_max; Hh = g^-1/2 Q^T H Q g^-1/2
    // (Q's columns in Q, eigenvalues on the diagonal of G afterwards)
    jacobi_eig(G, Q, n, perm, cs, sn, red);
    if (tid == 0) {
      double gmax = 0;
      for (int a = 0; a < n; ++a) gmax = fmax(gmax, G[a][a]);
      int keep = 0;
      for (int a = 0; a < n; ++a) {
        if (G[a][a] > 1e-13 * gmax) {
          perm[keep] = a;
          gsc[keep] = 1.0 / sqrt(G[a][a]);
          ++keep;
        }
      }
      s_keep = keep;
    }
    __syncthreads();
    const int kp = s_keep;
    // Y <- H Q_keep g^-1/2   (n x kp)
    for (int i = tid; i < n * kp; i += blockDim.x) {
      const int a = i % n, b = i / n;
      double acc = 0;
      for (int c = 0; c < n; ++c) acc += H[a][c] * Q[c][perm[b]];
      Y[a][b] = acc * gsc[b];
    }
    __syncthreads();
    // G <- g^-1/2 Q_keep^T Y  (kp x kp), reusing G as the projected matrix
    for (int i = tid; i < kp * kp; i += blockDim.x) {
      const int a = i % kp, b = i / kp;
      double acc = 0;
      for (int c = 0; c < n; ++c) acc += Q[c][perm[a]] * Y[c][b];
      G[a][b] = acc * gsc[a];
    }
    __syncthreads();
    // keep the map from projected coordinates back to V: Mv = Q_keep g^-1/2
    // (n x kp) stored in H (H is free now)
    for (int i = tid; i < n * kp; i += blockDim.x) {
      const int a = i % n, b = i / n;
      H[a][b] = Q[a][perm[b]] * gsc[b];
    }
    __syncthreads();
    // symmetrize, eigen-decompose the projected matrix (eigenvectors in Q)
    for (int i = tid; i < kp * kp; i += blockDim.x) {
      const int a = i % kp, b = i / kp;
      if (a < b) {
        const double m = 0.5 * (G[a][b] + G[b][a]);
        G[a][b] = G[b][a] = m;
      }
    }
    __syncthreads();
    jacobi_eig(G, Q, kp, perm, cs, sn, red);
    // order eigenvalues descending: perm holds the ordering
    if (tid == 0) {
      for (int a = 0; a < kp; ++a) perm[a] = a;
      for (int a = 0; a < kp; ++a)
        for (int b = a + 1; b < kp; ++b)
          if (G[perm[b]][perm[b]] > G[perm[a]][perm[a]]) {
            int t = perm[a];
            perm[a] = perm[b];
            perm[b] = t;
          }
      for (int q = 0; q < s; ++q) theta[q] = (q < kp) ? G[perm[q]][perm[q]] : 0.0;
      s_nb = nb;
    }
    __syncthreads();
    // coefficients of the new X in V: C = Mv Q[:, top s]  (n x s), in Y
    for (int i = tid; i < n * s; i += blockDim.x) {
      const int a = i % n, q = i / n;
      double acc = 0;
      if (q < kp)
        for (int c = 0; c < kp; ++c) acc += H[a][c] * Q[c][perm[q]];
      Y[a][q] = acc;
    }
    __syncthreads();
    // new X = V C and its A-image into the scratch blocks T1, T2
    for (int i = tid; i < d * s; i += blockDim.x) {
      const int r = i % d, q = i / d;
      double x = 0, ax = 0;
      for (int b = 0; b < n; ++b) {
        const double c = Y[b][q];
        const int bb = b / s, col = b % s;
        x += c * blk(bb)[r + (int64_t)col * d];
        ax += c * ablk(bb)[r + (int64_t)col * d];
      }
      T1[i] = x;
      T2[i] = ax;
    }
    __syncthreads();
    if (nb > 1) {
      // new P = the W and P part of V C; written into the X / AX slots first
      // (the old X is not read by this pass, the old W and P still are)
      for (int i = tid; i < d * s; i += blockDim.x) {
        const int r = i % d, q = i / d;
        double p = 0, ap = 0;
        for (int b = s; b < n; ++b) {
          const double c = Y[b][q];
          const int bb = b / s, col = b % s;
          p += c * blk(bb)[r + (int64_t)col * d];
          ap += c * ablk(bb)[r + (int64_t)col * d];
        }
        X[i] = p;
        AX[i] = ap;
      }
      __syncthreads();
      for (int i = tid; i < d * s; i += blockDim.x) {
        P[i] = X[i];
        AP[i] = AX[i];
      }
      have_p = 1;
      __syncthreads();
    }
    for (int i = tid; i < d * s; i += blockDim.x) {
      X[i] = T1[i];
      AX[i] = T2[i];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[blockIdx.x].iters = it;
    out[blockIdx.x].converged = done ? 1 : 0;
    out[blockIdx.x].nconv = nconv;
  }
  // eigenvalues into the first column of T1 for the host
  __syncthreads();
  for (int q = tid; q < s; q += blockDim.x) T1[q] = theta[q];
}

}  // namespace

// ---------------------------------------------------------------------------
// host orchestration

namespace {

struct PairHost {
  int f, gi, sub[2];
  std::vector<int> pos_s[2], pos_n[2];
  std::vector<int> cidx;     // indices into the shared list of the non-corner dofs
  std::vector<double> wi;    // renormalized weight of side i on every c dof
  std::vector<double> Q;     // rigid traces on s (n_s x nq, orthonormal columns)
  int nq = 0;
  double rho = 0;
  std::vector<double> Z;     // n_c x d, column-major
  int d = 0;
  std::vector<int> face_c;   // c-indices of the face glob dofs (glob order)
};

struct Pool {
  DevAlloc *A;
  std::vector<DBuf> bufs;
  template <class T>
  T *up(hipStream_t st, const std::vector<T> &v) {
    DBuf b;
    b.bytes = std::max<size_t>(v.size() * sizeof(T), 8);
    b.p = A->get(b.bytes);
    if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    bufs.push_back(b);
    return b.as<T>();
  }
  double *zeros(hipStream_t st, int64_t n) {
    DBuf b;
    b.bytes = std::max<size_t>(n * sizeof(double), 8);
    b.p = A->get(b.bytes);
    HIPCHK(hipMemsetAsync(b.p, 0, b.bytes, st));
    bufs.push_back(b);
    return b.as<double>();
  }
  ~Pool() {
    for (auto &b : bufs) A->put(b.p, b.bytes);
  }
};

void orthonormalize(std::vector<double> &Q, int n, int &k) {
  int out = 0;
  for (int c = 0; c < k; ++c) {
    double *v = &Q[(size_t)c * n];
    for (int pass = 0; pass < 2; ++pass)
      for (int p = 0; p < out; ++p) {
        const double *u = &Q[(size_t)p * n];
        double dt = 0;
        for (int r = 0; r < n; ++r) dt += u[r] * v[r];
        for (int r = 0; r < n; ++r) v[r] -= dt * u[r];
      }
    double nr = 0;
    for (int r = 0; r < n; ++r) nr += v[r] * v[r];
    nr = std::sqrt(nr);
    if (nr < 1e-10) continue;
    double *o = &Q[(size_t)out * n];
    for (int r = 0; r < n; ++r) o[r] = v[r] / nr;
    ++out;
  }
  k = out;
  Q.resize((size_t)out * n);
}

}  // namespace

AdaptResult run_adapt(Problem &P, Solver &S, AdaptState &st, double tau) {
  AdaptResult res;
  hipStream_t stream = S.stream;
  S.factor_schur();  // Schur complements S_i (original basis) in S.d_S
  const Layout &L = S.L;
  const int dpn = P.mesh.dpn;
  const int nf = (int)P.face_ids.size();
  st.eigs.assign(nf, {});
  std::vector<char> is_corner(P.n_glob, 0);
  for (int64_t g : P.corner_gdofs) is_corner[g] = 1;
  std::vector<PairHost> pairs;
  for (int f = 0; f < nf; ++f) {
    PairHost ph;
    ph.f = f;
    ph.gi = P.face_ids[f];
    const Glob &gl = P.globs[ph.gi];
    ph.sub[0] = gl.subs[0];
    ph.sub[1] = gl.subs[1];
    const Sub &Si = P.subs[ph.sub[0]], &Sj = P.subs[ph.sub[1]];
    std::vector<int64_t> gi_(Si.gdof.begin() + Si.nI, Si.gdof.end());
    std::vector<int64_t> gj_(Sj.gdof.begin() + Sj.nI, Sj.gdof.end());
    std::vector<int64_t> sh;
    std::set_intersection(gi_.begin(), gi_.end(), gj_.begin(), gj_.end(), std::back_inserter(sh));
    const int ns_ = (int)sh.size();
    for (int a = 0; a < 2; ++a) {
      const auto &gg = a == 0 ? gi_ : gj_;
      std::vector<char> in(gg.size(), 0);
      for (int64_t g : sh) {
        const int p = (int)(std::lower_bound(gg.begin(), gg.end(), g) - gg.begin());
        ph.pos_s[a].push_back(p);
        in[p] = 1;
      }
      for (int p = 0; p < (int)gg.size(); ++p)
        if (!in[p]) ph.pos_n[a].push_back(p);
    }
    std::vector<int> c_of(ns_, -1);
    for (int k = 0; k < ns_; ++k)
      if (!is_corner[sh[k]]) {
        c_of[k] = (int)ph.cidx.size();
        ph.cidx.push_back(k);
        const double di = Si.diag[Si.nI + ph.pos_s[0][k]], dj = Sj.diag[Sj.nI + ph.pos_s[1][k]];
        ph.wi.push_back(di / (di + dj));
      }
    const int nc = (int)ph.cidx.size();
    if (nc == 0) continue;
    // regularization of the parallel sum when both substructures float
    double rho = 0;
    for (int k = 0; k < ns_; ++k)
      rho = std::max({rho, Si.diag[Si.nI + ph.pos_s[0][k]], Sj.diag[Sj.nI + ph.pos_s[1][k]]});
    ph.rho = rho;
    if (Si.floating && Sj.floating) {
      int nq = dpn == 1 ? 1 : 6;
      ph.Q.assign((size_t)nq * ns_, 0.0);
      double cen[3] = {0, 0, 0};
      for (int k = 0; k < ns_; ++k) {
        const int64_t node = P.glob2full[sh[k]] / dpn;
        for (int c = 0; c < 3; ++c) cen[c] += P.mesh.xyz[3 * node + c] / ns_;
      }
      for (int k = 0; k < ns_; ++k) {
        const int64_t full = P.glob2full[sh[k]];
        const int64_t node = full / dpn;
        const int comp = (int)(full % dpn);
        if (dpn == 1) {
          ph.Q[k] = 1.0;
          continue;
        }
        const double x = P.mesh.xyz[3 * node] - cen[0], y = P.mesh.xyz[3 * node + 1] - cen[1],
                     z = P.mesh.xyz[3 * node + 2] - cen[2];
        ph.Q[(size_t)comp * ns_ + k] = 1.0;
        const double rot[3][3] = {{0, -z, y}, {z, 0, -x}, {-y, x, 0}};
        for (int r = 0; r < 3; ++r) ph.Q[(size_t)(3 + r) * ns_ + k] = rot[r][comp];
      }
      orthonormalize(ph.Q, ns_, nq);
      ph.nq = nq;
    }
    // basis of the J space from the change of variables of the shared globs
    std::vector<std::vector<double>> cols;
    for (size_t g2 = 0; g2 < P.globs.size(); ++g2) {
      const Glob &G = P.globs[g2];
      if (std::find(G.subs.begin(), G.subs.end(), ph.sub[0]) == G.subs.end() ||
          std::find(G.subs.begin(), G.subs.end(), ph.sub[1]) == G.subs.end())
        continue;
      const GlobCov &cv = P.cov[g2];
      std::vector<int> crow(G.dofs.size());
      for (size_t t = 0; t < G.dofs.size(); ++t) {
        const int k = (int)(std::lower_bound(sh.begin(), sh.end(), G.dofs[t]) - sh.begin());
        crow[t] = c_of[k];
      }
      std::vector<char> expl(G.dofs.size(), 0);
      for (int k = 0; k < cv.m; ++k) expl[cv.perm[k]] = 1;
      for (size_t t = 0; t < G.dofs.size(); ++t) {
        if (expl[t]) continue;
        std::vector<double> col(nc, 0.0);
        col[crow[t]] = 1.0;
        for (int k = 0; k < cv.m; ++k) col[crow[cv.perm[k]]] += cv.trow[(size_t)k * cv.n + t];
        cols.push_back(std::move(col));
      }
      if ((int)g2 == ph.gi)
        for (size_t t = 0; t < G.dofs.size(); ++t) ph.face_c.push_back(crow[t]);
    }
    ph.d = (int)cols.size();
    if (ph.d == 0) continue;
    ph.Z.resize((size_t)nc * ph.d);
    for (int c = 0; c < ph.d; ++c)
      std::copy(cols[c].begin(), cols[c].end(), ph.Z.begin() + (size_t)c * nc);
    pairs.push_back(std::move(ph));
  }
  const int np = (int)pairs.size();
  res.n_pairs = np;
  if (np == 0) return res;

  // ---- device stage 1: Schur complements of S_i onto each pair's shared dofs
  Pool pool{&S.alloc};
  const int nside = 2 * np;
  std::vector<int64_t> src_off(nside), off_nn(nside), off_ns(nside), off_sh(nside), off_ss(nside);
  std::vector<int> lds(nside), nn(nside), nsv(nside);
  std::vector<int> idx_s, idx_n;
  std::vector<int64_t> idx_s_off(nside), idx_n_off(nside);
  int64_t tnn = 0, tns = 0, tsh = 0;
  int max_nn = 0, max_ns = 0;
  for (int p = 0; p < np; ++p)
    for (int a = 0; a < 2; ++a) {
      const int e = 2 * p + a, sub = pairs[p].sub[a];
      src_off[e] = L.offGG[sub];
      lds[e] = L.nG[sub];
      nn[e] = (int)pairs[p].pos_n[a].size();
      nsv[e] = (int)pairs[p].pos_s[a].size();
      max_nn = std::max(max_nn, nn[e]);
      max_ns = std::max(max_ns, nsv[e]);
      off_nn[e] = tnn;
      tnn += (int64_t)nn[e] * nn[e];
      off_ns[e] = tns;
      tns += (int64_t)nn[e] * nsv[e];
      off_sh[e] = tsh;
      off_ss[e] = tsh + (int64_t)nsv[e] * nsv[e];
      tsh += 2 * (int64_t)nsv[e] * nsv[e];
      idx_s_off[e] = (int64_t)idx_s.size();
      idx_s.insert(idx_s.end(), pairs[p].pos_s[a].begin(), pairs[p].pos_s[a].end());
      idx_n_off[e] = (int64_t)idx_n.size();
      idx_n.insert(idx_n.end(), pairs[p].pos_n[a].begin(), pairs[p].pos_n[a].end());
    }
  double *Snn = pool.zeros(stream, tnn), *Sns = pool.zeros(stream, tns), *Sh = pool.zeros(stream, tsh);
  int64_t *d_src_off = pool.up(stream, src_off);
  int *d_lds = pool.up(stream, lds), *d_nn = pool.up(stream, nn), *d_ns = pool.up(stream, nsv);
  int *d_idx_s = pool.up(stream, idx_s), *d_idx_n = pool.up(stream, idx_n);
  int64_t *d_idx_s_off = pool.up(stream, idx_s_off), *d_idx_n_off = pool.up(stream, idx_n_off);
  int64_t *d_off_nn = pool.up(stream, off_nn), *d_off_ns = pool.up(stream, off_ns);
  int64_t *d_off_sh = pool.up(stream, off_sh), *d_off_ss = pool.up(stream, off_ss);
  const double *Sd = S.d_S.as<double>();
  auto gather = [&](double *dst, const int64_t *doff, const int *ri, const int64_t *rio, const int *nr,
                    const int *ci, const int64_t *cio, const int *ncl, int64_t maxe) {
    gather_rc_kernel<<<dim3(nblocks(maxe), nside), TPB, 0, stream>>>(Sd, d_src_off, d_lds, dst, doff, ri,
                                                                     rio, nr, ci, cio, ncl);
    HIPCHK(hipGetLastError());
  };
  gather(Snn, d_off_nn, d_idx_n, d_idx_n_off, d_nn, d_idx_n, d_idx_n_off, d_nn, (int64_t)max_nn * max_nn);
  gather(Sns, d_off_ns, d_idx_n, d_idx_n_off, d_nn, d_idx_s, d_idx_s_off, d_ns, (int64_t)max_nn * max_ns);
  gather(Sh, d_off_sh, d_idx_s, d_idx_s_off, d_ns, d_idx_s, d_idx_s_off, d_ns, (int64_t)max_ns * max_ns);
  gather(Sh, d_off_ss, d_idx_s, d_idx_s_off, d_ns, d_idx_s, d_idx_s_off, d_ns, (int64_t)max_ns * max_ns);
  std::vector<MatDesc> mdn(nside);
  std::vector<GemmDesc> gsh(nside);
  for (int e = 0; e < nside; ++e) {
    mdn[e] = MatDesc{off_nn[e], off_ns[e], nn[e], nsv[e], std::max(1, nn[e]), std::max(1, nn[e])};
    gsh[e] = GemmDesc{off_ns[e], off_ns[e], off_sh[e], nsv[e], nsv[e], nn[e], std::max(1, nn[e]),
                      std::max(1, nn[e]), std::max(1, nsv[e])};
  }
  MatDesc *d_mdn = pool.up(stream, mdn);
  GemmDesc *d_gsh = pool.up(stream, gsh);
  int *d_stat = pool.up(stream, std::vector<int>(3 * np + 2 * nside + 4, 0));
  HIPCHK(DenseOps<double>::potrf(stream, Snn, d_mdn, mdn.data(), nside, d_stat));
  HIPCHK(DenseOps<double>::trsm(stream, Snn, Sns, d_mdn, mdn.data(), nside, false));
  // Sh gets the Schur complement; Sns and Sh live in different pools
  HIPCHK(DenseOps<double>::gemm(stream, Sns, Sns, Sh, d_gsh, nside, max_ns, max_ns, true, false,
                                -1.0, 1.0, false));

  // ---- stage 2: parallel sum and the reduced pair matrices
  std::vector<int64_t> off_i(np), off_j(np), off_p(np), q_off(np), off_c(np), c_off(np), off_z(np),
      off_cz(np), off_dd(np);
  std::vector<int> nsp(np), nqv(np), ncv(np), dv(np);
  std::vector<double> rho(np), Qall, wall, Zall;
  std::vector<int> call;
  int64_t tp = 0, tc = 0, tz = 0, tdd = 0, tcz = 0;
  int max_c = 0, max_d = 0;
  for (int p = 0; p < np; ++p) {
    const PairHost &ph = pairs[p];
    off_i[p] = off_sh[2 * p];
    off_j[p] = off_sh[2 * p + 1];
    nsp[p] = nsv[2 * p];
    off_p[p] = tp;
    tp += (int64_t)nsp[p] * nsp[p];
    q_off[p] = (int64_t)Qall.size();
    Qall.insert(Qall.end(), ph.Q.begin(), ph.Q.end());
    nqv[p] = ph.nq;
    rho[p] = ph.rho;
    ncv[p] = (int)ph.cidx.size();
    dv[p] = ph.d;
    c_off[p] = (int64_t)call.size();
    call.insert(call.end(), ph.cidx.begin(), ph.cidx.end());
    wall.insert(wall.end(), ph.wi.begin(), ph.wi.end());
    off_c[p] = tc;
    tc += (int64_t)ncv[p] * ncv[p];
    off_z[p] = (int64_t)Zall.size();
    Zall.insert(Zall.end(), ph.Z.begin(), ph.Z.end());
    off_cz[p] = tcz;
    tcz += (int64_t)ncv[p] * dv[p];
    off_dd[p] = tdd;
    tdd += (int64_t)dv[p] * dv[p];
    max_c = std::max(max_c, ncv[p]);
    max_d = std::max(max_d, dv[p]);
  }
  std::vector<int64_t> off_ss_i(np), off_ss_j(np);
  for (int p = 0; p < np; ++p) off_ss_i[p] = off_ss[2 * p], off_ss_j[p] = off_ss[2 * p + 1];
  double *Ssum = pool.zeros(stream, tp), *Xb = pool.zeros(stream, tp), *BJf = pool.zeros(stream, tp);
  double *d_Q = pool.up(stream, Qall), *d_rho = pool.up(stream, rho);
  int64_t *d_off_i = pool.up(stream, off_i), *d_off_j = pool.up(stream, off_j),
          *d_off_p = pool.up(stream, off_p), *d_q_off = pool.up(stream, q_off);
  int *d_nsp = pool.up(stream, nsp), *d_nq = pool.up(stream, nqv);
  int max_sp = 0;
  for (int p = 0; p < np; ++p) max_sp = std::max(max_sp, nsp[p]);
  pair_sum_kernel<<<dim3(nblocks((int64_t)max_sp * max_sp), np), TPB, 0, stream>>>(
      Sh, d_off_i, d_off_j, d_nsp, Ssum, Xb, BJf, d_off_p, d_Q, d_q_off, d_nq, d_rho);
  HIPCHK(hipGetLastError());
  std::vector<MatDesc> mds(np);
  std::vector<GemmDesc> gbj(np);
  for (int p = 0; p < np; ++p) {
    mds[p] = MatDesc{off_p[p], off_p[p], nsp[p], nsp[p], std::max(1, nsp[p]), std::max(1, nsp[p])};
    gbj[p] = GemmDesc{off_i[p], off_p[p], off_p[p], nsp[p], nsp[p], nsp[p], std::max(1, nsp[p]),
                      std::max(1, nsp[p]), std::max(1, nsp[p])};
  }
  MatDesc *d_mds = pool.up(stream, mds);
  GemmDesc *d_gbj = pool.up(stream, gbj);
  int *stat2 = d_stat + nside;
  HIPCHK(DenseOps<double>::potrf(stream, Ssum, d_mds, mds.data(), np, stat2));
  HIPCHK(DenseOps<double>::trsm(stream, Ssum, Xb, d_mds, mds.data(), np, false));
  HIPCHK(DenseOps<double>::trsm(stream, Ssum, Xb, d_mds, mds.data(), np, true));
  // BJ = Sh_i - Sh_i X   (A = Sh pool, B = Xb pool, C = BJf pool)
  {
    // the gemm wrapper takes one pool per operand
    HIPCHK(DenseOps<double>::gemm(stream, Sh, Xb, BJf, d_gbj, np, max_sp, max_sp, false, false,
                                  -1.0, 1.0, false));
  }
  double *Mc = pool.zeros(stream, tc), *BJc = pool.zeros(stream, tc);
  int *d_call = pool.up(stream, call), *d_nc = pool.up(stream, ncv);
  int64_t *d_c_off = pool.up(stream, c_off), *d_off_c = pool.up(stream, off_c);
  int64_t *d_off_ss_i = pool.up(stream, off_ss_i), *d_off_ss_j = pool.up(stream, off_ss_j);
  double *d_w = pool.up(stream, wall);
  pair_restrict_kernel<<<dim3(nblocks((int64_t)max_c * max_c), np), TPB, 0, stream>>>(
      Sh, d_off_ss_i, d_off_ss_j, BJf, d_off_p, d_nsp, d_call, d_c_off, d_nc, d_w, Mc, BJc, d_off_c);
  HIPCHK(hipGetLastError());
  // My = Z^T M Z, By = Z^T BJ Z
  double *Zd = pool.up(stream, Zall), *T1 = pool.zeros(stream, tcz), *My = pool.zeros(stream, tdd),
         *By = pool.zeros(stream, tdd), *Cp = pool.zeros(stream, tdd);
  std::vector<GemmDesc> g1(np), g2(np);
  for (int p = 0; p < np; ++p) {
    g1[p] = GemmDesc{off_c[p], off_z[p], off_cz[p], ncv[p], dv[p], ncv[p], std::max(1, ncv[p]),
                     std::max(1, ncv[p]), std::max(1, ncv[p])};
    g2[p] = GemmDesc{off_z[p], off_cz[p], off_dd[p], dv[p], dv[p], ncv[p], std::max(1, ncv[p]),
                     std::max(1, ncv[p]), std::max(1, dv[p])};
  }
  GemmDesc *d_g1 = pool.up(stream, g1), *d_g2 = pool.up(stream, g2);
  HIPCHK(DenseOps<double>::gemm(stream, Mc, Zd, T1, d_g1, np, max_c, max_d, false, false, 1.0, 0.0, false));
  HIPCHK(DenseOps<double>::gemm(stream, Zd, T1, My, d_g2, np, max_d, max_d, true, false, 1.0, 0.0, false));
  HIPCHK(DenseOps<double>::gemm(stream, BJc, Zd, T1, d_g1, np, max_c, max_d, false, false, 1.0, 0.0, false));
  HIPCHK(DenseOps<double>::gemm(stream, Zd, T1, By, d_g2, np, max_d, max_d, true, false, 1.0, 0.0, false));
  // C' = L^-1 My L^-T with By = L L^T
  std::vector<MatDesc> mdd(np);
  for (int p = 0; p < np; ++p)
    mdd[p] = MatDesc{off_dd[p], off_dd[p], dv[p], dv[p], std::max(1, dv[p]), std::max(1, dv[p])};
  MatDesc *d_mdd = pool.up(stream, mdd);
  int64_t *d_off_dd = pool.up(stream, off_dd);
  int *d_dv = pool.up(stream, dv);
  int *stat3 = stat2 + np;
  HIPCHK(DenseOps<double>::potrf(stream, By, d_mdd, mdd.data(), np, stat3));
  // My <- L^-1 My ; Cp <- My^T ; Cp <- L^-1 Cp   (My's pool is the B operand)
  HIPCHK(DenseOps<double>::trsm(stream, By, My, d_mdd, mdd.data(), np, false));
  transpose_kernel<<<dim3(nblocks((int64_t)max_d * max_d), np), TPB, 0, stream>>>(My, Cp, d_off_dd, d_dv);
  HIPCHK(hipGetLastError());
  HIPCHK(DenseOps<double>::trsm(stream, By, Cp, d_mdd, mdd.data(), np, false));

  // ---- stage 3: batched LOBPCG on C', with spectral deflation when a block
  // holds only eigenvalues >= tau (C' <- C' - X Theta X^T, run again)
  const int s_max = LOB_MAXB / 3;
  std::vector<LobDesc> ld(np);
  int64_t tv = 0, ty = 0;
  std::vector<int64_t> xoff(np), off_y(np);
  for (int p = 0; p < np; ++p) {
    const int s = std::min(dv[p], s_max);
    ld[p].a_off = off_dd[p];
    ld[p].d = dv[p];
    ld[p].s = s;
    ld[p].need = 1;
    ld[p].tau = tau;
    xoff[p] = tv;
    tv += (int64_t)8 * dv[p] * s;
    off_y[p] = ty;
    ty += (int64_t)dv[p] * dv[p];  // room for every eigenvector of the pair
  }
  double *LP = pool.zeros(stream, tdd + tv);
  HIPCHK(hipMemcpyAsync(LP, Cp, sizeof(double) * tdd, hipMemcpyDeviceToDevice, stream));
  double *Yv = pool.zeros(stream, ty);
  for (int p = 0; p < np; ++p) {
    ld[p].v_off = tdd + xoff[p];
    ld[p].t_off = tdd + xoff[p] + (int64_t)6 * dv[p] * ld[p].s;
  }
  DBuf outb;
  outb.bytes = sizeof(LobOut) * np;
  outb.p = S.alloc.get(outb.bytes);
  pool.bufs.push_back(outb);
  DBuf ldb;
  ldb.bytes = sizeof(LobDesc) * np;
  ldb.p = S.alloc.get(ldb.bytes);
  pool.bufs.push_back(ldb);
  const int maxit = 2000;
  const double tol = 1e-8, tol_ind = 1e-5;
  std::vector<int> ksel(np, 0), active(np);
  std::vector<std::vector<double>> evs(np);
  std::iota(active.begin(), active.end(), 0);
  for (int round = 0; round < 64 && !active.empty(); ++round) {
    const int na = (int)active.size();
    std::vector<LobDesc> lda(na);
    std::vector<double> X0all;
    for (int a = 0; a < na; ++a) {
      const int p = active[a];
      ld[p].s = std::min(dv[p] - ksel[p], s_max);
      lda[a] = ld[p];
      // seeded start block (splitmix64 of face, round, column, row)
      std::vector<double> x0((size_t)dv[p] * ld[p].s);
      for (int q = 0; q < ld[p].s; ++q)
        for (int r = 0; r < dv[p]; ++r) {
          uint64_t z = 0x9E3779B97F4A7C15ull *
                       (uint64_t)((((int64_t)pairs[p].f * 64 + round) * 131071 + q) * 1000003 + r + 1);
          z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
          z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
          z ^= z >> 31;
          x0[(size_t)q * dv[p] + r] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
        }
      HIPCHK(hipMemcpyAsync(LP + ld[p].v_off, x0.data(), sizeof(double) * x0.size(),
                            hipMemcpyHostToDevice, stream));
      X0all.swap(x0);
      HIPCHK(hipStreamSynchronize(stream));
    }
    HIPCHK(hipMemcpyAsync(ldb.p, lda.data(), sizeof(LobDesc) * na, hipMemcpyHostToDevice, stream));
    lobpcg_kernel<<<na, 256, 0, stream>>>(LP, ldb.as<LobDesc>(), outb.as<LobOut>(), maxit, tol,
                                          tol_ind);
    HIPCHK(hipGetLastError());
    std::vector<LobOut> lo(na);
    HIPCHK(hipMemcpyAsync(lo.data(), outb.p, sizeof(LobOut) * na, hipMemcpyDeviceToHost, stream));
    std::vector<std::vector<double>> th(na);
    for (int a = 0; a < na; ++a) {
      const int p = active[a];
      th[a].resize(ld[p].s);
      HIPCHK(hipMemcpyAsync(th[a].data(), LP + ld[p].t_off, sizeof(double) * ld[p].s,
                            hipMemcpyDeviceToHost, stream));
    }
    HIPCHK(hipStreamSynchronize(stream));
    std::vector<int> next;
    std::vector<GemmDesc> gdef;
    for (int a = 0; a < na; ++a) {
      const int p = active[a];
      const int s = ld[p].s;
      res.iters += lo[a].iters;
      if (!lo[a].converged) res.unconverged++;
      int k = 0;
      while (k < s && th[a][k] >= tau) ++k;
      evs[p].insert(evs[p].end(), th[a].begin(), th[a].end());
      // keep the selected eigenvectors
      if (k > 0)
        HIPCHK(hipMemcpyAsync(Yv + off_y[p] + (int64_t)ksel[p] * dv[p], LP + ld[p].v_off,
                              sizeof(double) * dv[p] * k, hipMemcpyDeviceToDevice, stream));
      ksel[p] += k;
      if (k < s) {
        res.omega = std::max(res.omega, th[a][k]);
      } else if (ksel[p] < dv[p]) {
        next.push_back(p);
        // deflate: C' <- C' - (X Theta) X^T, X Theta built in the T1 scratch
        std::vector<double> hx((size_t)dv[p] * s);
        HIPCHK(hipMemcpyAsync(hx.data(), LP + ld[p].v_off, sizeof(double) * hx.size(),
                              hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (int q = 0; q < s; ++q)
          for (int r = 0; r < dv[p]; ++r) hx[(size_t)q * dv[p] + r] *= th[a][q];
        HIPCHK(hipMemcpyAsync(LP + ld[p].t_off, hx.data(), sizeof(double) * hx.size(),
                              hipMemcpyHostToDevice, stream));
        gdef.push_back(GemmDesc{ld[p].t_off, ld[p].v_off, off_dd[p], dv[p], dv[p], s, dv[p], dv[p],
                                dv[p]});
      }
    }
    if (!gdef.empty()) {
      GemmDesc *d_gdef = pool.up(stream, gdef);
      int mx = 0;
      for (auto &g : gdef) mx = std::max(mx, g.M);
      HIPCHK(DenseOps<double>::gemm(stream, LP, LP, LP, d_gdef, (int)gdef.size(), mx, mx, false, true,
                                    -1.0, 1.0, false));
    }
    active.swap(next);
  }
  // eigenvectors back to J space: y = L^-T x, J = Z y, v = M J
  std::vector<int64_t> off_jv(np);
  int64_t tj = 0;
  int max_k = 1;
  for (int p = 0; p < np; ++p) {
    off_jv[p] = tj;
    tj += (int64_t)ncv[p] * std::max(1, ksel[p]);
    max_k = std::max(max_k, ksel[p]);
  }
  double *Jv = pool.zeros(stream, tj), *Vv = pool.zeros(stream, tj);
  std::vector<MatDesc> mdy(np);
  std::vector<GemmDesc> gz(np), gm(np);
  for (int p = 0; p < np; ++p) {
    mdy[p] = MatDesc{off_dd[p], off_y[p], dv[p], ksel[p], std::max(1, dv[p]), std::max(1, dv[p])};
    gz[p] = GemmDesc{off_z[p], off_y[p], off_jv[p], ncv[p], ksel[p], dv[p], std::max(1, ncv[p]),
                     std::max(1, dv[p]), std::max(1, ncv[p])};
    gm[p] = GemmDesc{off_c[p], off_jv[p], off_jv[p], ncv[p], ksel[p], ncv[p], std::max(1, ncv[p]),
                     std::max(1, ncv[p]), std::max(1, ncv[p])};
  }
  MatDesc *d_mdy = pool.up(stream, mdy);
  GemmDesc *d_gz = pool.up(stream, gz), *d_gm = pool.up(stream, gm);
  double *Vtmp = pool.zeros(stream, tj);
  HIPCHK(DenseOps<double>::trsm(stream, By, Yv, d_mdy, mdy.data(), np, true));
  HIPCHK(DenseOps<double>::gemm(stream, Zd, Yv, Jv, d_gz, np, max_c, max_k, false, false, 1.0, 0.0, false));
  HIPCHK(DenseOps<double>::gemm(stream, Mc, Jv, Vtmp, d_gm, np, max_c, max_k, false, false, 1.0, 0.0, false));
  (void)Vv;
  std::vector<double> hv(tj);
  std::vector<int> hstat(3 * np + 2 * nside + 4);
  HIPCHK(hipMemcpyAsync(hv.data(), Vtmp, sizeof(double) * tj, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hstat.data(), d_stat, sizeof(int) * hstat.size(), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  for (int e = 0; e < nside + 2 * np; ++e)
    if (hstat[e])
      throw NotSpdError("adaptive pair problems: non-positive pivot in a pair factor (Assumption 2 may fail)");
  // ---- host: face rows
  for (int p = 0; p < np; ++p) {
    const PairHost &ph = pairs[p];
    const int nc = ncv[p];
    std::vector<double> ev = evs[p];
    std::sort(ev.begin(), ev.end(), [](double x, double y) { return x > y; });
    st.eigs[ph.f] = ev;
    const int k = ksel[p];
    if (k == 0) continue;
    const Glob &gl = P.globs[ph.gi];
    const GlobCov &cv = P.cov[ph.gi];
    const int nfd = (int)gl.dofs.size();
    std::vector<double> Hq;
    int m = cv.m;
    if (m > 0) {
      Hq = cv.hrow;
      orthonormalize(Hq, nfd, m);
    }
    std::vector<double> rows;
    for (int q = 0; q < k; ++q) {
      std::vector<double> r(nfd);
      for (int t = 0; t < nfd; ++t) r[t] = hv[off_jv[p] + (size_t)q * nc + ph.face_c[t]];
      // project onto the null space of the face's existing constraint rows
      for (int a = 0; a < m; ++a) {
        double dt = 0;
        for (int t = 0; t < nfd; ++t) dt += Hq[(size_t)a * nfd + t] * r[t];
        for (int t = 0; t < nfd; ++t) r[t] -= dt * Hq[(size_t)a * nfd + t];
      }
      double mx = 0;
      for (double v : r) mx = std::max(mx, std::fabs(v));
      if (mx == 0) continue;
      for (double &v : r) v /= mx;
      rows.insert(rows.end(), r.begin(), r.end());
    }
    const int added = (int)(rows.size() / nfd);
    P.extra_rows[ph.gi].insert(P.extra_rows[ph.gi].end(), rows.begin(), rows.end());
    P.extra_k[ph.gi] += added;
    res.n_added += added;
  }
  return res;
}

}  // namespace bddc
