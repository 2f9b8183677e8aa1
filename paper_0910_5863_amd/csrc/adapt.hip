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
#include <cstdio>
#include <cstdlib>

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

// Ssum = Sh_i + Sh_j + rho Q Q^T ; Xb = Sh_j  (per pair, n x n, ld n)
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
  Xb[off_p[e] + i] = Sh[off_j[e] + i];
  BJ[off_p[e] + i] = 0.0;
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

// dst[idx[i]] = val[i]
__global__ void scatter_values_kernel(const int64_t *idx, const double *val, int64_t n, double *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = val[i];
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

// A <- (A + A^T) / 2 in place (entries a >= b of every entry touch both halves)
__global__ void symmetrize_kernel(double *A, const int64_t *off, const int *n) {
  const int e = blockIdx.y;
  const int64_t m = n[e];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * m) return;
  const int r = (int)(i % m), c = (int)(i / m);
  if (r <= c) return;
  double *a = A + off[e];
  const double v = 0.5 * (a[r + (int64_t)c * m] + a[c + (int64_t)r * m]);
  a[r + (int64_t)c * m] = v;
  a[c + (int64_t)r * m] = v;
}

// ---------------------------------------------------------------------------
// batched LOBPCG: dominant eigenpairs of a symmetric d x d matrix per entry

constexpr int LOB_S = LOB_MAXB / 3;  // block size (columns of X, W and P)
constexpr int LOCK_MAX = 256;        // eigenvectors locked from earlier rounds
constexpr int STAGE_ROWS = 256;      // rows of a block staged in LDS per pass
constexpr int DOT_ROWS = 64;         // rows per chunk of the block products U^T V
constexpr int DOT_PER_THREAD = (LOB_MAXB * LOB_MAXB + 255) / 256;

struct LobDesc {
  int64_t a_off;    // d x d matrix (ld d)
  int64_t v_off;    // 6 blocks of d x s: X, AX, W, AW, P, AP (ld d)
  int64_t t_off;    // 2 blocks of d x s scratch
  int64_t lock_off; // nl locked orthonormal eigenvectors (d x nl, ld d)
  int nl;
  int d, s;
  int need;         // number of leading eigenpairs that must converge (>= 1)
  double tau;       // threshold: pairs with theta >= tau are needed, plus one below
};

struct LobOut {
  int iters;
  int converged;
  int nconv;
  // time per phase (wall clock ticks, thread 0): A products, orthonormalization,
  // Rayleigh-Ritz products, Rayleigh-Ritz eigensolves
  long long ticks[4];
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
// Sweeps stop when every off-diagonal entry is below 1e-15 sqrt(|h_pp h_qq|)
// (relative accuracy for semidefinite H) or below 1e-17 of the Frobenius norm
// (rotations preserve it; smaller entries cannot move the eigenpairs), or the
// off-diagonal mass is below 1e-30 of the total, or after 20 sweeps.
__device__ void jacobi_eig(double (*H)[LOB_MAXB + 1], double (*V)[LOB_MAXB + 1], int n,
                           double *cs, double *sn, double *red) {
  __shared__ int pp[LOB_MAXB / 2 + 1], qq[LOB_MAXB / 2 + 1];
  const int tid = threadIdx.x;  // launched with 256 threads
  for (int i = tid; i < n * n; i += blockDim.x) V[i % n][i / n] = (i % n == i / n) ? 1.0 : 0.0;
  const int m = (n + 1) / 2 * 2;  // even number of players (a dummy when n is odd)
  // round-robin schedule: player 0 stays, the others move one place per step,
  // so at step t position i >= 1 holds player 1 + ((i - 1 - t) mod (m - 1))
  auto player = [m](int i, int t) {
    if (i == 0) return 0;
    const int r = (i - 1 - t) % (m - 1);
    return 1 + (r < 0 ? r + m - 1 : r);
  };
  __syncthreads();
  double tot = 0;
  for (int i = tid; i < n * n; i += blockDim.x) tot += H[i % n][i / n] * H[i % n][i / n];
  tot = block_sum(tot, red);
  const double floor_abs = 1e-17 * sqrt(tot);
  for (int sweep = 0; sweep < 20; ++sweep) {
    double off = 0, viol = 0;
    for (int i = tid; i < n * n; i += blockDim.x) {
      const int a = i % n, b = i / n;
      if (a == b) continue;
      const double h = H[a][b];
      off += h * h;
      if (fabs(h) > fmax(1e-15 * sqrt(fabs(H[a][a] * H[b][b])), floor_abs)) viol += 1;
    }
    off = block_sum(off, red);
    viol = block_sum(viol, red);
    if (viol == 0 || off <= 1e-30 * tot || tot == 0) break;
    for (int step = 0; step < m - 1; ++step) {
      // the step's pairs (player(k), player(m-1-k)), k < m/2, and rotations
      if (tid < m / 2) {
        int p = player(tid, step), q = player(m - 1 - tid, step);
        if (p > q) {
          const int t = p;
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
        pp[tid] = p;
        qq[tid] = q;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // 256 threads: pair slot tid & 31, every 8th column / row from tid >> 5
      const int k = tid & 31, g = tid >> 5;
      const bool act = k < m / 2 && qq[min(k, m / 2 - 1)] < n;
      const int p = act ? pp[k] : 0, q = act ? qq[k] : 0;
      const double c = act ? cs[k] : 1.0, s = act ? sn[k] : 0.0;
      // rows: H <- J^T H
      if (act)
        for (int col = g; col < n; col += 8) {
          const double hp = H[p][col], hq = H[q][col];
          H[p][col] = c * hp - s * hq;
          H[q][col] = s * hp + c * hq;
        }
      __syncthreads();
      // columns: H <- H J, V <- V J
      if (act)
        for (int row = g; row < n; row += 8) {
          const double hp = H[row][p], hq = H[row][q];
          H[row][p] = c * hp - s * hq;
          H[row][q] = s * hp + c * hq;
          const double vp = V[row][p], vq = V[row][q];
          V[row][p] = c * vp - s * vq;
          V[row][q] = s * vp + c * vq;
        }
      __syncthreads();
    }
  }
}

// One work-group per entry.  The basis V = [X W P] is kept orthonormal
// explicitly: W (the residuals) is orthogonalized against X and P by two
// passes of block Gram-Schmidt, P (the W and P part of the new Ritz vectors)
// against the new X, and each block is orthonormalized by the scaled
// eigen-decomposition of its Gram matrix (columns of a near-dependent block
// are dropped).  The Rayleigh-Ritz step is then the standard symmetric problem
// V^T A V, solved in LDS by Jacobi rotations.  Blocks live in global memory;
// every update of a block is row-owned (one thread writes a whole row), so
// blocks are updated in place.
__global__ __launch_bounds__(256) void lobpcg_kernel(double *pool, const LobDesc *desc,
                                                     LobOut *out, int maxit, double tol,
                                                     double tol_ind) {
  __shared__ double Hs[LOB_MAXB][LOB_MAXB + 1];  // projected / Gram matrices
  __shared__ double Qs[LOB_MAXB][LOB_MAXB + 1];  // their eigenvectors
  __shared__ double Cs[LOB_MAXB][2 * LOB_S + 1]; // Ritz coefficients (X part, P part)
  __shared__ double Ms[LOB_S][LOB_S + 1];        // orthonormalizing map of a block
  __shared__ double stage[STAGE_ROWS * LOB_S];    // staged rows, or locked coefficients
  __shared__ double su[DOT_ROWS][LOB_MAXB + 1];   // row chunks of block products
  __shared__ double sv[DOT_ROWS][LOB_MAXB + 1];
  __shared__ double theta[LOB_MAXB], gsc[LOB_MAXB], dinv[LOB_MAXB], res[LOB_S];
  __shared__ double cs[LOB_MAXB / 2 + 1], sn[LOB_MAXB / 2 + 1], red[8];
  __shared__ int perm[LOB_MAXB + 2];
  __shared__ int s_keep, s_done;
  const LobDesc D = desc[blockIdx.x];
  const int d = D.d, s = D.s, tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  const double *A = pool + D.a_off;
  double *X = pool + D.v_off, *AX = X + (int64_t)d * s, *W = AX + (int64_t)d * s;
  double *AW = W + (int64_t)d * s, *P = AW + (int64_t)d * s, *AP = P + (int64_t)d * s;
  double *T1 = pool + D.t_off;
  const double *YL = pool + D.lock_off;
  const int nl = D.nl;
  int nw = 0, npc = 0;  // columns held in W and P
  long long ticks[4] = {0, 0, 0, 0};  // phase timing (see LobOut)

  // o[a * ldo + b] = U[:, a] . V[:, b]  (one wave per entry)
  auto dots = [&](const double *U, int nu, const double *V, int nv, double *o, int ldo) {
    for (int i = wave; i < nu * nv; i += nwave) {
      const int a = i % nu, b = i / nu;
      const double *u = U + (int64_t)a * d, *v = V + (int64_t)b * d;
      double acc = 0;
      for (int r = lane; r < d; r += 64) acc += u[r] * v[r];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (lane == 0) o[a * ldo + b] = acc;
    }
    __syncthreads();
  };
  // o[a * ldo + b] = u_a . v_b for nu, nv <= LOB_MAXB columns given by
  // accessors: the rows go through LDS in chunks, each thread owns a few
  // entries and sums them in row order (no atomics, fixed order)
  auto block_dot = [&](auto ucol, int nu, auto vcol2, int nv, double *o, int ldo) {
    const int ne = nu * nv;
    double acc[DOT_PER_THREAD];
#pragma unroll
    for (int q = 0; q < DOT_PER_THREAD; ++q) acc[q] = 0;
    for (int c0 = 0; c0 < d; c0 += DOT_ROWS) {
      const int cn = min(DOT_ROWS, d - c0);
      __syncthreads();
      for (int i = tid; i < DOT_ROWS * nu; i += nt) {
        const int r = i % DOT_ROWS, a = i / DOT_ROWS;
        su[r][a] = r < cn ? ucol(a)[c0 + r] : 0.0;
      }
      for (int i = tid; i < DOT_ROWS * nv; i += nt) {
        const int r = i % DOT_ROWS, b = i / DOT_ROWS;
        sv[r][b] = r < cn ? vcol2(b)[c0 + r] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < DOT_PER_THREAD; ++q) {
        const int e = tid + q * nt;
        if (e < ne) {
          const int a = e % nu, b = e / nu;
          double t = 0;
          for (int r = 0; r < cn; ++r) t += su[r][a] * sv[r][b];
          acc[q] += t;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < DOT_PER_THREAD; ++q) {
      const int e = tid + q * nt;
      if (e < ne) o[(e % nu) * ldo + e / nu] = acc[q];
    }
    __syncthreads();
  };
  auto cols = [d](const double *base) {
    return [base, d](int a) { return base + (int64_t)a * d; };
  };
  // V[:, b] -= sum_a U[:, a] c[a * ldc + b] for b < nv (AV -= AU c alongside)
  auto sub_prod = [&](double *V, double *AV, int nv, const double *U, const double *AU, int nu,
                      const double *c, int ldc) {
    for (int r = tid; r < d; r += nt) {
      double acc[LOB_S], aacc[LOB_S];
#pragma unroll
      for (int q = 0; q < LOB_S; ++q) acc[q] = aacc[q] = 0;
      // eight columns of U (and A U) loaded per batch
      for (int a0 = 0; a0 < nu; a0 += 8) {
        double u8[8], au8[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          u8[t] = a0 + t < nu ? U[r + (int64_t)(a0 + t) * d] : 0.0;
          au8[t] = (AV && a0 + t < nu) ? AU[r + (int64_t)(a0 + t) * d] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (a0 + t >= nu) break;
          const double *ca = c + (a0 + t) * ldc;
#pragma unroll
          for (int q = 0; q < LOB_S; ++q) {
            if (q < nv) {
              acc[q] += u8[t] * ca[q];
              aacc[q] += au8[t] * ca[q];
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < LOB_S; ++q) {
        if (q < nv) {
          V[r + (int64_t)q * d] -= acc[q];
          if (AV) AV[r + (int64_t)q * d] -= aacc[q];
        }
      }
    }
    __syncthreads();
  };
  // V[:, 0..kp) = V[:, 0..nv) M  (M in Ms)
  auto right_mul = [&](double *V, int nv, int kp) {
    for (int r = tid; r < d; r += nt) {
      double acc[LOB_S], vr[LOB_S];
#pragma unroll
      for (int q = 0; q < LOB_S; ++q) acc[q] = 0;
#pragma unroll
      for (int b = 0; b < LOB_S; ++b) vr[b] = b < nv ? V[r + (int64_t)b * d] : 0.0;
#pragma unroll
      for (int b = 0; b < LOB_S; ++b) {
        if (b >= nv) break;
        const double v = vr[b];
#pragma unroll
        for (int q = 0; q < LOB_S; ++q)
          if (q < kp) acc[q] += v * Ms[b][q];
      }
#pragma unroll
      for (int q = 0; q < LOB_S; ++q)
        if (q < kp) V[r + (int64_t)q * d] = acc[q];
    }
    __syncthreads();
  };
  // orthonormalize the nv columns of V (AV alongside when given): with
  // Dg = diag(G)^-1/2, Dg G Dg = Q diag(g) Q^T, V <- V Dg Q g^-1/2 over g > thr.
  // Returns the number of columns kept.
  auto svqb = [&](double *V, double *AV, int nv, double thr) -> int {
    if (nv == 0) return 0;
    block_dot(cols(V), nv, cols(V), nv, &Hs[0][0], LOB_MAXB + 1);
    for (int a = tid; a < nv; a += nt) dinv[a] = Hs[a][a] > 0 ? 1.0 / sqrt(Hs[a][a]) : 0.0;
    __syncthreads();
    for (int i = tid; i < nv * nv; i += nt) {
      const int a = i % nv, b = i / nv;
      Hs[a][b] *= dinv[a] * dinv[b];
    }
    __syncthreads();
    jacobi_eig(Hs, Qs, nv, cs, sn, red);
    if (tid == 0) {
      int keep = 0;
      for (int a = 0; a < nv; ++a)
        if (Hs[a][a] > thr) {
          perm[keep] = a;
          gsc[keep] = 1.0 / sqrt(Hs[a][a]);
          ++keep;
        }
      s_keep = keep;
    }
    __syncthreads();
    const int kp = s_keep;
    for (int i = tid; i < nv * kp; i += nt) {
      const int b = i % nv, q = i / nv;
      Ms[b][q] = dinv[b] * Qs[b][perm[q]] * gsc[q];
    }
    __syncthreads();
    right_mul(V, nv, kp);
    if (AV) right_mul(AV, nv, kp);
    return kp;
  };
  // orthonormalization of a well-conditioned block: V <- V L^-T with
  // V^T V = L L^T (Cholesky in LDS).  Returns false (V untouched) if a pivot
  // falls below 1e-8 of its diagonal entry (condition above 1e4: the caller
  // then uses the eigen-decomposition, which drops dependent columns).
  auto cholqr = [&](double *V, double *AV, int nv) -> bool {
    if (nv == 0) return true;
    block_dot(cols(V), nv, cols(V), nv, &Hs[0][0], LOB_MAXB + 1);
    if (tid == 0) {
      int ok = 1;
      for (int j = 0; j < nv && ok; ++j) {
        double dj = Hs[j][j];
        for (int k = 0; k < j; ++k) dj -= Hs[j][k] * Hs[j][k];
        if (!(dj > 1e-8 * Hs[j][j])) {
          ok = 0;
          break;
        }
        dj = sqrt(dj);
        Hs[j][j] = dj;
        for (int i = j + 1; i < nv; ++i) {
          double v = Hs[i][j];
          for (int k = 0; k < j; ++k) v -= Hs[i][k] * Hs[j][k];
          Hs[i][j] = v / dj;
        }
      }
      s_keep = ok;
    }
    __syncthreads();
    if (!s_keep) return false;
    // columns of L^-1 (thread j), then Ms = L^-T
    if (tid < nv) {
      const int j = tid;
      for (int i = 0; i < nv; ++i) Qs[i][j] = 0.0;
      for (int i = j; i < nv; ++i) {
        double y = (i == j) ? 1.0 : 0.0;
        for (int m = j; m < i; ++m) y -= Hs[i][m] * Qs[m][j];
        Qs[i][j] = y / Hs[i][i];
      }
    }
    __syncthreads();
    for (int i = tid; i < nv * nv; i += nt) {
      const int b = i % nv, q = i / nv;
      Ms[b][q] = q >= b ? Qs[q][b] : 0.0;
    }
    __syncthreads();
    right_mul(V, nv, nv);
    if (AV) right_mul(AV, nv, nv);
    return true;
  };
  // V <- V - YL (YL^T V): keep a block orthogonal to the locked vectors
  auto project_locked = [&](double *V, int nv) {
    if (nl == 0 || nv == 0) return;
    dots(YL, nl, V, nv, stage, LOB_S);
    sub_prod(V, nullptr, nv, YL, nullptr, nl, stage, LOB_S);
  };
  // AV = A V for nv columns; V staged through LDS in chunks of rows
  auto apply_A = [&](const double *V, double *AV, int nv) {
    for (int r0 = 0; r0 < d; r0 += nt) {
      const int r = r0 + tid;
      double acc[LOB_S];
#pragma unroll
      for (int q = 0; q < LOB_S; ++q) acc[q] = 0;
      for (int c0 = 0; c0 < d; c0 += STAGE_ROWS) {
        const int cn = min(STAGE_ROWS, d - c0);
        __syncthreads();
        for (int i = tid; i < cn * LOB_S; i += nt) {
          const int c = i % cn, q = i / cn;
          stage[c * LOB_S + q] = q < nv ? V[c0 + c + (int64_t)q * d] : 0.0;
        }
        __syncthreads();
        if (r < d) {
          // eight loads of A in flight per thread
          for (int c = 0; c < cn; c += 8) {
            double a8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a8[u] = c + u < cn ? A[r + (int64_t)(c0 + c + u) * d] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              if (c + u < cn) {
#pragma unroll
                for (int q = 0; q < LOB_S; ++q) acc[q] += a8[u] * stage[(c + u) * LOB_S + q];
              }
            }
          }
        }
      }
      if (r < d)
        for (int q = 0; q < nv; ++q) AV[r + (int64_t)q * d] = acc[q];
    }
    __syncthreads();
  };
  // column b of V = [X W P] and of A V
  auto vcol = [&](int b) -> const double * {
    return b < s ? X + (int64_t)b * d
                 : (b < s + nw ? W + (int64_t)(b - s) * d : P + (int64_t)(b - s - nw) * d);
  };
  auto avcol = [&](int b) -> const double * {
    return b < s ? AX + (int64_t)b * d
                 : (b < s + nw ? AW + (int64_t)(b - s) * d : AP + (int64_t)(b - s - nw) * d);
  };
  // Rayleigh-Ritz on the current n = s + nw + npc columns: theta, and the
  // coefficients of the new X (Cs[:, 0..s)) and of the new P (Cs[:, s..2s):
  // the same vectors without their X rows)
  auto rayleigh_ritz = [&](int n) {
    // H = V^T A V, symmetrized
    block_dot(vcol, n, avcol, n, &Hs[0][0], LOB_MAXB + 1);
    for (int i = tid; i < n * n; i += nt) {
      const int a = i % n, b = i / n;
      if (a < b) {
        const double h = 0.5 * (Hs[a][b] + Hs[b][a]);
        Hs[a][b] = Hs[b][a] = h;
      }
    }
    __syncthreads();
    const long long tj = wall_clock64();
    jacobi_eig(Hs, Qs, n, cs, sn, red);
    ticks[3] += wall_clock64() - tj;
    if (tid == 0) {
      for (int a = 0; a < n; ++a) perm[a] = a;
      for (int a = 0; a < s; ++a)
        for (int b = a + 1; b < n; ++b)
          if (Hs[perm[b]][perm[b]] > Hs[perm[a]][perm[a]]) {
            const int t = perm[a];
            perm[a] = perm[b];
            perm[b] = t;
          }
      for (int q = 0; q < s; ++q) theta[q] = Hs[perm[q]][perm[q]];
    }
    __syncthreads();
    for (int i = tid; i < n * s; i += nt) {
      const int b = i % n, q = i / n;
      const double c = Qs[b][perm[q]];
      Cs[b][q] = c;
      Cs[b][LOB_S + q] = b < s ? 0.0 : c;
    }
    __syncthreads();
  };
  // X <- V Cx, P <- V Cp and their images (row-owned, in place)
  auto ritz_update = [&](int n, bool with_p) {
    for (int pass = 0; pass < 2; ++pass) {
      double *XO = pass ? AX : X, *PO = pass ? AP : P;
      for (int r = tid; r < d; r += nt) {
        double ax[LOB_S], ap[LOB_S];
#pragma unroll
        for (int q = 0; q < LOB_S; ++q) ax[q] = ap[q] = 0;
        for (int b = 0; b < n; ++b) {
          const double v = (pass ? avcol(b) : vcol(b))[r];
#pragma unroll
          for (int q = 0; q < LOB_S; ++q) {
            ax[q] += v * Cs[b][q];
            ap[q] += v * Cs[b][LOB_S + q];
          }
        }
#pragma unroll
        for (int q = 0; q < LOB_S; ++q) {
          if (q < s) {
            XO[r + (int64_t)q * d] = ax[q];
            if (with_p) PO[r + (int64_t)q * d] = ap[q];
          }
        }
      }
      __syncthreads();
    }
  };

  int it = 0, nconv = 0;
  bool done = false;
  for (int q = tid; q < LOB_MAXB; q += nt) theta[q] = 0;
  __syncthreads();
  // start block: orthonormal and orthogonal to the locked vectors
  int kx = s;
  for (int pass = 0; pass < 2 && kx == s; ++pass) {
    project_locked(X, s);
    if (pass == 0 || !cholqr(X, nullptr, s)) kx = svqb(X, nullptr, s, 1e-10);
  }
  if (kx == s) {
    long long t0 = wall_clock64();
    apply_A(X, AX, s);
    ticks[0] += wall_clock64() - t0;
    t0 = wall_clock64();
    rayleigh_ritz(s);
    ticks[2] += wall_clock64() - t0;
    ritz_update(s, false);
  }
  for (it = 1; it <= maxit && kx == s; ++it) {
    // residuals W = A X - X theta and their norms
    for (int i = tid; i < d * s; i += nt) W[i] = AX[i] - X[i] * theta[i / d];
    __syncthreads();
    project_locked(W, s);
    for (int q = wave; q < s; q += nwave) {
      double acc = 0;
      for (int r = lane; r < d; r += 64) acc += W[r + (int64_t)q * d] * W[r + (int64_t)q * d];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (lane == 0) res[q] = sqrt(acc);
    }
    __syncthreads();
    // the pairs with theta >= tau must converge to tol; the first one below
    // tau only sets the indicator and converges to tol_ind
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
    if (s_done) {
      done = true;
      break;
    }
    if (it == maxit) break;
    // search directions: unit residuals, orthonormal and orthogonal to X, P
    for (int i = tid; i < d * s; i += nt) {
      const int q = i / d;
      W[i] = res[q] > 0 ? W[i] / res[q] : 0.0;
    }
    __syncthreads();
    long long to = wall_clock64();
    nw = s;
    for (int pass = 0; pass < 2 && nw > 0; ++pass) {
      project_locked(W, nw);
      block_dot(cols(X), s, cols(W), nw, &Cs[0][0], 2 * LOB_S + 1);
      sub_prod(W, nullptr, nw, X, nullptr, s, &Cs[0][0], 2 * LOB_S + 1);
      if (npc > 0) {
        block_dot(cols(P), npc, cols(W), nw, &Cs[0][0], 2 * LOB_S + 1);
        sub_prod(W, nullptr, nw, P, nullptr, npc, &Cs[0][0], 2 * LOB_S + 1);
      }
      if (!cholqr(W, nullptr, nw)) nw = svqb(W, nullptr, nw, 1e-10);
    }
    ticks[1] += wall_clock64() - to;
    if (nw == 0 && npc == 0) break;  // no direction left: stagnation
    long long t1 = wall_clock64();
    apply_A(W, AW, nw);
    ticks[0] += wall_clock64() - t1;
    const int n = s + nw + npc;
    t1 = wall_clock64();
    rayleigh_ritz(n);
    ticks[2] += wall_clock64() - t1;
    ritz_update(n, true);
    // P: orthogonal to the new X, orthonormal
    to = wall_clock64();
    npc = s;
    for (int pass = 0; pass < 2 && npc > 0; ++pass) {
      block_dot(cols(X), s, cols(P), npc, &Cs[0][0], 2 * LOB_S + 1);
      sub_prod(P, AP, npc, X, AX, s, &Cs[0][0], 2 * LOB_S + 1);
      if (!cholqr(P, AP, npc)) npc = svqb(P, AP, npc, 1e-10);
    }
    ticks[1] += wall_clock64() - to;
    nw = 0;
  }
  if (tid == 0) {
    out[blockIdx.x].iters = it;
    out[blockIdx.x].converged = done ? 1 : 0;
    out[blockIdx.x].nconv = nconv;
    for (int q = 0; q < 4; ++q) out[blockIdx.x].ticks[q] = ticks[q];
  }
  // eigenvalues into the first column of T1 for the host
  __syncthreads();
  for (int q = tid; q < s; q += nt) T1[q] = theta[q];
}

}  // namespace

// ---------------------------------------------------------------------------
// host orchestration

namespace {

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
  const auto t_start = std::chrono::steady_clock::now();
  auto log = [&](const char *what) {
    if (!S.verbose) return;
    HIPCHK(hipStreamSynchronize(stream));
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    std::fprintf(stderr, "[bddc adapt %8.3f s] %s\n", el, what);
    std::fflush(stderr);
  };
  S.factor_schur();  // Schur complements S_i (original basis) in S.d_S
  log("schur complements");
  const Layout &L = S.L;
  const int dpn = P.mesh.dpn;
  const int nf = (int)P.face_ids.size();
  st.eigs.assign(nf, {});
  std::vector<char> is_corner(P.n_glob, 0);
  for (int64_t g : P.corner_gdofs) is_corner[g] = 1;
  // the pair structure depends on the mesh, the partition and the constraints
  // chosen at setup only (adaptive rows of earlier calls are removed first):
  // built once, then reused
  if (!st.pairs_ready) {
    std::vector<AdaptPair> &pairs = st.pairs;
    pairs.clear();
    for (int f = 0; f < nf; ++f) {
      AdaptPair ph;
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
      // Z is sparse: one unit entry per column plus the explicit averages' rows
      ph.zptr.assign(1, 0);
      for (int c = 0; c < ph.d; ++c) {
        for (int r = 0; r < nc; ++r)
          if (cols[c][r] != 0.0) {
            ph.zrow.push_back(r);
            ph.zval.push_back(cols[c][r]);
          }
        ph.zptr.push_back((int)ph.zrow.size());
      }
      pairs.push_back(std::move(ph));
    }
    st.pairs_ready = true;
  }
  const std::vector<AdaptPair> &pairs = st.pairs;
  const int np = (int)pairs.size();
  res.n_pairs = np;
  log("pair index data (host)");
  if (np == 0) return res;

  // ---- device stage 1: Schur complements of S_i onto each pair's shared dofs
  Pool pool{&S.alloc};
  // inverses of the diagonal blocks of a batch of factors (written by potrf)
  auto dinv_for = [&](const std::vector<MatDesc> &md, double *&dv, int64_t *&doff) {
    std::vector<int64_t> off;
    const int64_t t = dinv_layout(md.data(), (int)md.size(), off);
    dv = pool.zeros(stream, t);
    doff = pool.up(stream, off);
  };
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
  double *dv_n;
  int64_t *do_n;
  dinv_for(mdn, dv_n, do_n);
  HIPCHK(DenseOps<double>::potrf(stream, Snn, d_mdn, mdn.data(), nside, d_stat, dv_n, do_n));
  auto check = [&](int first, int count, const char *what) {
    std::vector<int> hs(count);
    HIPCHK(hipMemcpyAsync(hs.data(), d_stat + first, sizeof(int) * count, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    int bad = 0, firstbad = -1;
    for (int e = 0; e < count; ++e)
      if (hs[e]) bad++, firstbad = firstbad < 0 ? e : firstbad;
    if (bad)
      throw NotSpdError(std::string("adaptive pair problems: ") + what + ": " + std::to_string(bad) +
                        " factors with a non-positive pivot (first entry " + std::to_string(firstbad) +
                        "); Assumption 2 may not hold");
  };
  check(0, nside, "non-shared interface blocks");
  HIPCHK(DenseOps<double>::trsm(stream, Snn, Sns, d_mdn, mdn.data(), nside, false, dv_n, do_n));
  // Sh gets the Schur complement; Sns and Sh live in different pools
  HIPCHK(DenseOps<double>::gemm(stream, Sns, Sns, Sh, d_gsh, nside, max_ns, max_ns, true, false,
                                -1.0, 1.0, false, gsh.data()));

  log("pair Schur complements");
  // ---- stage 2: parallel sum and the reduced pair matrices
  std::vector<int64_t> off_i(np), off_j(np), off_p(np), q_off(np), off_c(np), c_off(np), off_z(np),
      off_cz(np), off_dd(np);
  std::vector<int> nsp(np), nqv(np), ncv(np), dv(np);
  std::vector<double> rho(np), Qall, wall, zval;
  std::vector<int64_t> zdst;
  std::vector<int> call;
  int64_t tp = 0, tc = 0, tz = 0, tdd = 0, tcz = 0;
  int max_c = 0, max_d = 0;
  for (int p = 0; p < np; ++p) {
    const AdaptPair &ph = pairs[p];
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
    off_z[p] = tz;
    for (int c = 0; c < ph.d; ++c)
      for (int k = ph.zptr[c]; k < ph.zptr[c + 1]; ++k) {
        zdst.push_back(tz + ph.zrow[k] + (int64_t)c * ncv[p]);
        zval.push_back(ph.zval[k]);
      }
    tz += (int64_t)ncv[p] * dv[p];
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
  double *dv_s;
  int64_t *do_s;
  dinv_for(mds, dv_s, do_s);
  HIPCHK(DenseOps<double>::potrf(stream, Ssum, d_mds, mds.data(), np, stat2, dv_s, do_s));
  check(nside, np, "sum of the Schur complements");
  HIPCHK(DenseOps<double>::trsm(stream, Ssum, Xb, d_mds, mds.data(), np, false, dv_s, do_s));
  HIPCHK(DenseOps<double>::trsm(stream, Ssum, Xb, d_mds, mds.data(), np, true, dv_s, do_s));
  // BJ = Sh_i (Sh_i + Sh_j)^+ Sh_j, the product form of the parallel sum (no
  // cancellation between the two large terms of Sh_i - Sh_i (..)^+ Sh_i when
  // the coefficients of i and j differ by orders of magnitude)
  HIPCHK(DenseOps<double>::gemm(stream, Sh, Xb, BJf, d_gbj, np, max_sp, max_sp, false, false, 1.0,
                                0.0, false, gbj.data()));
  symmetrize_kernel<<<dim3(nblocks((int64_t)max_sp * max_sp), np), TPB, 0, stream>>>(BJf, d_off_p, d_nsp);
  HIPCHK(hipGetLastError());
  double *Mc = pool.zeros(stream, tc), *BJc = pool.zeros(stream, tc);
  int *d_call = pool.up(stream, call), *d_nc = pool.up(stream, ncv);
  int64_t *d_c_off = pool.up(stream, c_off), *d_off_c = pool.up(stream, off_c);
  int64_t *d_off_ss_i = pool.up(stream, off_ss_i), *d_off_ss_j = pool.up(stream, off_ss_j);
  double *d_w = pool.up(stream, wall);
  pair_restrict_kernel<<<dim3(nblocks((int64_t)max_c * max_c), np), TPB, 0, stream>>>(
      Sh, d_off_ss_i, d_off_ss_j, BJf, d_off_p, d_nsp, d_call, d_c_off, d_nc, d_w, Mc, BJc, d_off_c);
  HIPCHK(hipGetLastError());
  // My = Z^T M Z, By = Z^T BJ Z
  double *Zd = pool.zeros(stream, tz);
  {
    const int64_t *d_zdst = pool.up(stream, zdst);
    const double *d_zval = pool.up(stream, zval);
    scatter_values_kernel<<<nblocks((int64_t)zdst.size()), TPB, 0, stream>>>(d_zdst, d_zval,
                                                                         (int64_t)zdst.size(), Zd);
    HIPCHK(hipGetLastError());
  }
  double *T1 = pool.zeros(stream, tcz), *My = pool.zeros(stream, tdd),
         *By = pool.zeros(stream, tdd), *Cp = pool.zeros(stream, tdd);
  std::vector<GemmDesc> g1(np), g2(np);
  for (int p = 0; p < np; ++p) {
    g1[p] = GemmDesc{off_c[p], off_z[p], off_cz[p], ncv[p], dv[p], ncv[p], std::max(1, ncv[p]),
                     std::max(1, ncv[p]), std::max(1, ncv[p])};
    g2[p] = GemmDesc{off_z[p], off_cz[p], off_dd[p], dv[p], dv[p], ncv[p], std::max(1, ncv[p]),
                     std::max(1, ncv[p]), std::max(1, dv[p])};
  }
  GemmDesc *d_g1 = pool.up(stream, g1), *d_g2 = pool.up(stream, g2);
  HIPCHK(DenseOps<double>::gemm(stream, Mc, Zd, T1, d_g1, np, max_c, max_d, false, false, 1.0, 0.0, false, g1.data()));
  HIPCHK(DenseOps<double>::gemm(stream, Zd, T1, My, d_g2, np, max_d, max_d, true, false, 1.0, 0.0, false, g2.data()));
  HIPCHK(DenseOps<double>::gemm(stream, BJc, Zd, T1, d_g1, np, max_c, max_d, false, false, 1.0, 0.0, false, g1.data()));
  HIPCHK(DenseOps<double>::gemm(stream, Zd, T1, By, d_g2, np, max_d, max_d, true, false, 1.0, 0.0, false, g2.data()));
  // C' = L^-1 My L^-T with By = L L^T
  std::vector<MatDesc> mdd(np);
  for (int p = 0; p < np; ++p)
    mdd[p] = MatDesc{off_dd[p], off_dd[p], dv[p], dv[p], std::max(1, dv[p]), std::max(1, dv[p])};
  MatDesc *d_mdd = pool.up(stream, mdd);
  int64_t *d_off_dd = pool.up(stream, off_dd);
  int *d_dv = pool.up(stream, dv);
  int *stat3 = stat2 + np;
  double *dv_y;
  int64_t *do_y;
  dinv_for(mdd, dv_y, do_y);
  HIPCHK(DenseOps<double>::potrf(stream, By, d_mdd, mdd.data(), np, stat3, dv_y, do_y));
  check(nside + np, np, "jump-space denominator");
  // My <- L^-1 My ; Cp <- My^T ; Cp <- L^-1 Cp   (My's pool is the B operand)
  HIPCHK(DenseOps<double>::trsm(stream, By, My, d_mdd, mdd.data(), np, false, dv_y, do_y));
  transpose_kernel<<<dim3(nblocks((int64_t)max_d * max_d), np), TPB, 0, stream>>>(My, Cp, d_off_dd, d_dv);
  HIPCHK(hipGetLastError());
  HIPCHK(DenseOps<double>::trsm(stream, By, Cp, d_mdd, mdd.data(), np, false, dv_y, do_y));
  // the two solves leave C' symmetric only to ~kappa(By) eps; LOBPCG's
  // residuals cannot drop below that asymmetry, so C' is symmetrized
  symmetrize_kernel<<<dim3(nblocks((int64_t)max_d * max_d), np), TPB, 0, stream>>>(Cp, d_off_dd, d_dv);
  HIPCHK(hipGetLastError());

  log("reduced pair matrices");
  // ---- stage 3: batched LOBPCG on C'.  When a block holds only eigenvalues
  // >= tau, its vectors are locked and the pair runs again on the orthogonal
  // complement of every locked vector.
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
  double *LP = pool.zeros(stream, tdd + tv + ty);
  HIPCHK(hipMemcpyAsync(LP, Cp, sizeof(double) * tdd, hipMemcpyDeviceToDevice, stream));
  double *Yv = LP + tdd + tv;  // selected eigenvectors, also the locked block
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
  const int maxit = 1000;
  const double tol = 1e-8, tol_ind = 1e-5;
  std::vector<int> ksel(np, 0), active(np);
  std::vector<std::vector<double>> evs(np);
  std::iota(active.begin(), active.end(), 0);
  for (int round = 0; round < 64 && !active.empty(); ++round) {
    const int na = (int)active.size();
    std::vector<LobDesc> lda(na);
    std::vector<int64_t> x0off(na + 1, 0);
    for (int a = 0; a < na; ++a) {
      const int p = active[a];
      x0off[a + 1] = x0off[a] + (int64_t)dv[p] * std::min(dv[p] - ksel[p], s_max);
    }
    std::vector<double> X0all(x0off[na]);
    for (int a = 0; a < na; ++a) {
      const int p = active[a];
      ld[p].s = std::min(dv[p] - ksel[p], s_max);
      ld[p].lock_off = tdd + tv + off_y[p];
      ld[p].nl = ksel[p];
      if (ksel[p] > LOCK_MAX) throw ArgError("more than 256 adaptive rows on one face");
      lda[a] = ld[p];
      // seeded start block (splitmix64 of face, round, column, row)
      double *x0 = X0all.data() + x0off[a];
      for (int q = 0; q < ld[p].s; ++q)
        for (int r = 0; r < dv[p]; ++r) {
          uint64_t z = 0x9E3779B97F4A7C15ull *
                       (uint64_t)((((int64_t)pairs[p].f * 64 + round) * 131071 + q) * 1000003 + r + 1);
          z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
          z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
          z ^= z >> 31;
          x0[(size_t)q * dv[p] + r] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
        }
      HIPCHK(hipMemcpyAsync(LP + ld[p].v_off, x0, sizeof(double) * (x0off[a + 1] - x0off[a]),
                            hipMemcpyHostToDevice, stream));
    }
    HIPCHK(hipMemcpyAsync(ldb.p, lda.data(), sizeof(LobDesc) * na, hipMemcpyHostToDevice, stream));
    {
      LaunchScope ls(stream, "lobpcg_kernel", 0, 0);
      lobpcg_kernel<<<na, 256, 0, stream>>>(LP, ldb.as<LobDesc>(), outb.as<LobOut>(), maxit, tol,
                                            tol_ind);
      HIPCHK(hipGetLastError());
    }
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
    if (LaunchTiming *lt = launch_timing()) {
      // algorithmic work: per iteration one pass over the pair matrix C'
      // (d x d) multiplying the s-column search block
      double by = 0, fl = 0;
      for (int a = 0; a < na; ++a) {
        const double dd = dv[active[a]], it = lo[a].iters;
        by += it * 8.0 * dd * dd;
        fl += it * 2.0 * dd * dd * ld[active[a]].s;
      }
      lt->launch_amend(by, fl);
    }
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
      } else if (ksel[p] < dv[p] && lo[a].converged) {
        next.push_back(p);  // the block held only selected pairs: lock them, go on
      }
    }
    if (S.verbose) {
      int mx = 0, nu = 0;
      std::string bad;
      for (int a = 0; a < na; ++a) {
        mx = std::max(mx, lo[a].iters);
        if (!lo[a].converged) {
          nu++;
          if (nu <= 12) bad += " " + std::to_string(pairs[active[a]].f) + "(nconv " +
                               std::to_string(lo[a].nconv) + ")";
        }
      }
      long long tk[4] = {0, 0, 0, 0};
      for (int a = 0; a < na; ++a)
        for (int q = 0; q < 4; ++q) tk[q] = std::max(tk[q], lo[a].ticks[q]);
      char buf[320];
      std::snprintf(buf, sizeof buf,
                    "LOBPCG round %d: %d pairs, max iters %d, unconverged %d, continuing %d; max ms: "
                    "A %.2f, orth %.2f, RR %.2f (eig %.2f);",
                    round, na, mx, nu, (int)next.size(), tk[0] * 1e-5, tk[1] * 1e-5, tk[2] * 1e-5,
                    tk[3] * 1e-5);
      log((std::string(buf) + bad).c_str());
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
  // (the factor By of the pair denominators, whose block inverses are dv_y)
  HIPCHK(DenseOps<double>::trsm(stream, By, Yv, d_mdy, mdy.data(), np, true, dv_y, do_y));
  HIPCHK(DenseOps<double>::gemm(stream, Zd, Yv, Jv, d_gz, np, max_c, max_k, false, false, 1.0, 0.0, false, gz.data()));
  HIPCHK(DenseOps<double>::gemm(stream, Mc, Jv, Vtmp, d_gm, np, max_c, max_k, false, false, 1.0, 0.0, false, gm.data()));
  (void)Vv;
  std::vector<double> hv(tj);
  std::vector<int> hstat(3 * np + 2 * nside + 4);
  HIPCHK(hipMemcpyAsync(hv.data(), Vtmp, sizeof(double) * tj, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hstat.data(), d_stat, sizeof(int) * hstat.size(), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  for (int e = 0; e < nside + 2 * np; ++e)
    if (hstat[e])
      throw NotSpdError("adaptive pair problems: non-positive pivot in a pair factor (Assumption 2 may fail)");
  log("eigenvectors to jump space");
  // ---- host: face rows
  for (int p = 0; p < np; ++p) {
    const AdaptPair &ph = pairs[p];
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
  log("face rows (host)");
  return res;
}

}  // namespace bddc
