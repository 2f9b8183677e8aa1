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
#include <functional>
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

// block offsets of a flat launch (seg_entry): entry e gets
// ceil(count[e] / per_block) blocks; the last value is the grid size
inline std::vector<int64_t> seg_offsets(const std::vector<int64_t> &count, int64_t per_block) {
  std::vector<int64_t> off(count.size() + 1, 0);
  for (size_t e = 0; e < count.size(); ++e)
    off[e + 1] = off[e] + (std::max<int64_t>(count[e], 0) + per_block - 1) / per_block;
  if (off.back() > INT32_MAX) throw ArgError("flat launch over more than 2^31 blocks");
  return off;
}

// Flat launches over entries of uneven sizes.  Entry e owns the blocks
// [boff[e], boff[e+1]) of the launch, enough for its own elements at
// SEG_CHUNK per block (the host's seg_offsets), so no block is launched for
// the padding of the smaller entries; a block finds its entry by binary
// search over boff (uniform over the block) and covers SEG_ITEMS elements
// per thread, coalesced.
constexpr int SEG_ITEMS = 4;
constexpr int64_t SEG_CHUNK = (int64_t)TPB * SEG_ITEMS;

__device__ __forceinline__ int seg_entry(const int64_t *boff, int n, int64_t b) {
  int lo = 0, hi = n;  // boff[lo] <= b < boff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// dst[e] (rows x cols, ld = rows) = src_sub[ridx, cidx] of the source matrix
__global__ void gather_rc_kernel(const double *src, const int64_t *src_off, const int *lds,
                                 double *dst, const int64_t *dst_off, const int *ridx,
                                 const int64_t *ridx_off, const int *nrow, const int *cidx,
                                 const int64_t *cidx_off, const int *ncol, const int64_t *boff,
                                 int cnt) {
  const int64_t b = blockIdx.x;
  const int e = seg_entry(boff, cnt, b);
  const int64_t nr = nrow[e], nc = ncol[e];
  const int64_t i0 = (b - boff[e]) * SEG_CHUNK + threadIdx.x;
  const double *s = src + src_off[e];
  const int *ri = ridx + ridx_off[e], *ci = cidx + cidx_off[e];
  const int64_t ld = lds[e];
  double *d = dst + dst_off[e];
#pragma unroll
  for (int it = 0; it < SEG_ITEMS; ++it) {
    const int64_t i = i0 + (int64_t)it * TPB;
    if (i < nr * nc) {
      const int a = (int)(i % nr), c = (int)(i / nr);
      d[i] = s[ri[a] + (int64_t)ci[c] * ld];
    }
  }
}

// Ssum = Sh_i + Sh_j + rho Q Q^T ; Xb = Sh_j  (per pair, n x n, ld n; flat
// launch, seg_entry)
__global__ void pair_sum_kernel(const double *Sh, const int64_t *off_i, const int64_t *off_j,
                                const int *ns, double *Ssum, double *Xb, double *BJ,
                                const int64_t *off_p, const double *Q, const int64_t *q_off,
                                const int *nq, const double *rho, const int64_t *boff, int cnt) {
  const int64_t blk = blockIdx.x;
  const int e = seg_entry(boff, cnt, blk);
  const int64_t n = ns[e];
  const int64_t i0 = (blk - boff[e]) * SEG_CHUNK + threadIdx.x;
  const double *Si = Sh + off_i[e], *Sj = Sh + off_j[e], *Qe = Q + q_off[e];
  const int kq = nq[e];
  const double rh = rho[e];
#pragma unroll
  for (int it = 0; it < SEG_ITEMS; ++it) {
    const int64_t i = i0 + (int64_t)it * TPB;
    if (i >= n * n) break;
    const int r = (int)(i % n), c = (int)(i / n);
    double v = Si[i] + Sj[i];
    for (int k = 0; k < kq; ++k) v += rh * Qe[r + k * n] * Qe[c + k * n];
    Ssum[off_p[e] + i] = v;
    Xb[off_p[e] + i] = Sj[i];
    BJ[off_p[e] + i] = 0.0;
  }
}

// compact c x c blocks: M = Dj Si Dj + Di Sj Di, BJ = (Sh_i - Sh_i X)[c,c]
// (flat launch, seg_entry)
__global__ void pair_restrict_kernel(const double *Sss, const int64_t *off_si,
                                     const int64_t *off_sj, const double *BJfull,
                                     const int64_t *off_p, const int *ns, const int *cidx,
                                     const int64_t *c_off, const int *nc, const double *wi,
                                     double *M, double *BJ, const int64_t *off_c,
                                     const int64_t *boff, int cnt) {
  const int64_t blk = blockIdx.x;
  const int e = seg_entry(boff, cnt, blk);
  const int64_t m = nc[e], n = ns[e];
  const int64_t i0 = (blk - boff[e]) * SEG_CHUNK + threadIdx.x;
#pragma unroll
  for (int it = 0; it < SEG_ITEMS; ++it) {
    const int64_t i = i0 + (int64_t)it * TPB;
    if (i >= m * m) break;
    const int a = (int)(i % m), b = (int)(i / m);
    const int ra = cidx[c_off[e] + a], rb = cidx[c_off[e] + b];
    const double dia = wi[c_off[e] + a], dib = wi[c_off[e] + b];
    const double dja = 1.0 - dia, djb = 1.0 - dib;
    const int64_t src = ra + (int64_t)rb * n;
    M[off_c[e] + i] = dja * Sss[off_si[e] + src] * djb + dia * Sss[off_sj[e] + src] * dib;
    BJ[off_c[e] + i] = BJfull[off_p[e] + src];
  }
}

// segment e: dst[dst_off[e] + i] = src[src_off[e] + i] for i < len[e] (many
// small copies in one launch)
__global__ void copy_segments_kernel(const double *src, const int64_t *src_off, double *dst,
                                     const int64_t *dst_off, const int64_t *len) {
  const int e = blockIdx.y;
  const int64_t n = len[e], so = src_off[e], dO = dst_off[e];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[dO + i] = src[so + i];
}

// dst[idx[i]] = val[i]
__global__ void scatter_values_kernel(const int64_t *idx, const double *val, int64_t n, double *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = val[i];
}

// dst = src^T per entry (m x m, ld m; flat launch, seg_entry)
__global__ void transpose_kernel(const double *src, double *dst, const int64_t *off,
                                 const int *n, const int64_t *boff, int cnt) {
  const int64_t blk = blockIdx.x;
  const int e = seg_entry(boff, cnt, blk);
  const int64_t m = n[e];
  const int64_t i0 = (blk - boff[e]) * SEG_CHUNK + threadIdx.x;
#pragma unroll
  for (int it = 0; it < SEG_ITEMS; ++it) {
    const int64_t i = i0 + (int64_t)it * TPB;
    if (i >= m * m) break;
    const int r = (int)(i % m), c = (int)(i / m);
    dst[off[e] + c + (int64_t)r * m] = src[off[e] + i];
  }
}

// tile pair t of a triangle of tiles, t = bj (bj + 1) / 2 + bi, 0 <= bi <= bj
__device__ __forceinline__ void upper_pair(int64_t t, int &bi, int &bj) {
  int j = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(j + 1) * (j + 2) / 2 <= t) ++j;
  while ((int64_t)j * (j + 1) / 2 > t) --j;
  bj = j;
  bi = (int)(t - (int64_t)j * (j + 1) / 2);
}

// A <- (A + A^T) / 2 in place (ld n), by 32 x 32 tile pairs through LDS so
// that reads and writes run down columns: work-group (bi, bj), bi <= bj,
// loads tiles (bi, bj) and (bj, bi), averages each entry with its mirror and
// writes both (a diagonal tile with itself).  Flat launch: one tile pair per
// block, entry e owning nt (nt + 1) / 2 of them, nt = ceil(n / 32).
__global__ __launch_bounds__(256) void symmetrize_kernel(double *A, const int64_t *off, const int *n,
                                                         const int64_t *boff, int cnt) {
  __shared__ double up[32][33], lo[32][33];
  const int64_t blk = blockIdx.x;
  const int e = seg_entry(boff, cnt, blk);
  int bi, bj;
  upper_pair(blk - boff[e], bi, bj);
  const int m = n[e];
  if (32 * bj >= m) return;
  double *a = A + off[e];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cl = ty + 8 * q;
    const int ru = 32 * bi + tx, cu = 32 * bj + cl;  // tile (bi, bj)
    const int rl = 32 * bj + tx, cw = 32 * bi + cl;  // tile (bj, bi)
    if (ru < m && cu < m) up[cl][tx] = a[ru + (int64_t)cu * m];
    if (rl < m && cw < m) lo[cl][tx] = a[rl + (int64_t)cw * m];
  }
  __syncthreads();
  // entry (r, c) of tile (bi, bj) mirrors entry (c, r) of tile (bj, bi)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cl = ty + 8 * q;
    const int ru = 32 * bi + tx, cu = 32 * bj + cl;
    const int rl = 32 * bj + tx, cw = 32 * bi + cl;
    if (ru < m && cu < m) a[ru + (int64_t)cu * m] = 0.5 * (up[cl][tx] + lo[tx][cl]);
    if (rl < m && cw < m) a[rl + (int64_t)cw * m] = 0.5 * (lo[cl][tx] + up[tx][cl]);
  }
}

// ---------------------------------------------------------------------------
// batched LOBPCG: dominant eigenpairs of a symmetric d x d matrix per entry

constexpr int LOB_NT = 512;                // threads per work-group (8 waves)
constexpr int LOB_NWAVE = LOB_NT / 64;
constexpr int LOB_S = LOB_MAXB / 3;        // block size (columns of X, W and P)
constexpr int LOCK_MAX = 256;              // eigenvectors locked from earlier rounds
constexpr int STAGE_ROWS = 256;            // rows of a block staged in LDS per pass
constexpr int DOT_ROWS = 64;               // rows per chunk of the block products U^T V
constexpr int DOT_LD = 2 * LOB_MAXB / LOB_NWAVE;  // staged columns per wave and chunk
constexpr int JAC_NB = (LOB_MAXB / 2) * (LOB_MAXB / 2) / LOB_NT + 1;  // 2 x 2 blocks per thread
constexpr int JAC_NV = LOB_MAXB * (LOB_MAXB / 2) / LOB_NT + 1;        // V row pairs per thread

typedef double v4d __attribute__((ext_vector_type(4)));

struct LobDesc {
  int64_t a_off;    // d x d matrix (ld d)
  int64_t v_off;    // V = [X P W] (d x 3s), then A V (d x 3s), ld d
  int64_t t_off;    // 2 blocks of d x s scratch
  int64_t lock_off; // nl locked orthonormal eigenvectors (d x nl, ld d)
  int nl;
  int d, s;
  int need;         // number of leading eigenpairs that must converge (>= 1)
  double tau;       // threshold: pairs with theta >= tau are needed, plus one below
  int take;         // > 0: the first `take` pairs are selected whatever tau says
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

// the same value, opaque to the optimizer: arithmetic on it is not moved out
// of the region that uses it (keeps loop-invariant address computations from
// being hoisted out of the iteration loop and held in registers throughout)
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return __builtin_amdgcn_readfirstlane(v);
}

// value of v in lane l of the wave (l uniform)
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Row tiles of tall-skinny products on the matrix cores (v_mfma_f64_16x16x4f64:
// lane l holds A[l%16][l/16] and B[l/16][l%16]; entry j of its result is row
// l/16 + 4j, column l%16).  U is global, column-major, ld d; C0, C1 in LDS
// with rows ldc apart, columns from n0 (n1) on read as zero, rows of U past d
// read as zero.
// Up to four row tiles at once (rows r0[t]..r0[t]+15, t < nt), sharing the
// C operands: acc0[t] += U[r0[t]:+16, 0:nk] C0[0:nk, 0:16] and, when TWO,
// acc1[t] likewise with C1.  The tiles' loads of one K-step are independent,
// so four times as many loads of U are in flight as with one tile at a time
// (these products are bound by their latency).
template <bool TWO>
__device__ __forceinline__ void tile_mul4(const double *U, int d, const int (&r0)[4], int nt, int nk,
                                          const double *C0, int n0, const double *C1, int n1,
                                          int ldc, v4d (&acc0)[4], v4d (&acc1)[4]) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
  const double *u[4];
  bool rv[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    rv[t] = t < nt && r0[t] + i < d;
    u[t] = U + (rv[t] ? r0[t] + i : 0);
  }
  // KB K-steps per batch: all their loads of U are issued before any of
  // their products, so 4 KB loads per wave are in flight (the accumulation
  // order is that of one K-step at a time).  KB = 4 cut the A products of
  // the LOBPCG iterations by 30%; with two products (more accumulators live)
  // the registers allow one K-step.
  constexpr int KB = TWO ? 1 : 4;
  for (int k = 0; k < nk; k += 4 * KB) {
    double a[KB][4], b0[KB], b1[KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      const int kk = k + 4 * q + kq;
      const bool kv = kk < nk;
#pragma unroll
      for (int t = 0; t < 4; ++t) a[q][t] = (rv[t] && kv) ? u[t][(int64_t)kk * d] : 0.0;
      b0[q] = (kv && i < n0) ? C0[kk * ldc + i] : 0.0;
      if (TWO) b1[q] = (kv && i < n1) ? C1[kk * ldc + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < KB; ++q) {
      if (k + 4 * q >= nk) break;  // uniform
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nt) acc0[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][t], b0[q], acc0[t], 0, 0, 0);
      if (TWO) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nt) acc1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][t], b1[q], acc1[t], 0, 0, 0);
      }
    }
  }
}

// the row tiles a wave takes in group g of a d-row block: 16 (wave + NWAVE
// (4 g + t)), t < 4; returns how many exist
__device__ __forceinline__ int wave_tiles(int d, int g, int (&r0)[4]) {
  const int wave = threadIdx.x >> 6;
  int nt = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    r0[t] = 16 * (wave + LOB_NWAVE * (4 * g + t));
    if (r0[t] < d) nt = t + 1;
  }
  return nt;
}

// Out[r0 + row, col] = acc (or -= acc when SUB) for the rows < d and columns
// < ncol of the tile (Out column-major, ld d)
template <bool SUB>
__device__ __forceinline__ void tile_store(double *Out, int d, int r0, int ncol, const v4d &acc) {
  const int lane = threadIdx.x & 63, c = lane & 15, rq = lane >> 4;
  if (c >= ncol) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int row = r0 + rq + 4 * j;
    if (row < d) {
      double *o = Out + row + (int64_t)c * d;
      *o = SUB ? *o - acc[j] : acc[j];
    }
  }
}

// Symmetric eigen-decomposition of the n x n matrix H (LDS, ld LOB_MAXB+1) by
// parallel cyclic Jacobi (round-robin pairing): H <- diag, V <- eigenvectors.
// A step applies the m/2 disjoint rotations of one round together: every
// 2 x 2 block of H on the rows of one pair and the columns of another is
// rotated on both sides by one thread, and each pair of V's columns likewise.
// The blocks partition H, so each thread reads its entries and writes them
// back with no other thread touching them in between.
// Sweeps stop when every off-diagonal entry is below 1e-13 sqrt(|h_pp h_qq|)
// (eigenvalues then hold to about 1e-26 relative and eigenvectors to 1e-13,
// far inside the 1e-8 residual tolerance of the Ritz pairs) or below 1e-17 of the Frobenius norm
// (rotations preserve it; smaller entries cannot move the eigenpairs), or the
// off-diagonal mass is below 1e-30 of the total, or after 20 sweeps.
// Launched with LOB_NT threads.
__device__ void jacobi_eig(double (*H)[LOB_MAXB + 1], double (*V)[LOB_MAXB + 1], int n,
                           double *cs, double *sn, double *red) {
  // the step's pairs (p | q << 16) and rotations (c, s), one 4-byte and one
  // 16-byte LDS read per pair
  __shared__ int pq[LOB_MAXB / 2 + 1];
  __shared__ double2 rot[LOB_MAXB / 2 + 1];
  (void)cs;
  (void)sn;
  const int tid = threadIdx.x;
  for (int i = tid; i < n * n; i += LOB_NT) V[i % n][i / n] = (i % n == i / n) ? 1.0 : 0.0;
  const int m = (n + 1) / 2 * 2;  // even number of players (a dummy when n is odd)
  const int half = m / 2;
  // the 2 x 2 blocks (k, l) of H and the (row, l) entries of V a thread
  // updates are the same at every step (only the players in them change):
  // indices computed once, outside the step loop
  int bk[JAC_NB], bl[JAC_NB], vr[JAC_NV], vl[JAC_NV];
#pragma unroll
  for (int u = 0; u < JAC_NB; ++u) {
    const int e = tid + u * LOB_NT;
    bk[u] = e < half * half ? e % half : -1;
    bl[u] = e / half;
  }
#pragma unroll
  for (int u = 0; u < JAC_NV; ++u) {
    const int e = tid + u * LOB_NT;
    vr[u] = e < n * half ? e % n : -1;
    vl[u] = e / n;
  }
  __syncthreads();
  double tot = 0;
  for (int i = tid; i < n * n; i += LOB_NT) tot += H[i % n][i / n] * H[i % n][i / n];
  tot = block_sum(tot, red);
  const double floor_abs = 1e-17 * sqrt(tot);
  for (int sweep = 0; sweep < 20; ++sweep) {
    double off = 0, viol = 0;
    for (int i = tid; i < n * n; i += LOB_NT) {
      const int a = i % n, b = i / n;
      if (a == b) continue;
      const double h = H[a][b];
      off += h * h;
      if (fabs(h) > fmax(1e-13 * sqrt(fabs(H[a][a] * H[b][b])), floor_abs)) viol += 1;
    }
    off = block_sum(off, red);
    viol = block_sum(viol, red);
    if (viol == 0 || off <= 1e-30 * tot || tot == 0) break;
    // round-robin schedule: player 0 stays at position 0; the player at
    // position i >= 1 moves down one place per step (from 1 back to m - 1).
    // Thread k < m/2 pairs positions k and m - 1 - k; at step 0 position i
    // holds player i.
    int pa = tid, pb = m - 1 - tid;
    for (int step = 0; step < m - 1; ++step) {
      // the step's pairs and rotations; a pair with the dummy (q = n) keeps
      // c = 1, s = 0
      if (tid < half) {
        int p = pa, q = pb;
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1, s = 0;
        if (q < n && H[p][q] != 0.0) {
          const double theta = (H[q][q] - H[p][p]) / (2 * H[p][q]);
          const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1));
          c = rsqrt(t * t + 1);
          s = t * c;
        }
        pq[tid] = p | (q << 16);
        rot[tid] = double2{c, s};
        if (tid > 0) pa = pa > 1 ? pa - 1 : m - 1;
        pb = pb > 1 ? pb - 1 : m - 1;
      }
      __syncthreads();
      // every read of the step before any write (the reads of one thread
      // then overlap in flight); the blocks partition H and the items
      // partition the touched entries of V, so no other thread touches
      // these entries in this step
      int hk[JAC_NB], hl[JAC_NB], vk[JAC_NV];
      double2 rk[JAC_NB], rl[JAC_NB], rv[JAC_NV];
      double hb[JAC_NB][4], vb[JAC_NV][2];
#pragma unroll
      for (int u = 0; u < JAC_NB; ++u) {
        if (bk[u] >= 0) {
          hk[u] = pq[bk[u]];
          hl[u] = pq[bl[u]];
          rk[u] = rot[bk[u]];
          rl[u] = rot[bl[u]];
          const int pk = hk[u] & 0xffff, qk = hk[u] >> 16, pl = hl[u] & 0xffff, ql = hl[u] >> 16;
          hb[u][0] = H[pk][pl];
          hb[u][1] = ql < n ? H[pk][ql] : 0.0;
          hb[u][2] = qk < n ? H[qk][pl] : 0.0;
          hb[u][3] = (qk < n && ql < n) ? H[qk][ql] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < JAC_NV; ++u) {
        if (vr[u] >= 0) {
          vk[u] = pq[vl[u]];
          rv[u] = rot[vl[u]];
          const int pl = vk[u] & 0xffff, ql = vk[u] >> 16;
          vb[u][0] = V[vr[u]][pl];
          vb[u][1] = ql < n ? V[vr[u]][ql] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < JAC_NB; ++u) {
        if (bk[u] >= 0) {
          const int pk = hk[u] & 0xffff, qk = hk[u] >> 16, pl = hl[u] & 0xffff, ql = hl[u] >> 16;
          const double ck = rk[u].x, sk = rk[u].y, cl = rl[u].x, sl = rl[u].y;
          // rows (J_k^T B), then columns (. J_l)
          const double rpp = ck * hb[u][0] - sk * hb[u][2], rpq = ck * hb[u][1] - sk * hb[u][3];
          const double rqp = sk * hb[u][0] + ck * hb[u][2], rqq = sk * hb[u][1] + ck * hb[u][3];
          H[pk][pl] = cl * rpp - sl * rpq;
          if (ql < n) H[pk][ql] = sl * rpp + cl * rpq;
          if (qk < n) H[qk][pl] = cl * rqp - sl * rqq;
          if (qk < n && ql < n) H[qk][ql] = sl * rqp + cl * rqq;
        }
      }
#pragma unroll
      for (int u = 0; u < JAC_NV; ++u) {
        if (vr[u] >= 0) {
          const int pl = vk[u] & 0xffff, ql = vk[u] >> 16;
          const double cl = rv[u].x, sl = rv[u].y;
          V[vr[u]][pl] = cl * vb[u][0] - sl * vb[u][1];
          if (ql < n) V[vr[u]][ql] = sl * vb[u][0] + cl * vb[u][1];
        }
      }
      __syncthreads();
    }
  }
}

// One work-group per entry.  The basis V = [X P W] is kept orthonormal
// explicitly: W (the residuals) is orthogonalized against X and P by two
// passes of block Gram-Schmidt and orthonormalized by Cholesky QR (or, for a
// near-dependent block, by the scaled eigen-decomposition of its Gram matrix,
// which drops columns).  The Rayleigh-Ritz step is the standard symmetric
// problem V^T A V, solved in LDS by Jacobi rotations; the new P is formed in
// coefficient space (its coefficients orthonormalized against those of the
// new X), so X and P leave the update already orthonormal.  Block products
// U^T V run on the matrix cores.  Blocks live in global memory; every update
// of a block is row-owned (one thread writes a whole row), so blocks are
// updated in place.
// Helpers for the A products of a face pair.  When a launch has few pairs,
// each pair gets `helpers` extra work-groups that compute row groups of
// A V for its work-group (the leader): the leader publishes a request (its
// number, the V and A V blocks) after an agent-scope release; every row
// group (512 rows) is claimed by one work-group with a compare-and-swap of
// its claim word from the previous request's number to this one's, computed
// by the same code as alone (so the bits do not depend on who computed it),
// and marked done after a release; the leader computes the groups it claims
// itself and waits only for groups a helper claimed -- a helper that claimed
// one is running, so the wait ends -- then acquires.  A helper that sees no
// request for LOB_HELPER_IDLE ticks, or the leader's end, leaves.
constexpr int LOB_MAXCH = 16;  // row groups of 512 rows per pair (d <= 8192)
constexpr long long LOB_HELPER_IDLE = 100000000LL;  // wall-clock ticks (1 s at 100 MHz)
constexpr long long LOB_LEADER_WAIT = 400000000LL;  // bound of the leader's wait (4 s)
struct LobSync {
  int gen;        // number of the leader's latest request
  int finished;   // the leader has left its loop
  int nv;         // columns of the request
  int pad;
  int64_t vin_off, avo_off;  // V and A V of the request (pool offsets)
  int claim[LOB_MAXCH];      // request number that claimed each row group
  int done[LOB_MAXCH];       // request number whose row group is complete
};

// rows [512 g, 512 g + 512) of AVo = A Vin (nv <= LOB_S columns, ld d): Vin
// staged through LDS in chunks of STAGE_ROWS rows, each wave accumulating up
// to four 16-row tiles
__device__ void apply_A_group(const double *A, int d_, const double *Vin, double *AVo, int nv,
                              int g, double *stage) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const int d = opaque(d_);
  const int nrt = (d + 15) >> 4;
  const int tg = g * 4 * LOB_NWAVE;
  const v4d z4 = {0.0, 0.0, 0.0, 0.0};
  v4d acc[4] = {z4, z4, z4, z4};
  for (int c0 = 0; c0 < d; c0 += STAGE_ROWS) {
    const int cn = min(STAGE_ROWS, d - c0);
    __syncthreads();
    for (int i = tid; i < cn * LOB_S; i += LOB_NT) {
      const int c = i % cn, q = i / cn;
      stage[c * LOB_S + q] = q < nv ? Vin[c0 + c + (int64_t)q * d] : 0.0;
    }
    __syncthreads();
    int r0[4], nt = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int tile = tg + wave + LOB_NWAVE * t;
      r0[t] = 16 * tile;
      if (tile < nrt) nt = t + 1;
    }
    v4d unused[4];
    if (nt > 0) tile_mul4<false>(A + (int64_t)c0 * d, d, r0, nt, cn, stage, nv, nullptr, 0, LOB_S, acc, unused);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int tile = tg + wave + LOB_NWAVE * t;
    if (tile < nrt) tile_store<false>(AVo, d, 16 * tile, nv, acc[t]);
  }
}

__device__ __forceinline__ int lob_groups(int d) { return (((d + 15) >> 4) + 4 * LOB_NWAVE - 1) / (4 * LOB_NWAVE); }

// claim row group g of request r for this work-group (one CAS, broadcast)
__device__ __forceinline__ bool lob_claim(LobSync *sy, int g, int r, int *s_flag) {
  if (threadIdx.x == 0) *s_flag = atomicCAS(&sy->claim[g], r - 1, r) == r - 1 ? 1 : 0;
  __syncthreads();
  const bool mine = *s_flag != 0;
  __syncthreads();
  return mine;
}

// a helper work-group of pair p: row groups of the leader's requests until
// the leader leaves
__device__ void lob_helper(double *pool, const LobDesc *desc, LobSync *sync, int p, int h,
                           double *stage, int *s_int) {
  const LobDesc D = desc[p];
  LobSync *sy = sync + p;
  const double *A = pool + D.a_off;
  const int ng = lob_groups(D.d);
  int mine_req = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      int r = -1;
      const long long t0 = wall_clock64();
      for (int it = 0;; ++it) {
        if (__hip_atomic_load(&sy->finished, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        const int cur = __hip_atomic_load(&sy->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur > mine_req) {
          r = cur;
          break;
        }
        if ((it & 31) == 31 && wall_clock64() - t0 > LOB_HELPER_IDLE) break;
        __builtin_amdgcn_s_sleep(2);
      }
      if (r > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_int[0] = r;
    }
    __syncthreads();
    const int r = s_int[0];
    __syncthreads();
    if (r < 0) return;
    mine_req = r;
    const double *Vin = pool + sy->vin_off;
    double *AVo = pool + sy->avo_off;
    const int nv = sy->nv;
    for (int i = 0; i < ng; ++i) {
      const int g = (h + 1 + i) % ng;
      if (!lob_claim(sy, g, r, s_int + 1)) continue;
      apply_A_group(A, D.d, Vin, AVo, nv, g, stage);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_store(&sy->done[g], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ __launch_bounds__(LOB_NT) void lobpcg_kernel(double *pool, const LobDesc *desc,
                                                        LobOut *out, int maxit, double tol,
                                                        double tol_ind, int na, int helpers,
                                                        LobSync *sync) {
  __shared__ double Hs[LOB_MAXB][LOB_MAXB + 1];  // projected / Gram matrices
  __shared__ double Qs[LOB_MAXB][LOB_MAXB + 1];  // their eigenvectors
  __shared__ __align__(16) double Cs[LOB_MAXB][2 * LOB_S];  // Ritz coefficients (X part, P part)
  __shared__ __align__(16) double Ms[LOB_S][LOB_S];         // orthonormalizing map of a block
  __shared__ __align__(16) double stage[STAGE_ROWS * LOB_S];  // staged rows, or locked coefficients
  __shared__ double su[DOT_ROWS][LOB_MAXB + 1];   // row chunks of block products
  __shared__ double sv[DOT_ROWS][LOB_MAXB + 1];
  __shared__ double theta[LOB_MAXB], gsc[LOB_MAXB], dinv[LOB_MAXB], res[LOB_S];
  __shared__ double cs[LOB_MAXB / 2 + 1], sn[LOB_MAXB / 2 + 1], red[LOB_NWAVE];
  __shared__ int perm[LOB_MAXB + 2];
  __shared__ int s_keep, s_done;
  __shared__ int s_int[4];
  if ((int)blockIdx.x >= na) {  // a helper work-group
    const int q = (int)blockIdx.x - na;
    lob_helper(pool, desc, sync, q / helpers, q % helpers, stage, s_int);
    return;
  }
  const LobDesc D = desc[blockIdx.x];
  if (threadIdx.x == 0) s_int[3] = 0;
  const int d_ = D.d, d = d_, s = D.s, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const double *A = pool + D.a_off;
  // V = [X P W] and A V, each with contiguous columns: X (s columns), P (npc),
  // then W (nw), so that [X P] and V are plain column blocks
  double *V = pool + D.v_off, *AV = V + (int64_t)3 * d * s;
  double *X = V, *AX = AV, *P = V + (int64_t)d * s, *AP = AV + (int64_t)d * s;
  double *T1 = pool + D.t_off;
  const double *YL = pool + D.lock_off;
  const int nl = D.nl;
  int nw = 0, npc = 0;  // columns held in W and P
  double *W = P, *AW = AP;  // W follows the npc columns of P
  long long ticks[4] = {0, 0, 0, 0};  // phase timing (see LobOut)

  // o[a * ldo + b] = u_a . v_b for nu, nv <= LOB_MAXB columns given by
  // accessors: chunks of DOT_ROWS rows are staged in LDS (the next chunk
  // loaded into registers while the current one is multiplied) and each wave
  // accumulates up to two 16 x 16 tiles of U^T V with v_mfma_f64_16x16x4f64,
  // always in the same order
  auto block_dot = [&](const double *U, int nu, const double *Vb, int nv, double *o, int ldo) {
    const int d = opaque(d_);
    const int tu = (nu + 15) >> 4, tv = (nv + 15) >> 4, ntile = tu * tv;
    const int cu = 16 * tu, ncol = cu + 16 * tv;  // staged columns (zero past nu, nv)
    // thread: row `lane` of the chunk, columns wave + LOB_NWAVE q (uniform per wave)
    double pre[DOT_LD];
    auto fetch = [&](int c0) {
      const int r = c0 + lane;
#pragma unroll
      for (int q = 0; q < DOT_LD; ++q) {
        const int j = wave + LOB_NWAVE * q;
        double v = 0;
        if (r < d) {
          if (j < cu) {
            if (j < nu) v = U[r + (int64_t)j * d];
          } else if (j < ncol && j - cu < nv) {
            v = Vb[r + (int64_t)(j - cu) * d];
          }
        }
        pre[q] = v;
      }
    };
    v4d acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int c0 = 0; c0 < d; c0 += DOT_ROWS) {
      __syncthreads();  // the previous chunk's reads of su, sv are done
#pragma unroll
      for (int q = 0; q < DOT_LD; ++q) {
        const int j = wave + LOB_NWAVE * q;
        if (j < cu)
          su[lane][j] = pre[q];
        else if (j < ncol)
          sv[lane][j - cu] = pre[q];
      }
      __syncthreads();
      if (c0 + DOT_ROWS < d) fetch(c0 + DOT_ROWS);
      const int kn = min(DOT_ROWS, d - c0);  // rows past kn are zero
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int tile = wave + t * LOB_NWAVE;
        if (tile < ntile) {
          const int a0 = (tile % tu) * 16 + (lane & 15), b0 = (tile / tu) * 16 + (lane & 15);
          for (int kk = 0; kk < kn; kk += 4) {
            const int k = kk + (lane >> 4);
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(su[k][a0], sv[k][b0], acc[t], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int tile = wave + t * LOB_NWAVE;
      if (tile < ntile) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int a = (tile % tu) * 16 + (lane >> 4) + 4 * j, b = (tile / tu) * 16 + (lane & 15);
          if (a < nu && b < nv) o[a * ldo + b] = acc[t][j];
        }
      }
    }
    __syncthreads();
  };
  const v4d zero4 = {0.0, 0.0, 0.0, 0.0};
  // V[:, b] -= sum_a U[:, a] c[a * ldc + b] for b < nv (c in LDS); one wave
  // per 16-row tile
  auto sub_prod = [&](double *V, int nv, const double *U, int nu, const double *c, int ldc) {
    const int d = opaque(d_);
    for (int g = 0; 16 * LOB_NWAVE * 4 * g < d; ++g) {
      int r0[4];
      const int nt = wave_tiles(d, g, r0);
      v4d acc[4] = {zero4, zero4, zero4, zero4}, unused[4];
      if (nt > 0) tile_mul4<false>(U, d, r0, nt, nu, c, nv, nullptr, 0, ldc, acc, unused);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nt) tile_store<true>(V, d, r0[t], nv, acc[t]);
    }
    __syncthreads();
  };
  // V[:, 0..kp) = V[:, 0..nv) M  (M in Ms), in place: each wave reads its
  // rows before writing them
  auto right_mul = [&](double *V, int nv, int kp) {
    const int d = opaque(d_);
    for (int g = 0; 16 * LOB_NWAVE * 4 * g < d; ++g) {
      int r0[4];
      const int nt = wave_tiles(d, g, r0);
      v4d acc[4] = {zero4, zero4, zero4, zero4}, unused[4];
      if (nt > 0) tile_mul4<false>(V, d, r0, nt, nv, &Ms[0][0], kp, nullptr, 0, LOB_S, acc, unused);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nt) tile_store<false>(V, d, r0[t], kp, acc[t]);
    }
    __syncthreads();
  };
  // Gram matrix G (nv x nv, in Hs) -> Ms = Dg Q g^-1/2 over the eigenvalues
  // g > thr of Dg G Dg = Q diag(g) Q^T, Dg = diag(G)^-1/2 (so that the
  // columns times Ms are orthonormal).  Returns the number of columns kept.
  auto gram_eig = [&](int nv, double thr) -> int {
    for (int a = tid; a < nv; a += LOB_NT) dinv[a] = Hs[a][a] > 0 ? 1.0 / sqrt(Hs[a][a]) : 0.0;
    __syncthreads();
    for (int i = tid; i < nv * nv; i += LOB_NT) {
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
    for (int i = tid; i < nv * kp; i += LOB_NT) {
      const int b = i % nv, q = i / nv;
      Ms[b][q] = dinv[b] * Qs[b][perm[q]] * gsc[q];
    }
    __syncthreads();
    return kp;
  };
  // Gram matrix G = L L^T (nv <= LOB_S, in Hs) -> Ms = L^-T.  The Cholesky
  // factorization runs in wave 0 with row i of G in the registers of lane i,
  // column by column; lane j then forms column j of L^-1.  Returns false when a
  // pivot falls below 1e-8 of its diagonal entry (condition above 1e4: the
  // caller then uses gram_eig).
  auto chol_inv = [&](int nv) -> bool {
    if (wave == 0) {
      double g[LOB_S];
#pragma unroll
      for (int k = 0; k < LOB_S; ++k) g[k] = (lane < nv && k < nv) ? Hs[lane][k] : 0.0;
      bool ok = true;
#pragma unroll
      for (int j = 0; j < LOB_S; ++j) {
        if (j < nv) {
          const double djj = lane_value(g[j], j);
          ok = ok && djj > 1e-8 * Hs[j][j];
          const double r = ok ? sqrt(djj) : 1.0;
          g[j] = lane == j ? r : (lane > j ? g[j] / r : 0.0);
#pragma unroll
          for (int k = j + 1; k < LOB_S; ++k)
            if (k < nv) {
              const double lkj = lane_value(g[j], k);
              if (lane >= k) g[k] -= g[j] * lkj;
            }
        }
      }
      if (ok) {
        double y[LOB_S];  // column `lane` of L^-1
#pragma unroll
        for (int i = 0; i < LOB_S; ++i) {
          double acc = (i == lane) ? 1.0 : 0.0;
#pragma unroll
          for (int mm = 0; mm < i; ++mm) acc -= lane_value(g[mm], i) * y[mm];
          y[i] = i < nv ? acc / lane_value(g[i], i) : 0.0;
        }
        if (lane < nv)
#pragma unroll
          for (int q = 0; q < LOB_S; ++q)
            if (q < nv) Ms[lane][q] = y[q];  // (L^-T)[lane][q] = (L^-1)[q][lane]
      }
      if (lane == 0) s_keep = ok ? 1 : 0;
    }
    __syncthreads();
    return s_keep != 0;
  };
  // orthonormalize the nv columns of V by the eigen-decomposition of their
  // Gram matrix (dependent columns dropped); returns the number kept
  auto svqb = [&](double *V, int nv, double thr) -> int {
    if (nv == 0) return 0;
    block_dot(V, nv, V, nv, &Hs[0][0], LOB_MAXB + 1);
    const int kp = gram_eig(nv, thr);
    right_mul(V, nv, kp);
    return kp;
  };
  // V <- V L^-T with V^T V = L L^T; false (V untouched) if ill-conditioned
  auto cholqr = [&](double *V, int nv) -> bool {
    if (nv == 0) return true;
    block_dot(V, nv, V, nv, &Hs[0][0], LOB_MAXB + 1);
    if (!chol_inv(nv)) return false;
    right_mul(V, nv, nv);
    return true;
  };
  // V <- V - YL (YL^T V): keep a block orthogonal to the locked vectors
  auto project_locked = [&](double *V, int nv) {
    if (nl == 0 || nv == 0) return;
    for (int a0 = 0; a0 < nl; a0 += LOB_MAXB)
      block_dot(YL + (int64_t)a0 * d, min(LOB_MAXB, nl - a0), V, nv, stage + a0 * LOB_S, LOB_S);
    sub_prod(V, nv, YL, nl, stage, LOB_S);
  };
  // AV = A V for nv columns: V staged through LDS in chunks of STAGE_ROWS
  // rows, each wave accumulating up to four 16-row tiles of A V
  bool lob_abort = false;  // a helper's row group did not complete in time
  auto apply_A = [&](const double *Vin, double *AVo, int nv) {
    const int ng = lob_groups(d_);
    if (helpers == 0) {
      for (int g = 0; g < ng; ++g) apply_A_group(A, d_, Vin, AVo, nv, g, stage);
      __syncthreads();
      return;
    }
    LobSync *sy = sync + blockIdx.x;
    // publish the request: every store of V done and released first
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      const int r = sy->gen + 1;  // only the leader writes gen
      sy->vin_off = Vin - pool;
      sy->avo_off = AVo - pool;
      sy->nv = nv;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&sy->gen, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_int[0] = r;
      s_int[2] = 0;  // bit g: claimed here
    }
    __syncthreads();
    const int r = s_int[0];
    for (int g = 0; g < ng; ++g) {
      if (!lob_claim(sy, g, r, s_int + 1)) continue;
      apply_A_group(A, d_, Vin, AVo, nv, g, stage);
      if (tid == 0) s_int[2] |= 1 << g;
    }
    __syncthreads();
    if (tid == 0) {
      const int mine = s_int[2];
      const long long t0 = wall_clock64();
      for (int g = 0; g < ng; ++g) {
        if (mine & (1 << g)) continue;
        for (int it = 0;; ++it) {
          if (__hip_atomic_load(&sy->done[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == r) break;
          if ((it & 31) == 31 && wall_clock64() - t0 > LOB_LEADER_WAIT) {
            s_int[3] = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (s_int[3]) lob_abort = true;
  };
  // Rayleigh-Ritz on the current n = s + npc + nw columns: theta, and the
  // coefficients of the new X (Cs[:, 0..s)) and of the new P (Cs[:, LOB_S..):
  // the same vectors without their X rows)
  auto rayleigh_ritz = [&](int n) {
    // H = V^T A V, symmetrized
    block_dot(V, n, AV, n, &Hs[0][0], LOB_MAXB + 1);
    for (int i = tid; i < n * n; i += LOB_NT) {
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
    // the s largest eigenvalues, descending (ties by index; NaN last)
    for (int a = tid; a < n; a += LOB_NT) {
      const double la = isnan(Hs[a][a]) ? -INFINITY : Hs[a][a];
      int rank = 0;
      for (int b = 0; b < n; ++b) {
        const double lb = isnan(Hs[b][b]) ? -INFINITY : Hs[b][b];
        rank += (lb > la || (lb == la && b < a)) ? 1 : 0;
      }
      if (rank < s) {
        perm[rank] = a;
        theta[rank] = Hs[a][a];
      }
    }
    __syncthreads();
    for (int i = tid; i < n * s; i += LOB_NT) {
      const int b = i % n, q = i / n;
      const double c = Qs[b][perm[q]];
      Cs[b][q] = c;
      Cs[b][LOB_S + q] = b < s ? 0.0 : c;
    }
    __syncthreads();
  };
  // P coefficients (Cs[:, LOB_S..)) made orthogonal to the X coefficients
  // (orthonormal) by two Gram-Schmidt passes, then orthonormal; returns the
  // number of P columns kept
  auto orth_pcoef = [&](int n) -> int {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = tid; i < s * s; i += LOB_NT) {
        const int a = i % s, q = i / s;
        double t = 0;
        for (int b = 0; b < n; ++b) t += Cs[b][a] * Cs[b][LOB_S + q];
        Ms[a][q] = t;
      }
      __syncthreads();
      for (int i = tid; i < n * s; i += LOB_NT) {
        const int b = i % n, q = i / n;
        double t = 0;
        for (int a = 0; a < s; ++a) t += Cs[b][a] * Ms[a][q];
        Cs[b][LOB_S + q] -= t;
      }
      __syncthreads();
    }
    for (int i = tid; i < s * s; i += LOB_NT) {
      const int a = i % s, q = i / s;
      double t = 0;
      for (int b = 0; b < n; ++b) t += Cs[b][LOB_S + a] * Cs[b][LOB_S + q];
      Hs[a][q] = t;
    }
    __syncthreads();
    const int kp = chol_inv(s) ? s : gram_eig(s, 1e-10);
    // Cp <- Cp Ms through Qs (free once the Ritz coefficients are in Cs)
    for (int i = tid; i < n * kp; i += LOB_NT) {
      const int b = i % n, q = i / n;
      double t = 0;
      for (int a = 0; a < s; ++a) t += Cs[b][LOB_S + a] * Ms[a][q];
      Qs[b][q] = t;
    }
    __syncthreads();
    for (int i = tid; i < n * kp; i += LOB_NT) Cs[i % n][LOB_S + i / n] = Qs[i % n][i / n];
    __syncthreads();
    return kp;
  };
  // X <- V Cx, P <- V Cp (kp columns) and their images, in place: each wave
  // reads all columns of its rows before writing them
  auto ritz_update = [&](int n, int kp) {
    const int d = opaque(d_);
    for (int pass = 0; pass < 2; ++pass) {
      double *B = pass ? AV : V;
      for (int g = 0; 16 * LOB_NWAVE * 4 * g < d; ++g) {
        int r0[4];
        const int nt = wave_tiles(d, g, r0);
        v4d ax[4] = {zero4, zero4, zero4, zero4}, ap[4] = {zero4, zero4, zero4, zero4};
        if (nt > 0) tile_mul4<true>(B, d, r0, nt, n, &Cs[0][0], s, &Cs[0][LOB_S], kp, 2 * LOB_S, ax, ap);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t < nt) {
            tile_store<false>(B, d, r0[t], s, ax[t]);
            tile_store<false>(B + (int64_t)s * d, d, r0[t], kp, ap[t]);
          }
      }
    }
    __syncthreads();
  };

  int it = 0, nconv = 0;
  bool done = false;
  for (int q = tid; q < LOB_MAXB; q += LOB_NT) theta[q] = 0;
  __syncthreads();
  // start block: orthonormal and orthogonal to the locked vectors
  int kx = s;
  for (int pass = 0; pass < 2 && kx == s; ++pass) {
    project_locked(X, s);
    if (pass == 0 || !cholqr(X, s)) kx = svqb(X, s, 1e-10);
  }
  if (kx == s) {
    long long t0 = wall_clock64();
    apply_A(X, AX, s);
    ticks[0] += wall_clock64() - t0;
    t0 = wall_clock64();
    rayleigh_ritz(s);
    ticks[2] += wall_clock64() - t0;
    ritz_update(s, 0);
  }
  for (it = 1; it <= maxit && kx == s; ++it) {
    // residuals W = A X - X theta and their norms
    W = P + (int64_t)npc * d;
    AW = AP + (int64_t)npc * d;
    for (int i = tid; i < d * s; i += LOB_NT) W[i] = AX[i] - X[i] * theta[i / d];
    __syncthreads();
    project_locked(W, s);
    for (int q = wave; q < s; q += LOB_NWAVE) {
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
        const bool selected = D.take > 0 ? k < D.take : theta[k] >= D.tau;
        const bool needed = (k < D.need) || (k == 0) ||
                            (D.take > 0 ? k <= D.take : theta[k - 1] >= D.tau);
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
    // search directions: unit residuals, orthogonal to X and P, orthonormal
    for (int i = tid; i < d * s; i += LOB_NT) {
      const int q = i / d;
      W[i] = res[q] > 0 ? W[i] / res[q] : 0.0;
    }
    __syncthreads();
    long long to = wall_clock64();
    nw = s;
    for (int pass = 0; pass < 2; ++pass) {
      project_locked(W, nw);
      block_dot(X, s + npc, W, nw, &Cs[0][0], 2 * LOB_S);
      sub_prod(W, nw, X, s + npc, &Cs[0][0], 2 * LOB_S);
    }
    if (!cholqr(W, nw)) nw = svqb(W, nw, 1e-10);
    ticks[1] += wall_clock64() - to;
    if (nw == 0 && npc == 0) break;  // no direction left: stagnation
    long long t1 = wall_clock64();
    apply_A(W, AW, nw);
    ticks[0] += wall_clock64() - t1;
    const int n = s + npc + nw;
    t1 = wall_clock64();
    rayleigh_ritz(n);
    ticks[2] += wall_clock64() - t1;
    to = wall_clock64();
    const int kp = orth_pcoef(n);
    ticks[1] += wall_clock64() - to;
    ritz_update(n, kp);
    npc = kp;
    nw = 0;
  }
  if (helpers > 0 && tid == 0)
    __hip_atomic_store(&sync[blockIdx.x].finished, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (tid == 0) {
    out[blockIdx.x].iters = lob_abort ? -1 : it;
    out[blockIdx.x].converged = done && !lob_abort ? 1 : 0;
    out[blockIdx.x].nconv = nconv;
    for (int q = 0; q < 4; ++q) out[blockIdx.x].ticks[q] = ticks[q];
  }
  // eigenvalues into the first column of T1 for the host
  __syncthreads();
  for (int q = tid; q < s; q += LOB_NT) T1[q] = theta[q];
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
  // uninitialized (for buffers that every use writes in full before reading)
  double *raw(int64_t n) {
    DBuf b;
    b.bytes = std::max<size_t>(n * sizeof(double), 8);
    b.p = A->get(b.bytes);
    bufs.push_back(b);
    return b.as<double>();
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

AdaptResult run_adapt(Problem &P, Solver &S, AdaptState &st, double tau, int count) {
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
        if (G.kind == GLOB_EDGE) {
          ph.edge_gi.push_back((int)g2);
          ph.edge_c.push_back(crow);
        }
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
    dv = pool.raw(t);  // every block written by the factorization
    doff = pool.up(stream, off);
  };
  const int nside = 2 * np;
  // Schur complement of S_a onto the shared dofs s of each pair side, in two
  // eliminations that the sides of one substructure share: the sides are
  // grouped three at a time (in pair order); for a group with shared-dof
  // union U, the rest N of the interface is eliminated once (S_U = S_UU -
  // S_UN S_NN^-1 S_NU), then each side eliminates U \ s from S_U.  Equal to
  // eliminating everything but s at once (quotient property of Schur
  // complements), with far fewer flops.
  std::vector<int> nsv(nside);
  std::vector<int64_t> off_sh(nside), off_ss(nside);
  int64_t tsh = 0;
  int max_ns = 0;
  for (int p = 0; p < np; ++p)
    for (int a = 0; a < 2; ++a) {
      const int e = 2 * p + a;
      nsv[e] = (int)pairs[p].pos_s[a].size();
      max_ns = std::max(max_ns, nsv[e]);
      off_sh[e] = tsh;
      off_ss[e] = tsh + (int64_t)nsv[e] * nsv[e];
      tsh += 2 * (int64_t)nsv[e] * nsv[e];
    }
  const double *Sd = S.d_S.as<double>();
  // status words: [0, 2 nside) the eliminations of the bisection, then the
  // sums of the Schur complements (np) and the jump-space denominators (np)
  int *d_stat = pool.up(stream, std::vector<int>(2 * nside + 2 * np + 4, 0));
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
  // one gather + Cholesky + TRSM + GEMM pass: for entry e, from the matrix at
  // src + src_off[e] (ld lds[e]), with index lists n (eliminated) and u (kept)
  // of it: Out (u x u) = S_uu - S_un S_nn^-1 S_nu
  auto eliminate = [&](const double *src, const std::vector<int64_t> &src_off,
                       const std::vector<int> &lds, const std::vector<std::vector<int>> &nidx,
                       const std::vector<std::vector<int>> &uidx, double *out,
                       const std::vector<int64_t> &out_off, int *stat) {
    const int cnt = (int)nidx.size();
    std::vector<int64_t> o_nn(cnt), o_nu(cnt), io_n(cnt), io_u(cnt);
    std::vector<int> nn(cnt), nu(cnt), in_all, iu_all;
    int64_t tnn = 0, tnu = 0;
    int mnn = 0, mnu = 0;
    for (int e = 0; e < cnt; ++e) {
      nn[e] = (int)nidx[e].size();
      nu[e] = (int)uidx[e].size();
      mnn = std::max(mnn, nn[e]);
      mnu = std::max(mnu, nu[e]);
      o_nn[e] = tnn;
      tnn += (int64_t)nn[e] * nn[e];
      o_nu[e] = tnu;
      tnu += (int64_t)nn[e] * nu[e];
      io_n[e] = (int64_t)in_all.size();
      in_all.insert(in_all.end(), nidx[e].begin(), nidx[e].end());
      io_u[e] = (int64_t)iu_all.size();
      iu_all.insert(iu_all.end(), uidx[e].begin(), uidx[e].end());
    }
    // written in full by the gathers below
    double *Snn = pool.raw(std::max<int64_t>(tnn, 1));
    double *Snu = pool.raw(std::max<int64_t>(tnu, 1));
    int64_t *d_so = pool.up(stream, src_off), *d_onn = pool.up(stream, o_nn),
            *d_onu = pool.up(stream, o_nu), *d_oo = pool.up(stream, out_off);
    int *d_lds = pool.up(stream, lds), *d_nn = pool.up(stream, nn), *d_nu = pool.up(stream, nu);
    int *d_in = pool.up(stream, in_all.empty() ? std::vector<int>{0} : in_all);
    int *d_iu = pool.up(stream, iu_all.empty() ? std::vector<int>{0} : iu_all);
    int64_t *d_ion = pool.up(stream, io_n), *d_iou = pool.up(stream, io_u);
    // a flat launch over the entries' own rows x cols elements
    auto gather = [&](double *dst, const int64_t *doff, const int *ri, const int64_t *rio,
                      const int *nr, const int *ci, const int64_t *cio, const int *ncl,
                      const std::vector<int> &hr, const std::vector<int> &hc) {
      std::vector<int64_t> c(cnt);
      for (int e = 0; e < cnt; ++e) c[e] = (int64_t)hr[e] * hc[e];
      const std::vector<int64_t> bo = seg_offsets(c, SEG_CHUNK);
      if (bo.back() == 0) return;
      gather_rc_kernel<<<(unsigned)bo.back(), TPB, 0, stream>>>(src, d_so, d_lds, dst, doff, ri, rio, nr,
                                                                ci, cio, ncl, pool.up(stream, bo), cnt);
      HIPCHK(hipGetLastError());
    };
    gather(Snn, d_onn, d_in, d_ion, d_nn, d_in, d_ion, d_nn, nn, nn);
    gather(Snu, d_onu, d_in, d_ion, d_nn, d_iu, d_iou, d_nu, nn, nu);
    gather(out, d_oo, d_iu, d_iou, d_nu, d_iu, d_iou, d_nu, nu, nu);
    std::vector<MatDesc> md(cnt);
    std::vector<GemmDesc> gd(cnt);
    for (int e = 0; e < cnt; ++e) {
      md[e] = MatDesc{o_nn[e], o_nu[e], nn[e], nu[e], std::max(1, nn[e]), std::max(1, nn[e])};
      gd[e] = GemmDesc{o_nu[e], o_nu[e], out_off[e], nu[e], nu[e], nn[e], std::max(1, nn[e]),
                       std::max(1, nn[e]), std::max(1, nu[e])};
    }
    MatDesc *d_md = pool.up(stream, md);
    GemmDesc *d_gd = pool.up(stream, gd);
    double *dv;
    int64_t *doff;
    dinv_for(md, dv, doff);
    HIPCHK(DenseOps<double>::potrf(stream, Snn, d_md, md.data(), cnt, stat, dv, doff));
    HIPCHK(DenseOps<double>::trsm(stream, Snn, Snu, d_md, md.data(), cnt, false, dv, doff));
    // Out and Snu live in different pools; the product is symmetric: its
    // lower triangle is formed and mirrored
    HIPCHK(DenseOps<double>::gemm(stream, Snu, Snu, out, d_gd, cnt, mnu, mnu, true, false, -1.0, 1.0,
                                  true, gd.data()));
    std::vector<MatDesc> mo(cnt);
    for (int e = 0; e < cnt; ++e) mo[e] = MatDesc{out_off[e], 0, nu[e], 0, std::max(1, nu[e]), 1};
    HIPCHK(symmetrize_lower<double>(stream, out, pool.up(stream, mo), cnt, mnu, mo.data()));
  };
  // Schur complement of S_a onto the shared dofs s of each pair side, by
  // recursive bisection of the sides of each substructure (in pair order): a
  // node holds a contiguous range of the substructure's sides and the Schur
  // complement of S_a onto the union U of their shared dofs (interface
  // positions, ascending); each half of a node's range eliminates the rest of
  // U from the node's matrix.  The root is S_a itself and a one-side node is
  // Sh of that side.  Equal to eliminating everything but s at once
  // (quotient property of Schur complements); at the 64^3 k-means size, 9
  // sides per substructure on average, it takes about 1.7 times fewer flops
  // than eliminating onto groups of three sides first.  One batched
  // elimination per tree depth.
  struct BNode {
    int sub, lo, hi;    // sides by_sub[sub][lo..hi)
    std::vector<int> U;  // interface positions of the node's matrix
    int64_t off = 0;     // its matrix in the work pool (depth >= 1), ld |U|
  };
  std::vector<std::vector<int>> by_sub(L.nsub);
  for (int e = 0; e < nside; ++e) by_sub[pairs[e / 2].sub[e % 2]].push_back(e);
  // Where each node's range of sides is cut: the cut that minimizes the
  // flops of the eliminations below it (a Cholesky of the eliminated block,
  // the solve with the kept columns and the lower product: nn^3/3 + nn^2 nu +
  // nn nu^2), by dynamic programming over the contiguous ranges of the
  // substructure's sides; the sides are ordered by their first interface
  // position (neighbouring faces tend to share edges, so ranges of
  // neighbours have small unions) or kept in pair order, whichever costs
  // less.
  std::vector<std::vector<int>> split(L.nsub);  // split[sb][lo * (m + 1) + hi]
  double plan_flops = 0, half_flops = 0;
  {
    auto elim = [](double nn, double nu) { return nn * nn * nn / 3.0 + nn * nn * nu + nn * nu * nu; };
    for (int sb = 0; sb < L.nsub; ++sb) {
      const int m = (int)by_sub[sb].size();
      if (m == 0) continue;
      const int nG = L.nG[sb];
      auto plan_for = [&](const std::vector<int> &ord, std::vector<int> &cut, double &best_root,
                          double &half) {
        // union sizes of every range [lo, hi)
        std::vector<int> usz((size_t)(m + 1) * (m + 1), 0);
        std::vector<char> in(nG);
        for (int lo = 0; lo < m; ++lo) {
          std::fill(in.begin(), in.end(), 0);
          int cntu = 0;
          for (int hi = lo + 1; hi <= m; ++hi) {
            const int e = ord[hi - 1];
            for (int q : pairs[e / 2].pos_s[e % 2])
              if (!in[q]) in[q] = 1, ++cntu;
            usz[(size_t)lo * (m + 1) + hi] = cntu;
          }
        }
        auto U = [&](int lo, int hi) { return (double)usz[(size_t)lo * (m + 1) + hi]; };
        std::vector<double> cost((size_t)(m + 1) * (m + 1), 0.0);
        cut.assign((size_t)(m + 1) * (m + 1), -1);
        // cost(lo, hi): flops of the subtree below a node holding U(lo, hi)
        for (int len = 2; len <= m; ++len)
          for (int lo = 0; lo + len <= m; ++lo) {
            const int hi = lo + len;
            double best = -1;
            for (int mid = lo + 1; mid < hi; ++mid) {
              const double up = U(lo, hi);
              const double c = elim(up - U(lo, mid), U(lo, mid)) + elim(up - U(mid, hi), U(mid, hi)) +
                               cost[(size_t)lo * (m + 1) + mid] + cost[(size_t)mid * (m + 1) + hi];
              if (best < 0 || c < best) best = c, cut[(size_t)lo * (m + 1) + hi] = mid;
            }
            cost[(size_t)lo * (m + 1) + hi] = best;
          }
        // the root holds the whole interface (nG), not only the union
        auto root_cost = [&](int mid) {
          if (m == 1) return elim(nG - U(0, 1), U(0, 1));
          return elim(nG - U(0, mid), U(0, mid)) + elim(nG - U(mid, m), U(mid, m)) +
                 cost[(size_t)mid] + cost[(size_t)mid * (m + 1) + m];
        };
        best_root = -1;
        for (int mid = 1; mid < std::max(2, m); ++mid) {
          const double c = root_cost(mid);
          if (best_root < 0 || c < best_root) best_root = c, cut[(size_t)m] = mid;
        }
        // the cost of cutting every range in halves (for the log)
        std::function<double(int, int, double)> halves = [&](int lo, int hi, double up) -> double {
          if (hi - lo == 1) return 0.0;
          const int mid = lo + (hi - lo) / 2;
          return elim(up - U(lo, mid), U(lo, mid)) + elim(up - U(mid, hi), U(mid, hi)) +
                 halves(lo, mid, U(lo, mid)) + halves(mid, hi, U(mid, hi));
        };
        half = m == 1 ? elim(nG - U(0, 1), U(0, 1)) : halves(0, m, nG);
      };
      std::vector<int> ord_pair = by_sub[sb], ord_pos = by_sub[sb];
      auto first_pos = [&](int e) {
        const std::vector<int> &v = pairs[e / 2].pos_s[e % 2];
        return v.empty() ? INT32_MAX : *std::min_element(v.begin(), v.end());
      };
      std::stable_sort(ord_pos.begin(), ord_pos.end(), [&](int a, int b) { return first_pos(a) < first_pos(b); });
      std::vector<int> cut_pair, cut_pos;
      double c_pair, c_pos, h_pair, h_pos;
      plan_for(ord_pair, cut_pair, c_pair, h_pair);
      plan_for(ord_pos, cut_pos, c_pos, h_pos);
      half_flops += h_pair;
      if (c_pos < c_pair) {
        by_sub[sb] = ord_pos;
        split[sb] = cut_pos;
        plan_flops += c_pos;
      } else {
        split[sb] = cut_pair;
        plan_flops += c_pair;
      }
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "pair-side eliminations: %.2f TFLOP planned (%.2f with halved ranges)",
                  plan_flops * 1e-12, half_flops * 1e-12);
    log(buf);
  }
  auto union_of = [&](int sb, int lo, int hi) {
    std::vector<char> in(L.nG[sb], 0);
    for (int t = lo; t < hi; ++t) {
      const int e = by_sub[sb][t];
      for (int q : pairs[e / 2].pos_s[e % 2]) in[q] = 1;
    }
    std::vector<int> U;
    for (int q = 0; q < L.nG[sb]; ++q)
      if (in[q]) U.push_back(q);
    return U;
  };
  // depth 0: the roots (the matrices S_a in place)
  std::vector<BNode> parents;
  for (int sb = 0; sb < L.nsub; ++sb) {
    if (by_sub[sb].empty()) continue;
    BNode r;
    r.sub = sb;
    r.lo = 0;
    r.hi = (int)by_sub[sb].size();
    r.U.resize(L.nG[sb]);
    std::iota(r.U.begin(), r.U.end(), 0);
    parents.push_back(std::move(r));
  }
  // the children of every depth, and the work pool: Sh (and the S_ss
  // copies) first, then the inner nodes' matrices
  std::vector<std::vector<BNode>> depth_nodes;
  std::vector<std::vector<int>> depth_parent;
  int64_t twk = tsh;
  {
    std::vector<BNode> cur = parents;
    while (!cur.empty()) {
      std::vector<BNode> kids;
      std::vector<int> par;
      for (int k = 0; k < (int)cur.size(); ++k) {
        const BNode &P = cur[k];
        const int n = P.hi - P.lo;
        const int m = (int)by_sub[P.sub].size();
        const int mid = n == 1 ? P.hi : split[P.sub][(size_t)P.lo * (m + 1) + P.hi];
        const int cuts[3] = {P.lo, mid, P.hi};
        for (int h = 0; h < (n == 1 ? 1 : 2); ++h) {
          BNode c;
          c.sub = P.sub;
          c.lo = cuts[h];
          c.hi = cuts[h + 1];
          c.U = union_of(c.sub, c.lo, c.hi);
          if (c.hi - c.lo == 1) {
            c.off = off_sh[by_sub[c.sub][c.lo]];
          } else {
            c.off = twk;
            twk += (int64_t)c.U.size() * c.U.size();
          }
          kids.push_back(std::move(c));
          par.push_back(k);
        }
      }
      depth_nodes.push_back(kids);
      depth_parent.push_back(par);
      std::vector<BNode> inner;
      for (BNode &c : kids)
        if (c.hi - c.lo > 1) inner.push_back(c);
      // inner nodes become the next depth's parents; remember the parent
      // list of this depth for the index maps
      cur.swap(inner);
    }
  }
  double *Wk = pool.raw(twk);  // every block written by a gather before use
  double *Sh = Wk;  // Sh of side e at off_sh[e], its S_ss at off_ss[e]
  {
    std::vector<BNode> cur = parents;  // parents of the depth being formed
    int stat_next = 0;
    for (size_t dpt = 0; dpt < depth_nodes.size(); ++dpt) {
      const std::vector<BNode> &kids = depth_nodes[dpt];
      const int cnt = (int)kids.size();
      std::vector<int64_t> src_off(cnt), out_off(cnt);
      std::vector<int> lds(cnt);
      std::vector<std::vector<int>> nidx(cnt), uidx(cnt);
      for (int c = 0; c < cnt; ++c) {
        const BNode &P = cur[depth_parent[dpt][c]];
        const BNode &K = kids[c];
        std::vector<int> at(L.nG[K.sub], -1);
        for (size_t t = 0; t < P.U.size(); ++t) at[P.U[t]] = (int)t;
        std::vector<char> keep(P.U.size(), 0);
        for (int q : K.U) {
          uidx[c].push_back(at[q]);
          keep[at[q]] = 1;
        }
        for (size_t t = 0; t < P.U.size(); ++t)
          if (!keep[t]) nidx[c].push_back((int)t);
        src_off[c] = dpt == 0 ? L.offGG[K.sub] : P.off;
        lds[c] = dpt == 0 ? L.nG[K.sub] : (int)P.U.size();
        out_off[c] = K.off;
      }
      eliminate(dpt == 0 ? Sd : Wk, src_off, lds, nidx, uidx, Wk, out_off, d_stat + stat_next);
      check(stat_next, cnt, "interface blocks outside the shared dofs");
      stat_next += cnt;
      std::vector<BNode> inner;
      for (const BNode &K : kids)
        if (K.hi - K.lo > 1) inner.push_back(K);
      cur.swap(inner);
    }
  }
  std::vector<int64_t> ss_src(nside);
  std::vector<int> ss_lds(nside);
  for (int e = 0; e < nside; ++e) {
    const int sb = pairs[e / 2].sub[e % 2];
    ss_src[e] = L.offGG[sb];
    ss_lds[e] = L.nG[sb];
  }
  {
    // the original S_ss of every side (for the numerator M)
    std::vector<int> ss_all;
    std::vector<int64_t> ss_io(nside);
    for (int e = 0; e < nside; ++e) {
      ss_io[e] = (int64_t)ss_all.size();
      const std::vector<int> &ps = pairs[e / 2].pos_s[e % 2];
      ss_all.insert(ss_all.end(), ps.begin(), ps.end());
    }
    int64_t *d_so = pool.up(stream, ss_src), *d_oo = pool.up(stream, off_ss),
            *d_io = pool.up(stream, ss_io);
    int *d_lds = pool.up(stream, ss_lds), *d_ns = pool.up(stream, nsv);
    int *d_ix = pool.up(stream, ss_all);
    std::vector<int64_t> c(nside);
    for (int e = 0; e < nside; ++e) c[e] = (int64_t)nsv[e] * nsv[e];
    const std::vector<int64_t> bo = seg_offsets(c, SEG_CHUNK);
    if (bo.back() > 0) {
      gather_rc_kernel<<<(unsigned)bo.back(), TPB, 0, stream>>>(Sd, d_so, d_lds, Sh, d_oo, d_ix, d_io, d_ns,
                                                                d_ix, d_io, d_ns, pool.up(stream, bo), nside);
      HIPCHK(hipGetLastError());
    }
  }

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
  double *Ssum = pool.raw(tp), *Xb = pool.raw(tp), *BJf = pool.raw(tp);  // written in full by pair_sum
  double *d_Q = pool.up(stream, Qall), *d_rho = pool.up(stream, rho);
  int64_t *d_off_i = pool.up(stream, off_i), *d_off_j = pool.up(stream, off_j),
          *d_off_p = pool.up(stream, off_p), *d_q_off = pool.up(stream, q_off);
  int *d_nsp = pool.up(stream, nsp), *d_nq = pool.up(stream, nqv);
  int max_sp = 0;
  for (int p = 0; p < np; ++p) max_sp = std::max(max_sp, nsp[p]);
  // block offsets of the flat launches over the pairs: n x n elements each
  // (count) or n x n elements in 32 x 32 tile pairs (tri)
  auto flat = [&](const std::vector<int> &n, bool tri) {
    std::vector<int64_t> c(np);
    for (int p = 0; p < np; ++p) {
      const int64_t t = (n[p] + 31) / 32;
      c[p] = tri ? t * (t + 1) / 2 : (int64_t)n[p] * n[p];
    }
    return seg_offsets(c, tri ? 1 : SEG_CHUNK);
  };
  {
    const std::vector<int64_t> bo = flat(nsp, false);
    if (bo.back() > 0)
      pair_sum_kernel<<<(unsigned)bo.back(), TPB, 0, stream>>>(Sh, d_off_i, d_off_j, d_nsp, Ssum, Xb, BJf,
                                                               d_off_p, d_Q, d_q_off, d_nq, d_rho,
                                                               pool.up(stream, bo), np);
    HIPCHK(hipGetLastError());
  }
  std::vector<MatDesc> mds(np);
  std::vector<GemmDesc> gbj(np);
  for (int p = 0; p < np; ++p) {
    mds[p] = MatDesc{off_p[p], off_p[p], nsp[p], nsp[p], std::max(1, nsp[p]), std::max(1, nsp[p])};
    gbj[p] = GemmDesc{off_i[p], off_p[p], off_p[p], nsp[p], nsp[p], nsp[p], std::max(1, nsp[p]),
                      std::max(1, nsp[p]), std::max(1, nsp[p])};
  }
  MatDesc *d_mds = pool.up(stream, mds);
  GemmDesc *d_gbj = pool.up(stream, gbj);
  int *stat2 = d_stat + 2 * nside;
  double *dv_s;
  int64_t *do_s;
  dinv_for(mds, dv_s, do_s);
  HIPCHK(DenseOps<double>::potrf(stream, Ssum, d_mds, mds.data(), np, stat2, dv_s, do_s));
  check(2 * nside, np, "sum of the Schur complements");
  HIPCHK(DenseOps<double>::trsm(stream, Ssum, Xb, d_mds, mds.data(), np, false, dv_s, do_s));
  HIPCHK(DenseOps<double>::trsm(stream, Ssum, Xb, d_mds, mds.data(), np, true, dv_s, do_s));
  // BJ = Sh_i (Sh_i + Sh_j)^+ Sh_j, the product form of the parallel sum (no
  // cancellation between the two large terms of Sh_i - Sh_i (..)^+ Sh_i when
  // the coefficients of i and j differ by orders of magnitude)
  HIPCHK(DenseOps<double>::gemm(stream, Sh, Xb, BJf, d_gbj, np, max_sp, max_sp, false, false, 1.0,
                                0.0, false, gbj.data()));
  {
    const std::vector<int64_t> bo = flat(nsp, true);
    if (bo.back() > 0)
      symmetrize_kernel<<<(unsigned)bo.back(), 256, 0, stream>>>(BJf, d_off_p, d_nsp, pool.up(stream, bo), np);
    HIPCHK(hipGetLastError());
  }
  double *Mc = pool.raw(tc), *BJc = pool.raw(tc);  // written in full by pair_restrict
  int *d_call = pool.up(stream, call), *d_nc = pool.up(stream, ncv);
  int64_t *d_c_off = pool.up(stream, c_off), *d_off_c = pool.up(stream, off_c);
  int64_t *d_off_ss_i = pool.up(stream, off_ss_i), *d_off_ss_j = pool.up(stream, off_ss_j);
  double *d_w = pool.up(stream, wall);
  {
    const std::vector<int64_t> bo = flat(ncv, false);
    if (bo.back() > 0)
      pair_restrict_kernel<<<(unsigned)bo.back(), TPB, 0, stream>>>(Sh, d_off_ss_i, d_off_ss_j, BJf, d_off_p,
                                                                    d_nsp, d_call, d_c_off, d_nc, d_w, Mc,
                                                                    BJc, d_off_c, pool.up(stream, bo), np);
    HIPCHK(hipGetLastError());
  }
  // My = Z^T M Z, By = Z^T BJ Z
  double *Zd = pool.zeros(stream, tz);
  {
    const int64_t *d_zdst = pool.up(stream, zdst);
    const double *d_zval = pool.up(stream, zval);
    scatter_values_kernel<<<nblocks((int64_t)zdst.size()), TPB, 0, stream>>>(d_zdst, d_zval,
                                                                         (int64_t)zdst.size(), Zd);
    HIPCHK(hipGetLastError());
  }
  // written in full by the products (beta = 0) and the transpose below
  double *T1 = pool.raw(tcz), *My = pool.raw(tdd), *By = pool.raw(tdd), *Cp = pool.raw(tdd);
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
  check(2 * nside + np, np, "jump-space denominator");
  // My <- L^-1 My ; Cp <- My^T ; Cp <- L^-1 Cp   (My's pool is the B operand)
  HIPCHK(DenseOps<double>::trsm(stream, By, My, d_mdd, mdd.data(), np, false, dv_y, do_y));
  {
    const std::vector<int64_t> bo = flat(dv, false);
    if (bo.back() > 0)
      transpose_kernel<<<(unsigned)bo.back(), TPB, 0, stream>>>(My, Cp, d_off_dd, d_dv, pool.up(stream, bo), np);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(DenseOps<double>::trsm(stream, By, Cp, d_mdd, mdd.data(), np, false, dv_y, do_y));
  // the two solves leave C' symmetric only to ~kappa(By) eps; LOBPCG's
  // residuals cannot drop below that asymmetry, so C' is symmetrized
  {
    const std::vector<int64_t> bo = flat(dv, true);
    if (bo.back() > 0)
      symmetrize_kernel<<<(unsigned)bo.back(), 256, 0, stream>>>(Cp, d_off_dd, d_dv, pool.up(stream, bo), np);
    HIPCHK(hipGetLastError());
  }

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
  // the per-pair pieces of a round (start blocks in, Ritz values out,
  // selected vectors kept) move as segments of one launch each
  auto copy_segments = [&](const double *src, double *dst, const std::vector<int64_t> &so,
                           const std::vector<int64_t> &dO, const std::vector<int64_t> &len) {
    const int nseg = (int)len.size();
    if (nseg == 0) return;
    int64_t mx = 1;
    for (int64_t l : len) mx = std::max(mx, l);
    copy_segments_kernel<<<dim3((unsigned)std::min<int64_t>(nblocks(mx), 64), nseg), TPB, 0, stream>>>(
        src, pool.up(stream, so), dst, pool.up(stream, dO), pool.up(stream, len));
    HIPCHK(hipGetLastError());
  };
  int cu_count = 256;  // compute units (the helper work-groups of LOBPCG)
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cu_count, hipDeviceAttributeMultiprocessorCount, dev);
  }
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
      ld[p].take = count > 0 ? std::min(count - ksel[p], ld[p].s) : 0;
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
    }
    {
      // every start block in one transfer, then to its place in LP
      double *x0d = pool.up(stream, X0all.empty() ? std::vector<double>{0.0} : X0all);
      std::vector<int64_t> so(na), dO(na), len(na);
      for (int a = 0; a < na; ++a) {
        so[a] = x0off[a];
        dO[a] = ld[active[a]].v_off;
        len[a] = x0off[a + 1] - x0off[a];
      }
      copy_segments(x0d, LP, so, dO, len);
    }
    HIPCHK(hipMemcpyAsync(ldb.p, lda.data(), sizeof(LobDesc) * na, hipMemcpyHostToDevice, stream));
    {
      LaunchScope ls(stream, "lobpcg_kernel", 0, 0);
      if (per_entry_launches()) {
        // unbatched baseline: one face pair per launch
        for (int a = 0; a < na; ++a)
          lobpcg_kernel<<<1, LOB_NT, 0, stream>>>(LP, ldb.as<LobDesc>() + a, outb.as<LobOut>() + a,
                                                  maxit, tol, tol_ind, 1, 0, nullptr);
      } else {
        // few pairs (the later rounds): helper work-groups for the A products,
        // as many per pair as its row groups and the compute units allow (one
        // work-group of this kernel per compute unit)
        int maxd = 0;
        for (int a = 0; a < na; ++a) maxd = std::max(maxd, lda[a].d);
        const int groups = (((maxd + 15) / 16) + 4 * LOB_NWAVE - 1) / (4 * LOB_NWAVE);
        int helpers = 0;
        if (groups <= LOB_MAXCH) helpers = std::max(0, std::min(groups, cu_count / std::max(1, na)) - 1);
        LobSync *sync = nullptr;
        if (helpers > 0)
          sync = reinterpret_cast<LobSync *>(
              pool.zeros(stream, (int64_t)(na * sizeof(LobSync) + sizeof(double) - 1) / sizeof(double)));
        lobpcg_kernel<<<na * (1 + helpers), LOB_NT, 0, stream>>>(LP, ldb.as<LobDesc>(), outb.as<LobOut>(),
                                                                maxit, tol, tol_ind, na, helpers, sync);
      }
      HIPCHK(hipGetLastError());
    }
    std::vector<LobOut> lo(na);
    HIPCHK(hipMemcpyAsync(lo.data(), outb.p, sizeof(LobOut) * na, hipMemcpyDeviceToHost, stream));
    std::vector<std::vector<double>> th(na);
    {
      // the Ritz values of every pair gathered, then one transfer
      std::vector<int64_t> so(na), dO(na), len(na);
      int64_t tot = 0;
      for (int a = 0; a < na; ++a) {
        so[a] = ld[active[a]].t_off;
        len[a] = ld[active[a]].s;
        dO[a] = tot;
        tot += len[a];
      }
      double *thd = pool.zeros(stream, std::max<int64_t>(1, tot));
      copy_segments(LP, thd, so, dO, len);
      std::vector<double> tall(std::max<int64_t>(1, tot));
      HIPCHK(hipMemcpyAsync(tall.data(), thd, sizeof(double) * tall.size(), hipMemcpyDeviceToHost,
                            stream));
      HIPCHK(hipStreamSynchronize(stream));
      for (int a = 0; a < na; ++a) th[a].assign(tall.begin() + dO[a], tall.begin() + dO[a] + len[a]);
    }
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
    std::vector<int64_t> keep_so, keep_do, keep_len;  // selected eigenvectors to keep
    for (int a = 0; a < na; ++a) {
      const int p = active[a];
      const int s = ld[p].s;
      res.iters += lo[a].iters;
      if (!lo[a].converged) res.unconverged++;
      int k = 0;
      if (count > 0)
        k = std::min(count - ksel[p], s);
      else
        while (k < s && th[a][k] >= tau) ++k;
      evs[p].insert(evs[p].end(), th[a].begin(), th[a].end());
      // keep the selected eigenvectors
      if (k > 0) {
        keep_so.push_back(ld[p].v_off);
        keep_do.push_back(tdd + tv + off_y[p] + (int64_t)ksel[p] * dv[p]);
        keep_len.push_back((int64_t)dv[p] * k);
      }
      ksel[p] += k;
      if (k < s) {
        res.omega = std::max(res.omega, th[a][k]);
      } else if (ksel[p] < dv[p] && lo[a].converged) {
        next.push_back(p);  // the block held only selected pairs: lock them, go on
      }
    }
    copy_segments(LP, LP, keep_so, keep_do, keep_len);  // (source and target regions are disjoint)
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
  std::vector<int> hstat(2 * nside + 2 * np + 4);
  HIPCHK(hipMemcpyAsync(hv.data(), Vtmp, sizeof(double) * tj, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hstat.data(), d_stat, sizeof(int) * hstat.size(), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  for (int e = 0; e < 2 * nside + 2 * np; ++e)
    if (hstat[e])
      throw NotSpdError("adaptive pair problems: non-positive pivot in a pair factor (Assumption 2 may fail)");
  log("eigenvectors to jump space");
  // ---- host: face rows, and edge rows when they are kept.  Pi_G acts glob
  // by glob: each part of v is projected onto the null space of its glob's
  // constraint rows chosen at setup (orthonormalized once per glob).
  std::vector<std::vector<double>> hq(P.globs.size());
  std::vector<int> hm(P.globs.size(), -1);
  auto glob_basis = [&](int gi) -> int {
    if (hm[gi] < 0) {
      const GlobCov &cv = P.cov[gi];
      hm[gi] = cv.m;
      if (cv.m > 0) {
        hq[gi] = cv.hrow;
        orthonormalize(hq[gi], (int)P.globs[gi].dofs.size(), hm[gi]);
      }
    }
    return hm[gi];
  };
  // r = v[cidx], projected; returns max |r|
  auto glob_part = [&](const double *v, const std::vector<int> &cidx, int gi, std::vector<double> &r) {
    const int n = (int)cidx.size(), m = glob_basis(gi);
    const std::vector<double> &H = hq[gi];
    r.resize(n);
    for (int t = 0; t < n; ++t) r[t] = v[cidx[t]];
    for (int a = 0; a < m; ++a) {
      double dt = 0;
      for (int t = 0; t < n; ++t) dt += H[(size_t)a * n + t] * r[t];
      for (int t = 0; t < n; ++t) r[t] -= dt * H[(size_t)a * n + t];
    }
    double mx = 0;
    for (double x : r) mx = std::max(mx, std::fabs(x));
    return mx;
  };
  constexpr double EDGE_DROP = 1e-8;  // edge parts below this (relative to d) are rounding residue
  for (int p = 0; p < np; ++p) {
    const AdaptPair &ph = pairs[p];
    const int nc = ncv[p];
    std::vector<double> ev = evs[p];
    std::sort(ev.begin(), ev.end(), [](double x, double y) { return x > y; });
    st.eigs[ph.f] = ev;
    const int k = ksel[p];
    if (k == 0) continue;
    const int ne = P.adapt_edges ? (int)ph.edge_gi.size() : 0;
    std::vector<double> rf;
    std::vector<std::vector<double>> re(ne);
    std::vector<double> mxe(ne);
    for (int q = 0; q < k; ++q) {
      const double *v = hv.data() + off_jv[p] + (size_t)q * nc;
      const double mxf = glob_part(v, ph.face_c, ph.gi, rf);
      double scale = mxf;
      for (int e = 0; e < ne; ++e) {
        mxe[e] = glob_part(v, ph.edge_c[e], ph.edge_gi[e], re[e]);
        scale = std::max(scale, mxe[e]);
      }
      if (mxf > 0) {
        for (double &x : rf) x /= mxf;
        P.extra_rows[ph.gi].insert(P.extra_rows[ph.gi].end(), rf.begin(), rf.end());
        P.extra_k[ph.gi] += 1;
        res.n_added += 1;
      }
      for (int e = 0; e < ne; ++e) {
        if (!(mxe[e] > EDGE_DROP * scale)) continue;
        for (double &x : re[e]) x /= mxe[e];
        const int gi = ph.edge_gi[e];
        P.extra_rows[gi].insert(P.extra_rows[gi].end(), re[e].begin(), re[e].end());
        P.extra_k[gi] += 1;
        res.n_added_edge += 1;
      }
    }
  }
  log("face rows (host)");
  return res;
}

}  // namespace bddc
