// BDDC on the device: factorization of every substructure (batched), the
// preconditioner application and PCG on the reduced (interface) problem.
//
// Formulation.  The preconditioner is Algorithm 2 (Sec. 5).  Following the
// Remark after Algorithm 2 the explicit (average) variables produced by the
// change of variables are assembled like corners ("primal"), which gives the
// same operator as the projected system with Pibar and t (the projection
// averages the copies of every explicit variable).  Because (I - P) discards
// interior values and the residuals of the reduced problem vanish in the
// interiors (Remark after Lemma 1), every substructure problem is condensed
// onto its interface with the Schur complement S_i = A_GG - A_GI A_II^-1 A_IG:
//
//   factor:  A_II = L L^T (Cholesky),  Y = L^-1 A_IG,  S_i = A_GG - Y^T Y,
//            Sbar_i = T_i^T S_i T_i,   split into r (remaining) and pi
//            (corners and explicit averages) dofs,
//            Sbar_rr = Lr Lr^T,  Phi_i = -Sbar_rr^-1 Sbar_rpi,
//            S_pi^i = Sbar_pipi + Sbar_pir Phi_i,  S_c = sum R_pi^T S_pi R_pi,
//            S_c = Lc Lc^T.
//   apply:   b = T^T (delta . r_i) ;  y_r = Sbar_rr^-1 b_r ;
//            x_c = S_c^-1 sum R_pi^T (b_pi + Phi^T b_r) ;
//            x_r = y_r + Phi x_pi ;  z = sum_i R_i^T delta_i T_i x_i,
//            then (I - P): z_I = -A_II^-1 A_IG z_G per substructure.
//   PCG:     on interface vectors with q = sum R_i^T S_i R_i p; the interior
//            values of the solution are recovered at the end by one Dirichlet
//            solve per substructure.
#include <hip/hip_runtime.h>

#include <limits>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "device.h"
#include "solver.h"

namespace bddc {

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));             \
  } while (0)

void *DevAlloc::get(size_t bytes) {
  if (bytes == 0) return nullptr;
  void *p = nullptr;
  if (alloc) {
    p = alloc(bytes, user);
    if (!p) throw OomError("device allocation of " + std::to_string(bytes) + " bytes failed");
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw OomError("hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  held += bytes;
  return p;
}

void DevAlloc::put(void *p, size_t bytes) {
  if (!p) return;
  if (free)
    free(p, user);
  else
    (void)hipFree(p);
  held -= bytes;
}

// ---------------------------------------------------------------------------
// kernels

namespace {

constexpr int TPB = 256;

// at least one block: kernels bound-check their index, so empty work is a
// launch that returns at once instead of an invalid grid
inline unsigned nblocks(int64_t n, int tpb = TPB) {
  return (unsigned)std::max<int64_t>(1, (n + tpb - 1) / tpb);
}

// scatter the CSR substructure matrices into the dense blocks A_II, A_IG, A_GG
// A_GG blocks of the substructure matrices into the dense interface pool
__global__ void scatter_gg_kernel(const int *row_sub, const int *row_loc, const int64_t *rowptr,
                                  const int *col, const double *val, int64_t nrows, const int *nI,
                                  const int *nG, const int64_t *offGG, double *AGG) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  const int s = row_sub[g], r = row_loc[g];
  const int ni = nI[s], ng = nG[s];
  if (r < ni) return;
  for (int64_t k = rowptr[g]; k < rowptr[g + 1]; ++k) {
    const int c = col[k];
    if (c >= ni) AGG[offGG[s] + (r - ni) + (int64_t)(c - ni) * ng] = val[k];
  }
}

// S <- S T on every substructure (column pass) and S <- T^T S (row pass).
// T = I + E_p W per constrained glob (W = rows of T at the pivots minus the
// identity there), so a pass adds, for every glob position q_t, the pivot
// columns (rows) weighted by W[k, t].  Pivot values are copied to scratch
// first, so the update may overwrite them.
__global__ void xform_copy_pivots_kernel(const double *pool, const int64_t *offGG, const int *nG,
                                         const GlobXf *gx, int ngx, const int *pos,
                                         const int64_t *offG, double *scr, int rows) {
  const int g = blockIdx.y;
  if (g >= ngx) return;
  const GlobXf x = gx[g];
  const int s = x.sub, ng = nG[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng) return;
  const double *S = pool + offGG[s];
  for (int k = 0; k < x.m; ++k) {
    const int p = pos[x.piv_off + k] - (int)offG[s];
    // rows == 0: column p (entry i); rows == 1: row p (entry i)
    scr[x.scrS_off + (int64_t)k * ng + i] = rows ? S[p + (int64_t)i * ng] : S[i + (int64_t)p * ng];
  }
}

// y[idx[i]] += v for i < n (distinct indices)
__global__ void add_at_kernel(double *y, const int64_t *idx, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[idx[i]] += v;
}

// gather a sub-block: dst[a + b*ldd] = src[idx_r[a] + idx_c[b]*lds] per entry.
// A flat launch: entry s owns the blocks [boff[s], boff[s+1]) (GB_CHUNK of its
// nrows x ncols elements per block, host offsets from gather_offsets), so the
// smaller entries launch no padding.
constexpr int GB_ITEMS = 4;
constexpr int64_t GB_CHUNK = (int64_t)TPB * GB_ITEMS;
__global__ void gather_block_kernel(const double *src, const int64_t *src_off, const int *lds,
                                    double *dst, const int64_t *dst_off, const int *ldd,
                                    const int *ridx, const int64_t *ridx_off, const int *nrows,
                                    const int *cidx, const int64_t *cidx_off, const int *ncols,
                                    double scale, const int64_t *boff, int cnt) {
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = cnt;  // boff[lo] <= blk < boff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= blk)
      lo = mid;
    else
      hi = mid;
  }
  const int s = lo;
  const int64_t nr = nrows[s], nc = ncols[s];
  const int64_t i0 = (blk - boff[s]) * GB_CHUNK + threadIdx.x;
  const double *S = src + src_off[s];
  const int *ri = ridx + ridx_off[s], *ci = cidx + cidx_off[s];
  const int64_t ls = lds[s], ld = ldd[s];
  double *D = dst + dst_off[s];
#pragma unroll
  for (int it = 0; it < GB_ITEMS; ++it) {
    const int64_t i = i0 + (int64_t)it * TPB;
    if (i >= nr * nc) break;
    const int a = (int)(i % nr), c = (int)(i / nr);
    D[a + (int64_t)c * ld] = scale * S[ri[a] + (int64_t)ci[c] * ls];
  }
}

// block offsets of gather_block_kernel for entries of rows[s] x cols[s]
std::vector<int64_t> gather_offsets(const std::vector<int> &rows, const std::vector<int> &cols) {
  std::vector<int64_t> off(rows.size() + 1, 0);
  for (size_t s = 0; s < rows.size(); ++s)
    off[s + 1] = off[s] + ((int64_t)rows[s] * cols[s] + GB_CHUNK - 1) / GB_CHUNK;
  if (off.back() > INT32_MAX) throw ArgError("a gather of more than 2^31 blocks");
  return off;
}

// coarse matrix: S_c[a,b] = sum over substructures holding both a and b
__global__ void coarse_assemble_kernel(int nc, const int *c_ptr, const int *c_sub,
                                       const int *c_loc, const int64_t *offPP, const int *np,
                                       const double *Spi, const int *sub_cids,
                                       const int64_t *offP, double *Sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nc * nc) return;
  const int a = (int)(i % nc), b = (int)(i / nc);
  double acc = 0;
  for (int k = c_ptr[a]; k < c_ptr[a + 1]; ++k) {
    const int s = c_sub[k], la = c_loc[k];
    // local index of b in substructure s: coarse ids of s are ascending
    const int *ids = sub_cids + offP[s];
    int lo = 0, hi = np[s];
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (ids[mid] < b)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < np[s] && ids[lo] == b) acc += Spi[offPP[s] + la + (int64_t)lo * np[s]];
  }
  Sc[a + (int64_t)b * nc] = acc;
}

// dst[i] = src[idx[i]] * (w ? w[i] : 1), multi-column
__global__ void gather_kernel(const double *src, int64_t lds, const int64_t *idx,
                              const double *w, double *dst, int64_t ldd, int64_t n, int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = idx[i];
  const double ww = w ? w[i] : 1.0;
  for (int q = 0; q < nrhs; ++q) dst[i + q * ldd] = ww * src[j + q * lds];
}

__global__ void gather32_kernel(const double *src, int64_t lds, const int *idx, double *dst,
                                int64_t ldd, int64_t n, int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = idx[i];
  for (int q = 0; q < nrhs; ++q) dst[i + q * ldd] = src[j + q * lds];
}

__global__ void scatter32_kernel(const double *src, int64_t lds, const int *idx, double *dst,
                                 int64_t ldd, int64_t n, int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = idx[i];
  for (int q = 0; q < nrhs; ++q) dst[j + q * ldd] = src[i + q * lds];
}

// dst[g] = sum over the copies of g (fixed order) of w[c] * src[c]
__global__ void reduce_copies_kernel(const double *src, int64_t lds, const int *ptr,
                                     const int64_t *copies, const double *w, double *dst,
                                     int64_t ldd, int64_t n, int nrhs, double alpha, double beta) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  for (int q = 0; q < nrhs; ++q) {
    double acc = 0;
    for (int k = ptr[g]; k < ptr[g + 1]; ++k) {
      const int64_t c = copies[k];
      acc += (w ? w[c] : 1.0) * src[c + q * lds];
    }
    double *o = &dst[g + q * ldd];
    *o = (beta == 0.0) ? alpha * acc : alpha * acc + beta * (*o);
  }
}

// b <- T^T b on every constrained glob: pivot values to scratch, then one
// wave per (substructure, glob) adds W^T v to the glob positions.
// (column q of a block: blockIdx.y, vectors at stride ld, scratch at stride ls)
__global__ void vec_pivots_kernel(const double *b, const GlobXf *gx, int ngx, const int *pos,
                                  double *scr, int64_t ld, int64_t ls) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngx) return;
  b += blockIdx.y * ld;
  scr += blockIdx.y * ls;
  const GlobXf x = gx[g];
  for (int k = 0; k < x.m; ++k) scr[x.scr_off + k] = b[pos[x.piv_off + k]];
}

__global__ void apply_Tt_kernel(double *b, const GlobXf *gx, int ngx, const double *wmat,
                                const int *pos, const double *scr, int64_t ld, int64_t ls) {
  const int g = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= ngx) return;
  b += blockIdx.y * ld;
  scr += blockIdx.y * ls;
  const GlobXf x = gx[g];
  const double *wm = wmat + x.trow_off;
  const double *sc = scr + x.scr_off;
  for (int t = lane; t < x.ng; t += 64) {
    double acc = 0;
    // eight rows of W per batch: their loads issued together (the sum keeps
    // the order of one row at a time)
    int k = 0;
    for (; k + 8 <= x.m; k += 8) {
      double w8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w8[u] = wm[(int64_t)(k + u) * x.ng + t];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += w8[u] * sc[k + u];
    }
    for (; k < x.m; ++k) acc += wm[(int64_t)k * x.ng + t] * sc[k];
    b[pos[x.pos_off + t]] += acc;
  }
}

// x <- T x: new pivot values sum_t trow[k, t] x[q_t] into scratch (one wave
// per (glob, k)), then stored at the pivots.
__global__ void apply_T_dots_kernel(const double *xv, const GlobXf *gx, const int *gk_glob,
                                    const int *gk_k, int ngk, const double *trow, const int *pos,
                                    double *scr, int64_t ld, int64_t ls) {
  const int w = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= ngk) return;
  xv += blockIdx.y * ld;
  scr += blockIdx.y * ls;
  const GlobXf x = gx[gk_glob[w]];
  const int k = gk_k[w];
  double acc = 0;
  const double *tr = trow + x.trow_off + (int64_t)k * x.ng;
  const int *ps = pos + x.pos_off;
  // four chunks of 64 entries per batch: their loads issued together (each
  // lane's sum keeps the order of one chunk at a time)
  int t = lane;
  for (; t + 192 < x.ng; t += 256) {
    double tv[4], xw[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      tv[u] = tr[t + 64 * u];
      xw[u] = xv[ps[t + 64 * u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += tv[u] * xw[u];
  }
  for (; t < x.ng; t += 64) acc += tr[t] * xv[ps[t]];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) scr[x.scr_off + k] = acc;
}

__global__ void apply_T_store_kernel(double *xv, const GlobXf *gx, const int *gk_glob,
                                     const int *gk_k, int ngk, const int *pos, const double *scr,
                                     int64_t ld, int64_t ls) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= ngk) return;
  xv += blockIdx.y * ld;
  scr += blockIdx.y * ls;
  const GlobXf x = gx[gk_glob[w]];
  const int k = gk_k[w];
  xv[pos[x.piv_off + k]] = scr[x.scr_off + k];
}

// y_s = S_s x_s for symmetric S_s (column-major, both triangles stored)
// reading only the lower triangle, in two launches.  Work-group (J, s) takes
// the panel of S_s below the diagonal of column block J (columns 64J..64J+63,
// rows 64J..n-1): its columns give y[c] = sum_{r >= 64J} S[r][c] x[r] for c
// in the block (the diagonal block read whole), and its rows below the
// diagonal block give the partial sums a_J[r] = sum_c S[r][c] x[c], which
// stand for the upper triangle.  symv_reduce_kernel then adds, for r in
// block J, a_0[r] + ... + a_{J-1}[r] in that order, so the result does not
// depend on scheduling.  Partials of (s, J) start at off[s] + J n - 32 J (J+1)
// (panel J holds n - 64 (J+1) rows below its diagonal block).
// Eight waves of eight columns each; every element of S loaded is multiplied
// into all m <= M right-hand sides (x, y at column stride ldx, partials at
// ldp).  Per column the operations and their order do not depend on M.
constexpr int SYMV_NT = 512;
template <int M>
__global__ __launch_bounds__(SYMV_NT) void symv_panel_kernel(const double *spool, const int64_t *soff,
                                                             const int *nG, const double *x,
                                                             const int64_t *xoff, int64_t ldx,
                                                             double *y, double *part,
                                                             const int64_t *poff, int64_t ldp,
                                                             int s0, int m) {
  __shared__ double xcs[M][64];         // x at the panel's 64 columns
  __shared__ double red[2][M][8][64];   // row partial sums per wave (double buffered)
  const int s = blockIdx.y + s0, n = nG[s], c0 = 64 * blockIdx.x;
  if (c0 >= n) return;
  const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
  const double *A = spool + soff[s];
  const double *xs = x + xoff[s];
  for (int i = tid; i < M * 64; i += SYMV_NT) {
    const int q = i / 64, c = i % 64;
    xcs[q][c] = (q < m && c0 + c < n) ? xs[c0 + c + q * ldx] : 0.0;
  }
  __syncthreads();
  const int cg = c0 + 8 * g;  // this wave's 8 columns
  double dacc[8][M];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int q = 0; q < M; ++q) dacc[j][q] = 0.0;
  const int64_t pstart = poff[s] + (int64_t)blockIdx.x * n - 32ll * blockIdx.x * (blockIdx.x + 1);
  // the combining thread of the row partial sums: column tid / 64, row lane
  const int cq = tid >> 6;
  int buf = 0;
  for (int rt = c0; rt < n; rt += 64, buf ^= 1) {
    const int r = rt + lane;
    const bool rv = r < n;
    double xr[M];
#pragma unroll
    for (int q = 0; q < M; ++q) xr[q] = (rv && q < m) ? xs[r + q * ldx] : 0.0;
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (rv && cg + j < n) ? A[r + (int64_t)(cg + j) * n] : 0.0;
    double a[M];
#pragma unroll
    for (int q = 0; q < M; ++q) a[q] = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int q = 0; q < M; ++q) {
        dacc[j][q] += v[j] * xr[q];
        a[q] += v[j] * xcs[q][8 * g + j];
      }
    if (rt > c0) {  // rows below the diagonal block (uniform per work-group)
#pragma unroll
      for (int q = 0; q < M; ++q) red[buf][q][g][lane] = a[q];
      __syncthreads();
      if (cq < m && rv) {
        double t = red[buf][cq][0][lane];
#pragma unroll
        for (int w = 1; w < 8; ++w) t += red[buf][cq][w][lane];
        part[pstart + (r - (c0 + 64)) + cq * ldp] = t;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int q = 0; q < M; ++q) {
      double t = dacc[j][q];
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
      if (lane == 0 && q < m && cg + j < n) y[xoff[s] + cg + j + q * ldx] = t;
    }
}

__global__ void symv_reduce_kernel(const int *nG, const int64_t *xoff, int64_t ldx, double *y,
                                   const double *part, const int64_t *poff, int64_t ldp, int s0) {
  const int s = blockIdx.y + s0, n = nG[s];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int J = r / 64;
  const double *ps = part + poff[s] + blockIdx.z * ldp;
  double *yy = y + xoff[s] + r + blockIdx.z * ldx;
  double acc = *yy;
  for (int j = 0; j < J; ++j) acc += ps[(int64_t)j * n - 32ll * j * (j + 1) + (r - 64 * (j + 1))];
  *yy = acc;
}

// batched GEMV on column-major blocks: y_i = alpha op(A_i) x_i + beta y_i,
// for m <= M right-hand sides (x, y at column strides ldx, ldy) sharing the
// loads of A.
// trans: y[j] = sum_r A[r, j] x[r] (a wave per output, coalesced columns);
// notrans: y[r] = sum_j A[r, j] x[j] (a thread per output row).
template <int M>
__global__ void gemv_t_kernel(const double *apool, const int64_t *aoff, const int *rows,
                              const int *cols, const double *x, const int64_t *xoff, int64_t ldx,
                              double *y, const int64_t *yoff, int64_t ldy, double alpha,
                              double beta, int nrhs) {
  const int s = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (j >= cols[s]) return;
  const int m = rows[s];
  const double *A = apool + aoff[s] + (int64_t)j * m;
  const double *xx = x + xoff[s];
  double acc[M];
#pragma unroll
  for (int q = 0; q < M; ++q) acc[q] = 0;
  // four rows per lane per batch: their loads of A are issued together (the
  // sums keep the order of one row at a time)
  int r = lane;
  for (; r + 192 < m; r += 256) {
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = A[r + 64 * u];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < M; ++q)
        if (q < nrhs) acc[q] += a[u] * xx[r + 64 * u + q * ldx];
  }
  for (; r < m; r += 64) {
    const double a = A[r];
#pragma unroll
    for (int q = 0; q < M; ++q)
      if (q < nrhs) acc[q] += a * xx[r + q * ldx];
  }
#pragma unroll
  for (int q = 0; q < M; ++q) {
    for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, 64);
    if (lane == 0 && q < nrhs) {
      double *o = y + yoff[s] + j + q * ldy;
      *o = (beta == 0.0) ? alpha * acc[q] : alpha * acc[q] + beta * (*o);
    }
  }
}

template <int M>
__global__ void gemv_n_kernel(const double *apool, const int64_t *aoff, const int *rows,
                              const int *cols, const double *x, const int64_t *xoff, int64_t ldx,
                              double *y, const int64_t *yoff, int64_t ldy, double alpha,
                              double beta, int nrhs) {
  const int s = blockIdx.y;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = rows[s];
  if (r >= m) return;
  const int n = cols[s];
  const double *A = apool + aoff[s];
  const double *xx = x + xoff[s];
  double acc[M];
#pragma unroll
  for (int q = 0; q < M; ++q) acc[q] = 0;
  // eight columns per batch: their loads of A are issued together (the sums
  // keep the order of one column at a time)
  int j = 0;
  for (; j + 8 <= n; j += 8) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = A[r + (int64_t)(j + u) * m];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int q = 0; q < M; ++q)
        if (q < nrhs) acc[q] += a[u] * xx[j + u + q * ldx];
  }
  for (; j < n; ++j) {
    const double a = A[r + (int64_t)j * m];
#pragma unroll
    for (int q = 0; q < M; ++q)
      if (q < nrhs) acc[q] += a * xx[j + q * ldx];
  }
#pragma unroll
  for (int q = 0; q < M; ++q)
    if (q < nrhs) {
      double *o = y + yoff[s] + r + q * ldy;
      *o = (beta == 0.0) ? alpha * acc[q] : alpha * acc[q] + beta * (*o);
    }
}

// per-substructure CSR products between interior and interface parts:
// mode 0: y_G = A_GI x_I  (rows >= nI, cols < nI)
// mode 1: y_I = A_IG x_G  (rows < nI, cols >= nI)
__global__ void spmv_coupling_kernel(const int *row_sub, const int *row_loc, const int64_t *rowptr,
                                     const int *col, const double *val, int64_t nrows,
                                     const int *nI, const int64_t *offI, const int64_t *offG,
                                     const double *xI, const double *xG, double *yI, double *yG,
                                     int mode, int nrhs, int64_t ldI, int64_t ldG) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  const int s = row_sub[g], r = row_loc[g];
  const int ni = nI[s];
  if (mode == 0 && r < ni) return;
  if (mode == 1 && r >= ni) return;
  for (int q = 0; q < nrhs; ++q) {
    double acc = 0;
    for (int64_t k = rowptr[g]; k < rowptr[g + 1]; ++k) {
      const int c = col[k];
      if (mode == 0 && c < ni) acc += val[k] * xI[offI[s] + c + q * ldI];
      if (mode == 1 && c >= ni) acc += val[k] * xG[offG[s] + (c - ni) + q * ldG];
    }
    if (mode == 0)
      yG[offG[s] + (r - ni) + q * ldG] = acc;
    else
      yI[offI[s] + r + q * ldI] = acc;
  }
}

// y_i = A_i x_i for every substructure (all local rows), x and y split into
// the interior stack (local rows < nI) and the interface stack; a receives
// |A_i| |x_i| (the scale of the rounding in y)
__global__ void spmv_local_kernel(const int *row_sub, const int *row_loc, const int64_t *rowptr,
                                  const int *col, const double *val, int64_t nrows, const int *nI,
                                  const int64_t *offI, const int64_t *offG, const double *xI,
                                  const double *xG, double *yI, double *yG, double *aI,
                                  double *aG) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  const int s = row_sub[g], r = row_loc[g];
  const int ni = nI[s];
  double acc = 0, aacc = 0;
  for (int64_t k = rowptr[g]; k < rowptr[g + 1]; ++k) {
    const int c = col[k];
    const double t = val[k] * (c < ni ? xI[offI[s] + c] : xG[offG[s] + (c - ni)]);
    acc += t;
    aacc += fabs(t);
  }
  if (r < ni) {
    yI[offI[s] + r] = acc;
    aI[offI[s] + r] = aacc;
  } else {
    yG[offG[s] + (r - ni)] = acc;
    aG[offG[s] + (r - ni)] = aacc;
  }
}

// rt = f - (assembled product): interior dofs take their one substructure's
// row, interface dofs the sum over their copies (fixed order)
__global__ void residual_interior_kernel(const double *f, const int64_t *int_gdof,
                                         const double *yI, double *rt, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) rt[int_gdof[k]] = f[int_gdof[k]] - yI[k];
}
__global__ void residual_gamma_kernel(const double *f, const int64_t *gamma_gdof, const int *ptr,
                                      const int64_t *copies, const double *yG, double *rt,
                                      int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  double acc = 0;
  for (int k = ptr[g]; k < ptr[g + 1]; ++k) acc += yG[copies[k]];
  rt[gamma_gdof[g]] = f[gamma_gdof[g]] - acc;
}

// Symmetric diagonal scaling of the constrained local matrices (FP32 factor):
// s = diag(K_rr)^{-1/2} per remaining dof (1 where the diagonal is not
// positive: the factorization reports that pivot).
__global__ void rscale_kernel(const double *K, const int64_t *offRR, const int *nr,
                              const int64_t *offR, double *sc) {
  const int sub = blockIdx.y;
  const int n = nr[sub];
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const double d = K[offRR[sub] + a + (int64_t)a * n];
  sc[offR[sub] + a] = d > 0 ? 1.0 / sqrt(d) : 1.0;
}

// dst (FP32) = diag(rs) src diag(cs) for each substructure's n_r x ncol block
// (column-major, ld n_r; cs == nullptr: no column scaling)
__global__ void scale_f32_kernel(const double *src, float *dst, const int64_t *off, const int *nr,
                                 const int *ncol, const double *rs, const double *cs,
                                 const int64_t *offR) {
  const int sub = blockIdx.y;
  const int64_t n = nr[sub], m = ncol[sub];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * m) return;
  const int a = (int)(i % n), b = (int)(i / n);
  const double v = src[off[sub] + i] * rs[offR[sub] + a] * (cs ? cs[offR[sub] + b] : 1.0);
  dst[off[sub] + i] = (float)v;
}

// dst (FP64) = alpha diag(rs) src (+ dst when accumulate) for each
// substructure's n_r x ncol block (rs == nullptr: no scaling)
__global__ void unscale_f64_kernel(const float *src, double *dst, const int64_t *off, const int *nr,
                                   const int *ncol, const double *rs, const int64_t *offR,
                                   double alpha, int accumulate) {
  const int sub = blockIdx.y;
  const int64_t n = nr[sub], m = ncol[sub];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * m) return;
  const int a = (int)(i % n);
  const double v = alpha * (rs ? rs[offR[sub] + a] : 1.0) * (double)src[off[sub] + i];
  dst[off[sub] + i] = accumulate ? dst[off[sub] + i] + v : v;
}

// y = (D) x elementwise with a change of precision (d: per-element scale)
template <class S, class D>
__global__ void convert_scaled_kernel(const S *src, D *dst, const double *d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = i + blockIdx.y * n;  // column blockIdx.y of a block
  if (i < n) dst[k] = (D)(d[i] * (double)src[k]);
}

// dst = scale * src with a change of precision
template <class S, class D>
__global__ void convert_kernel(const S *src, D *dst, int64_t n, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (D)(scale * (double)src[i]);
}

__global__ void axpby_kernel(double *y, const double *x, double a, double b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = b * y[i] + a * x[i];
}

// deterministic dot products: stage 1 partial sums per block (fixed order);
// column q of a block (blockIdx.y) at a + q lda, b + q ldb, partials at
// part + q DOT_BLOCKS, result at out[q * kScStride]
constexpr int DOT_BLOCKS = 1024;
constexpr int kScStride = 16;  // PCG scalars per column
__global__ void dot_partial_kernel(const double *a, const double *b, int64_t n, int64_t lda,
                                   int64_t ldb, double *part) {
  __shared__ double sh[TPB];
  a += blockIdx.y * lda;
  b += blockIdx.y * ldb;
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x + blockIdx.y * DOT_BLOCKS] = sh[0];
}

__global__ void dot_final_kernel(const double *part, int nb, double *out) {
  __shared__ double sh[TPB];
  part += blockIdx.x * DOT_BLOCKS;
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x * kScStride] = sh[0];
}

// PCG scalars live on the device, kScStride per column q at sc + q
// kScStride: [0] = (r, z), [1] = (p, q), [2] = (r, r), [3] = alpha, [4] =
// beta, [5] = new (r, z), [6] = r0, [7] = rtol, [11] = (r, z_old).  Control
// words: ctl[0] = every column stopped; column q at ctl + kCtl0 + 4 q: [0] =
// stop, [1] = iterations done, [2] = converged, [3] = maxit.  A stopped
// column's x, r and p are left untouched by every later iteration (the
// columns of a block run in lock step until the last one stops), and so are
// iterations launched ahead of the host's check.  The Lanczos coefficients
// and residual history of column q sit at alphas / betas + q (kMaxIt + 1)
// and hist + q (kMaxIt + 2).
constexpr int kCtl0 = 4;
struct PcgInit {
  double r0[Solver::kMaxRhs], rtol[Solver::kMaxRhs];
};
__global__ void pcg_init_kernel(double *sc, int *ctl, PcgInit in, int m, int maxit) {
  const int q = threadIdx.x;
  if (q < m) {
    sc[q * kScStride + 6] = in.r0[q];
    sc[q * kScStride + 7] = in.rtol[q];
    int *c = ctl + kCtl0 + 4 * q;
    const bool zero = in.r0[q] == 0.0;  // nothing to solve: converged at once
    c[0] = zero ? 1 : 0;
    c[1] = 0;
    c[2] = zero ? 1 : 0;
    c[3] = maxit;
  }
  __syncthreads();
  if (q == 0) {
    int all = 1;
    for (int k = 0; k < m; ++k) all &= ctl[kCtl0 + 4 * k];
    ctl[0] = all;
  }
}
__global__ void pcg_alpha_kernel(double *sc, double *alphas, const int *ctl, int m) {
  const int q = threadIdx.x;
  if (q >= m || ctl[kCtl0 + 4 * q]) return;
  double *c = sc + q * kScStride;
  const double a = c[0] / c[1];
  c[3] = a;
  alphas[q * (Solver::kMaxIt + 1) + ctl[kCtl0 + 4 * q + 1]] = a;
}
// after (r, r): the relative residual of this iteration, and the stop test
__global__ void pcg_check_kernel(const double *sc, int *ctl, double *hist, int m) {
  const int q = threadIdx.x;
  if (q < m && !ctl[kCtl0 + 4 * q]) {
    const double *c = sc + q * kScStride;
    int *k = ctl + kCtl0 + 4 * q;
    const int it = k[1] + 1;
    const double rel = sqrt(c[2]) / c[6];
    hist[q * (Solver::kMaxIt + 2) + it] = rel;
    k[1] = it;
    if (!isfinite(rel)) {
      k[0] = 1;
    } else if (rel <= c[7]) {
      k[0] = 1;
      k[2] = 1;
    } else if (it >= k[3]) {
      k[0] = 1;
    }
  }
  __syncthreads();
  if (q == 0) {
    int all = 1;
    for (int j = 0; j < m; ++j) all &= ctl[kCtl0 + 4 * j];
    ctl[0] = all;
  }
}
// beta = (r, z) / (r_old, z_old) (Fletcher-Reeves), or with flexible set
// ((r, z) - (r, z_old)) / (r_old, z_old) (Polak-Ribiere, sc[11] = (r, z_old)):
// the form that tolerates a preconditioner that is not exactly symmetric
// positive definite, as with FP32 local factors
__global__ void pcg_beta_kernel(double *sc, double *betas, const int *ctl, int flexible, int m) {
  const int q = threadIdx.x;
  if (q >= m || ctl[kCtl0 + 4 * q]) return;
  double *c = sc + q * kScStride;
  const double b = (flexible ? c[5] - c[11] : c[5]) / c[0];
  c[4] = b;
  betas[q * (Solver::kMaxIt + 1) + ctl[kCtl0 + 4 * q + 1] - 1] = b;
  c[0] = c[5];
}
// x += alpha p ; r -= alpha q  (column blockIdx.y, vectors at stride n)
__global__ void pcg_update_kernel(double *x, double *r, const double *p, const double *q,
                                  const double *sc, const int *ctl, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || ctl[kCtl0 + 4 * c]) return;
  const double a = sc[c * kScStride + 3];
  const int64_t k = i + c * n;
  x[k] += a * p[k];
  r[k] -= a * q[k];
}
// p = z + beta p
__global__ void pcg_dir_kernel(double *p, const double *z, const double *sc, const int *ctl,
                               int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || ctl[kCtl0 + 4 * c]) return;
  const int64_t k = i + c * n;
  p[k] = z[k] + sc[c * kScStride + 4] * p[k];
}
__global__ void fill_kernel(double *dst, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}
__global__ void copy_kernel(double *dst, const double *src, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// timing

hipEvent_t Timer::get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

void Timer::begin(hipStream_t st, const char *name, double bytes, double flops) {
  if (mode == 1) record_begin(st, name, bytes, flops);
}

void Timer::end(hipStream_t st) {
  if (mode == 1) record_end(st);
}

void Timer::launch_begin(hipStream_t st, const char *kernel, double bytes, double flops) {
  if (mode == 2) record_begin(st, kernel, bytes, flops);
}

void Timer::launch_end(hipStream_t st) {
  if (mode == 2) record_end(st);
}

void Timer::launch_amend(double bytes, double flops) {
  if (mode == 2 && !pending.empty()) {
    pending.back().bytes = bytes;
    pending.back().flops = flops;
  }
}

void Timer::record_begin(hipStream_t st, const char *name, double bytes, double flops) {
  int idx = -1;
  for (size_t i = 0; i < names.size(); ++i)
    if (names[i] == name) idx = (int)i;
  if (idx < 0) {
    idx = (int)names.size();
    names.push_back(name);
    stats.push_back(KernelStat());
  }
  cur = idx;
  cur_a = get_event();
  cur_bytes = bytes;
  cur_flops = flops;
  HIPCHK(hipEventRecord(cur_a, st));
}

void Timer::record_end(hipStream_t st) {
  if (cur < 0) return;
  hipEvent_t b = get_event();
  HIPCHK(hipEventRecord(b, st));
  pending.push_back({cur, cur_a, b, cur_bytes, cur_flops});
  cur = -1;
}

void Timer::collect() {
  for (auto &p : pending) {
    float ms = 0;
    HIPCHK(hipEventSynchronize(p.b));
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    KernelStat &k = stats[p.idx];
    k.ms += ms;
    k.bytes += p.bytes;
    k.flops += p.flops;
    k.launches += 1;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void Timer::reset() {
  collect();
  names.clear();
  stats.clear();
}

Timer::~Timer() {
  for (auto &p : pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// host side

template <class T>
static DBuf upload(DevAlloc &A, hipStream_t st, const std::vector<T> &v) {
  DBuf b;
  b.bytes = std::max<size_t>(v.size() * sizeof(T), 1);
  b.p = A.get(b.bytes);
  if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return b;
}

static DBuf alloc0(DevAlloc &A, hipStream_t st, size_t bytes) {
  DBuf b;
  b.bytes = std::max<size_t>(bytes, 8);
  b.p = A.get(b.bytes);
  HIPCHK(hipMemsetAsync(b.p, 0, b.bytes, st));
  return b;
}

void Solver::release(DBuf &b) {
  if (b.p) alloc.put(b.p, b.bytes);
  b = DBuf();
}

void Solver::free_all() {
  drop_pcg_graph();
  for (DBuf *b : all_buffers()) release(*b);
  for (DBuf &b : sub_plan_bufs) release(b);
  sub_plan_bufs.clear();
  sub_plans.clear();
}

void Solver::drop_pcg_graph() {
  for (hipGraphExec_t &e : pcg_exec) {
    if (e) (void)hipGraphExecDestroy(e);
    e = nullptr;
  }
}

Solver::~Solver() {
  free_all();
  mf.release(alloc);
  for (hipEvent_t &e : pcg_ev)
    if (e) hipEventDestroy(e);
  if (cap_stream) hipStreamDestroy(cap_stream);
  if (pcg_pin) hipHostFree(pcg_pin);
}

// buffers that depend only on the mesh and partition (kept when the
// constraints change) and the ones that depend on the constraints
std::vector<DBuf *> Solver::struct_buffers() {
  return {&d_row_sub, &d_row_loc, &d_rowptr, &d_col, &d_val, &d_nI, &d_nG, &d_offI, &d_offG,
          &d_offGG, &d_S, &d_W, &d_descGG, &d_ifc_gamma, &d_ifc_delta, &d_gamma_ptr,
          &d_gamma_copies, &d_gamma_gdof, &d_int_gdof, &d_ifc_gdof, &d_vG, &d_vG2, &d_vI, &d_vI2,
          &d_gam_r, &d_gam_z, &d_gam_p, &d_gam_q, &d_gam_x, &d_sc, &d_part, &d_alphas, &d_betas,
          &d_pcg_ctl, &d_pcg_hist, &d_symv_part, &d_symv_off, &d_true_r, &d_true_d, &d_abs_I,
          &d_abs_G};
}

std::vector<DBuf *> Solver::cons_buffers() {
  return {&d_nr, &d_np, &d_offR, &d_offP, &d_offRR, &d_offRP, &d_offPP, &d_gb_rr, &d_gb_rp, &d_gb_pp,
          &d_Lrr, &d_Urr, &d_Phi,
          &d_Spi, &d_Lc, &d_Uc, &d_descRRT, &d_dinv_rr, &d_dinv_rr_off, &d_dinv_c, &d_dinv_c_off,
          &d_descRR, &d_descC, &d_spi_desc, &d_gx, &d_gx_ptr, &d_trow, &d_pos, &d_wmat,
          &d_gk_glob, &d_gk_k, &d_scr, &d_xf_cols, &d_xf_rows, &d_xf_map, &d_xf_map_off,
          &d_ridx, &d_ridx_off, &d_pidx, &d_pidx_off, &d_rabs,
          &d_pabs, &d_pcid, &d_sub_cids, &d_c_ptr, &d_c_sub, &d_c_loc, &d_c_copies,
          &d_trsv_rr_fwd, &d_trsv_rr_bwd, &d_trsv_rr_off, &d_trsv_c_fwd, &d_trsv_c_bwd,
          &d_trsv_c_off, &d_work_i, &d_status, &d_vR, &d_vR2, &d_vP, &d_vc, &d_descRRvec,
          &d_descCvec, &d_Lrr32, &d_Urr32, &d_dinv_rr32, &d_vR32, &d_Phi32, &d_rscale, &d_PhiF,
          &d_krrphi_desc};
}

std::vector<DBuf *> Solver::all_buffers() {
  std::vector<DBuf *> a = struct_buffers(), b = cons_buffers();
  a.insert(a.end(), b.begin(), b.end());
  return a;
}

// Host analysis after bddc_setup / adapt: layout, index maps, uploads of the
// substructure matrices.  Matrices and vectors are (re)allocated, except, when
// keep_interior is set (a rebuild for new constraints), the interior
// elimination and -- when current -- the Schur complements: neither depends
// on the constraints.
void Solver::build(const Problem &P, hipStream_t st, bool keep_interior) {
  // phase times of the host rebuild (printed when verbose)
  std::vector<std::pair<const char *, double>> marks;
  auto tmark = std::chrono::steady_clock::now();
  auto mark = [&](const char *what) {
    const auto t = std::chrono::steady_clock::now();
    marks.emplace_back(what, std::chrono::duration<double>(t - tmark).count());
    tmark = t;
  };
  const bool keep_struct = keep_interior && struct_ready;
  drop_pcg_graph();  // it holds the addresses of buffers released here
  for (DBuf *b : cons_buffers()) release(*b);
  if (!keep_struct) {
    for (DBuf *b : struct_buffers()) release(*b);
    mf.release(alloc);
    struct_ready = false;
    schur_ready = false;
  }
  stream = st;
  const int ns = (int)P.subs.size();
  if (!keep_struct) {
    L = Layout();
    L.nsub = ns;
    L.n_glob = P.n_glob;
    L.nI.resize(ns);
    L.nG.resize(ns);
    for (int s = 0; s < ns; ++s) {
      L.nI[s] = P.subs[s].nI;
      L.nG[s] = P.subs[s].nG;
    }
  }
  L.nr.assign(ns, 0);
  L.np.assign(ns, 0);
  L.max_nr = L.max_np = 0;
  // coarse numbering: corner dofs first (ascending), then explicit variables
  // glob by glob
  std::vector<int64_t> corner_cid(P.n_glob, -1);
  int64_t nc = 0;
  for (int64_t g : P.corner_gdofs) corner_cid[g] = nc++;
  std::vector<int64_t> glob_cid0(P.globs.size(), -1);
  for (size_t gi = 0; gi < P.globs.size(); ++gi) {
    glob_cid0[gi] = nc;
    nc += P.cov[gi].m;
  }
  L.n_coarse = nc;
  // per substructure pi dofs: (interface position, coarse id), sorted by coarse id
  std::vector<std::vector<std::pair<int, int>>> pis(ns);
  std::vector<std::vector<int>> rpos(ns);
  for (int s = 0; s < ns; ++s) {
    const Sub &S = P.subs[s];
    auto &pi = pis[s];
    for (size_t k = 0; k < S.corner_pos.size(); ++k)
      pi.push_back({S.corner_pos[k], (int)corner_cid[S.corner_gdof[k]]});
    for (size_t a = 0; a < S.glob_ids.size(); ++a) {
      const int gi = S.glob_ids[a];
      const GlobCov &c = P.cov[gi];
      for (int k = 0; k < c.m; ++k) pi.push_back({S.glob_pos[a][c.perm[k]], (int)(glob_cid0[gi] + k)});
    }
    std::sort(pi.begin(), pi.end(), [](auto &x, auto &y) { return x.second < y.second; });
    std::vector<char> isp(S.nG, 0);
    for (auto &x : pi) isp[x.first] = 1;
    for (int t = 0; t < S.nG; ++t)
      if (!isp[t]) rpos[s].push_back(t);
    L.np[s] = (int)pi.size();
    L.nr[s] = (int)rpos[s].size();
  }
  auto offsets = [&](const std::vector<int> &a, const std::vector<int> &b,
                     std::vector<int64_t> &off) {
    off.resize(ns);
    int64_t o = 0;
    for (int s = 0; s < ns; ++s) {
      off[s] = o;
      o += (int64_t)a[s] * (b.empty() ? 1 : b[s]);
    }
    return o;
  };
  L.sumR = offsets(L.nr, {}, L.offR);
  L.sumP = offsets(L.np, {}, L.offP);
  L.sRR = offsets(L.nr, L.nr, L.offRR);
  L.sRP = offsets(L.nr, L.np, L.offRP);
  L.sPP = offsets(L.np, L.np, L.offPP);
  for (int s = 0; s < ns; ++s) {
    L.max_nr = std::max(L.max_nr, L.nr[s]);
    L.max_np = std::max(L.max_np, L.np[s]);
  }
  d_nr = upload(alloc, st, L.nr);
  d_np = upload(alloc, st, L.np);
  d_offR = upload(alloc, st, L.offR);
  d_offP = upload(alloc, st, L.offP);
  d_offRR = upload(alloc, st, L.offRR);
  d_offRP = upload(alloc, st, L.offRP);
  d_offPP = upload(alloc, st, L.offPP);
  mark("layout");
  h_gb_rr = gather_offsets(L.nr, L.nr);
  h_gb_rp = gather_offsets(L.nr, L.np);
  h_gb_pp = gather_offsets(L.np, L.np);
  d_gb_rr = upload(alloc, st, h_gb_rr);
  d_gb_rp = upload(alloc, st, h_gb_rp);
  d_gb_pp = upload(alloc, st, h_gb_pp);
  if (!keep_struct) build_structure(P, st);
  // transforms
  // the rows of every glob's change of variables are stored once per glob
  // (the substructures sharing it point at the same rows) and W = those rows
  // minus the unit pivot entries is formed on the device, which keeps the
  // upload of the adaptive face rows to one copy
  std::vector<GlobXf> gx;
  std::vector<int> gx_ptr(ns + 1, 0), gk_glob, gk_k;
  std::vector<double> trow;
  std::vector<int64_t> glob_trow(P.cov.size(), -1), piv_idx;
  std::vector<int> pos;
  int64_t scr = 0, scrS = 0;
  for (int s = 0; s < ns; ++s) {
    const Sub &S = P.subs[s];
    for (size_t a = 0; a < S.glob_ids.size(); ++a) {
      const int gi = S.glob_ids[a];
      const GlobCov &c = P.cov[gi];
      if (c.m == 0) continue;
      GlobXf x;
      x.sub = s;
      x.m = c.m;
      x.ng = c.n;
      if (glob_trow[gi] < 0) {
        glob_trow[gi] = (int64_t)trow.size();
        trow.insert(trow.end(), c.trow.begin(), c.trow.end());
        for (int k = 0; k < c.m; ++k) piv_idx.push_back(glob_trow[gi] + (int64_t)k * c.n + c.perm[k]);
      }
      x.trow_off = glob_trow[gi];
      x.pos_off = (int64_t)pos.size();
      for (int t = 0; t < c.n; ++t) pos.push_back((int)(L.offG[s] + S.glob_pos[a][t]));
      x.piv_off = (int64_t)pos.size();
      for (int k = 0; k < c.m; ++k) pos.push_back((int)(L.offG[s] + S.glob_pos[a][c.perm[k]]));
      x.scr_off = scr;
      scr += c.m;
      x.scrS_off = scrS;
      scrS += (int64_t)c.m * S.nG;
      for (int k = 0; k < c.m; ++k) gk_glob.push_back((int)gx.size()), gk_k.push_back(k);
      gx.push_back(x);
      gx_ptr[s + 1]++;
    }
  }
  for (int s = 0; s < ns; ++s) gx_ptr[s + 1] += gx_ptr[s];
  n_gx = (int)gx.size();
  n_gk = (int)gk_glob.size();
  d_gx = upload(alloc, st, gx);
  d_gx_ptr = upload(alloc, st, gx_ptr);
  d_trow = upload(alloc, st, trow);
  d_wmat.bytes = d_trow.bytes;
  d_wmat.p = alloc.get(d_wmat.bytes);
  HIPCHK(hipMemcpyAsync(d_wmat.p, d_trow.p, d_trow.bytes, hipMemcpyDeviceToDevice, st));
  if (!piv_idx.empty()) {
    DBuf d_piv = upload(alloc, st, piv_idx);
    add_at_kernel<<<nblocks((int64_t)piv_idx.size()), TPB, 0, st>>>(d_wmat.as<double>(), d_piv.as<int64_t>(),
                                                                  (int64_t)piv_idx.size(), -1.0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    release(d_piv);
  }
  d_pos = upload(alloc, st, pos);
  d_gk_glob = upload(alloc, st, gk_glob);
  d_gk_k = upload(alloc, st, gk_k);
  scr_elems = std::max<int64_t>(scr, 1);  // per column
  d_scr = alloc0(alloc, st, sizeof(double) * (size_t)scr_elems * kMaxRhs);
  scrS_elems = scrS;
  {
    // T^T S T: the column pass adds (pivot columns, n_G x m) (W, m x ng) into
    // the glob's columns, the row pass W^T (pivot rows, m x n_G) into its rows
    h_xf_cols.clear();
    h_xf_rows.clear();
    std::vector<int> xmap;
    std::vector<int64_t> xmap_off;
    xf_max_ng = 0;
    for (const GlobXf &x : gx) {
      const int n = L.nG[x.sub];
      xmap_off.push_back((int64_t)xmap.size());
      for (int t = 0; t < x.ng; ++t) xmap.push_back(pos[x.pos_off + t] - (int)L.offG[x.sub]);
      h_xf_cols.push_back(GemmDesc{x.scrS_off, x.trow_off, L.offGG[x.sub], n, x.ng, x.m, n, x.ng, n});
      h_xf_rows.push_back(GemmDesc{x.trow_off, x.scrS_off, L.offGG[x.sub], x.ng, n, x.m, x.ng, n, n});
      xf_max_ng = std::max(xf_max_ng, x.ng);
    }
    d_xf_cols = upload(alloc, st, h_xf_cols);
    d_xf_rows = upload(alloc, st, h_xf_rows);
    d_xf_map = upload(alloc, st, xmap);
    d_xf_map_off = upload(alloc, st, xmap_off);
  }
  mark("transforms");
  // r / pi index maps (local interface positions and absolute positions)
  std::vector<int> ridx, pidx, rabs, pabs, pcid, sub_cids;
  std::vector<int64_t> ridx_off(ns), pidx_off(ns);
  for (int s = 0; s < ns; ++s) {
    ridx_off[s] = (int64_t)ridx.size();
    for (int t : rpos[s]) ridx.push_back(t), rabs.push_back((int)(L.offG[s] + t));
    pidx_off[s] = (int64_t)pidx.size();
    for (auto &x : pis[s]) {
      pidx.push_back(x.first);
      pabs.push_back((int)(L.offG[s] + x.first));
      pcid.push_back(x.second);
      sub_cids.push_back(x.second);
    }
  }
  d_ridx = upload(alloc, st, ridx);
  d_ridx_off = upload(alloc, st, ridx_off);
  d_pidx = upload(alloc, st, pidx);
  d_pidx_off = upload(alloc, st, pidx_off);
  d_rabs = upload(alloc, st, rabs);
  d_pabs = upload(alloc, st, pabs);
  d_pcid = upload(alloc, st, pcid);
  d_sub_cids = upload(alloc, st, sub_cids);
  // coarse copies
  std::vector<int> cptr(nc + 1, 0), csub, cloc;
  std::vector<int64_t> ccopies;
  for (int s = 0; s < ns; ++s)
    for (auto &x : pis[s]) cptr[x.second + 1]++;
  for (int64_t a = 0; a < nc; ++a) cptr[a + 1] += cptr[a];
  csub.resize(cptr[nc]);
  cloc.resize(cptr[nc]);
  ccopies.resize(cptr[nc]);
  {
    std::vector<int> fill(cptr.begin(), cptr.end() - 1);
    for (int s = 0; s < ns; ++s)
      for (int l = 0; l < L.np[s]; ++l) {
        const int a = pis[s][l].second;
        const int k = fill[a]++;
        csub[k] = s;
        cloc[k] = l;
        ccopies[k] = L.offP[s] + l;
      }
  }
  d_c_ptr = upload(alloc, st, cptr);
  d_c_sub = upload(alloc, st, csub);
  d_c_loc = upload(alloc, st, cloc);
  d_c_copies = upload(alloc, st, ccopies);
  // descriptors
  std::vector<MatDesc> dRR(ns), dRRv(ns), dRRT(ns);
  std::vector<GemmDesc> spi(ns);
  for (int s = 0; s < ns; ++s) {
    dRR[s] = MatDesc{L.offRR[s], L.offRP[s], L.nr[s], L.np[s], std::max(1, L.nr[s]), std::max(1, L.nr[s])};
    dRRv[s] = MatDesc{L.offRR[s], L.offR[s], L.nr[s], 1, std::max(1, L.nr[s]), (int)L.sumR};
    dRRT[s] = MatDesc{L.offRR[s], L.offRR[s], L.nr[s], 0, std::max(1, L.nr[s]), std::max(1, L.nr[s])};
    spi[s] = GemmDesc{L.offRP[s], L.offRP[s], L.offPP[s], L.np[s], L.np[s], L.nr[s],
                      std::max(1, L.nr[s]), std::max(1, L.nr[s]), std::max(1, L.np[s])};
  }
  h_descRR = dRR;
  d_descRR = upload(alloc, st, dRR);
  d_descRRvec = upload(alloc, st, dRRv);
  d_descRRT = upload(alloc, st, dRRT);
  d_spi_desc = upload(alloc, st, spi);
  h_spi = spi;
  if (factor_precision == 32) {
    // K_rr Phi per substructure (the Galerkin coarse matrix of the FP32 basis)
    std::vector<GemmDesc> kp(ns);
    for (int s = 0; s < ns; ++s)
      kp[s] = GemmDesc{L.offRR[s], L.offRP[s], L.offRP[s], L.nr[s], L.np[s], L.nr[s],
                       std::max(1, L.nr[s]), std::max(1, L.nr[s]), std::max(1, L.nr[s])};
    d_krrphi_desc = upload(alloc, st, kp);
    h_krrphi = kp;
  }
  MatDesc dc{0, 0, (int)nc, 0, (int)std::max<int64_t>(1, nc), (int)std::max<int64_t>(1, nc)};
  h_descC = {dc};
  d_descC = upload(alloc, st, h_descC);
  MatDesc dcv{0, 0, (int)nc, 1, (int)std::max<int64_t>(1, nc), (int)std::max<int64_t>(1, nc)};
  d_descCvec = upload(alloc, st, std::vector<MatDesc>{dcv});
  mark("index maps, descriptors");
  // trsv plans
  auto plan = [&](const std::vector<int> &n, DBuf &f, DBuf &b, DBuf &o, TrsvPlan &p) {
    std::vector<int> fw, bw, off;
    int total;
    make_trsv_orders(n, fw, bw, off, total);
    f = upload(alloc, st, fw);
    b = upload(alloc, st, bw);
    o = upload(alloc, st, off);
    p.batch = (int)n.size();
    p.total_blocks = total;
    p.d_order_fwd = f.as<int>();
    p.d_order_bwd = b.as<int>();
    p.d_flag_off = o.as<int>();
    p.tri_elems = 0;
    p.rows = 0;
    for (int v : n) {
      p.tri_elems += 0.5 * (double)v * (v + 1);
      p.rows += v;
    }
    return total;
  };
  int w1 = plan(L.nr, d_trsv_rr_fwd, d_trsv_rr_bwd, d_trsv_rr_off, plan_rr);
  // per_sub_launches: one plan per substructure (its blocks only; flags from 0)
  for (DBuf &b : sub_plan_bufs) release(b);
  sub_plan_bufs.clear();
  sub_plans.clear();
  if (per_sub_launches)
    for (int q = 0; q < ns; ++q) {
      const int nb = (L.nr[q] + NB - 1) / NB;
      std::vector<int> fw, bw, off(ns, 0);
      for (int k = 0; k < nb; ++k) {
        fw.push_back(q), fw.push_back(k);
        bw.push_back(q), bw.push_back(nb - 1 - k);
      }
      TrsvPlan pq;
      pq.batch = 1;
      pq.total_blocks = nb;
      sub_plan_bufs.push_back(upload(alloc, st, fw.empty() ? std::vector<int>{0} : fw));
      sub_plan_bufs.push_back(upload(alloc, st, bw.empty() ? std::vector<int>{0} : bw));
      sub_plan_bufs.push_back(upload(alloc, st, off));
      const size_t k = sub_plan_bufs.size();
      pq.d_order_fwd = sub_plan_bufs[k - 3].as<int>();
      pq.d_order_bwd = sub_plan_bufs[k - 2].as<int>();
      pq.d_flag_off = sub_plan_bufs[k - 1].as<int>();
      pq.tri_elems = 0.5 * (double)L.nr[q] * (L.nr[q] + 1);
      pq.rows = L.nr[q];
      sub_plans.push_back(pq);
    }
  int w3 = plan({(int)nc}, d_trsv_c_fwd, d_trsv_c_bwd, d_trsv_c_off, plan_c);
  d_work_i = alloc0(alloc, st, sizeof(int) * (size_t)(4 + std::max(w1, w3)));
  d_status = alloc0(alloc, st, sizeof(int) * (size_t)(2 * ns + 2));
  mark("triangular-solve plans");
  // matrices
  const bool p32 = factor_precision == 32;
  d_Lrr = alloc0(alloc, st, sizeof(double) * (size_t)L.sRR);
  d_Urr = alloc0(alloc, st, p32 ? 0 : sizeof(double) * (size_t)L.sRR);
  if (p32) {
    d_Lrr32 = alloc0(alloc, st, sizeof(float) * (size_t)L.sRR);
    d_Urr32 = alloc0(alloc, st, sizeof(float) * (size_t)L.sRR);
    d_vR32 = alloc0(alloc, st, sizeof(float) * (size_t)L.sumR * kMaxRhs);
    d_Phi32 = alloc0(alloc, st, sizeof(float) * (size_t)L.sRP);
    d_PhiF = alloc0(alloc, st, sizeof(double) * (size_t)std::max<int64_t>(1, L.sRP));
    d_rscale = alloc0(alloc, st, sizeof(double) * (size_t)std::max<int64_t>(1, L.sumR));
  }
  d_Phi = alloc0(alloc, st, sizeof(double) * (size_t)L.sRP);
  d_Spi = alloc0(alloc, st, sizeof(double) * (size_t)L.sPP);
  d_Lc = alloc0(alloc, st, sizeof(double) * (size_t)(nc * nc));
  d_Uc = alloc0(alloc, st, sizeof(double) * (size_t)(nc * nc));
  {
    // inverses of the NB x NB diagonal blocks of L_rr and L_c
    std::vector<int64_t> off(ns);
    int64_t tot = 0;
    for (int s = 0; s < ns; ++s) {
      off[s] = tot;
      tot += (int64_t)((L.nr[s] + NB - 1) / NB) * NB * NB;
    }
    d_dinv_rr = alloc0(alloc, st, sizeof(double) * (size_t)tot);
    if (p32) d_dinv_rr32 = alloc0(alloc, st, sizeof(float) * (size_t)tot);
    dinv_rr_elems = tot;
    d_dinv_rr_off = upload(alloc, st, off);
    h_dinv_rr_off = off;
    d_dinv_c = alloc0(alloc, st, sizeof(double) * (size_t)(((nc + NB - 1) / NB) * NB * NB));
    d_dinv_c_off = upload(alloc, st, std::vector<int64_t>{0});
  }
  // work vectors (nrhs up to kMaxRhs)
  const size_t R = kMaxRhs;
  d_vR = alloc0(alloc, st, sizeof(double) * L.sumR * R);
  d_vR2 = alloc0(alloc, st, sizeof(double) * L.sumR * R);
  d_vP = alloc0(alloc, st, sizeof(double) * L.sumP * R);
  d_vc = alloc0(alloc, st, sizeof(double) * nc * R);
  bytes_S = 0;
  bytes_Lrr_tri = 0;
  for (int s = 0; s < ns; ++s) {
    bytes_S += 8.0 * (double)L.nG[s] * L.nG[s];
    bytes_Lrr_tri += (p32 ? 4.0 : 8.0) * 0.5 * (double)L.nr[s] * (L.nr[s] + 1);
  }
  HIPCHK(hipStreamSynchronize(st));
  mark("matrices and work vectors");
  factored = false;
  struct_ready = true;
  if (verbose) {
    std::string line = "[bddc build]";
    char buf[96];
    for (auto &m : marks) {
      std::snprintf(buf, sizeof buf, " %s %.1f ms;", m.first, 1e3 * m.second);
      line += buf;
    }
    std::fprintf(stderr, "%s\n", line.c_str());
  }
}

// The part of the layout that depends only on the mesh and partition: the
// stacked substructure matrices, interface numbering and maps, the interface
// Schur complement pools, work vectors and the interior elimination.
void Solver::build_structure(const Problem &P, hipStream_t st) {
  const int ns = L.nsub;
  auto offsets = [&](const std::vector<int> &a, std::vector<int64_t> &off, bool square) {
    off.resize(ns);
    int64_t o = 0;
    for (int s = 0; s < ns; ++s) {
      off[s] = o;
      o += (int64_t)a[s] * (square ? a[s] : 1);
    }
    return o;
  };
  L.sumI = offsets(L.nI, L.offI, false);
  L.sumG = offsets(L.nG, L.offG, false);
  L.sGG = offsets(L.nG, L.offGG, true);
  L.max_nI = L.max_nG = 0;
  for (int s = 0; s < ns; ++s) {
    L.max_nI = std::max(L.max_nI, L.nI[s]);
    L.max_nG = std::max(L.max_nG, L.nG[s]);
  }
  // CSR stack
  std::vector<int> row_sub, row_loc, col;
  std::vector<int64_t> rowptr(1, 0);
  std::vector<double> val;
  for (int s = 0; s < ns; ++s) {
    const Csr &A = P.subs[s].A;
    for (int r = 0; r < A.n; ++r) {
      row_sub.push_back(s);
      row_loc.push_back(r);
      rowptr.push_back(rowptr.back() + (A.ptr[r + 1] - A.ptr[r]));
    }
    col.insert(col.end(), A.col.begin(), A.col.end());
    val.insert(val.end(), A.val.begin(), A.val.end());
  }
  n_rows = (int64_t)row_sub.size();
  nnz = (int64_t)val.size();
  d_row_sub = upload(alloc, st, row_sub);
  d_row_loc = upload(alloc, st, row_loc);
  d_rowptr = upload(alloc, st, rowptr);
  d_col = upload(alloc, st, col);
  d_val = upload(alloc, st, val);
  d_nI = upload(alloc, st, L.nI);
  d_nG = upload(alloc, st, L.nG);
  d_offI = upload(alloc, st, L.offI);
  d_offG = upload(alloc, st, L.offG);
  d_offGG = upload(alloc, st, L.offGG);
  // interface maps: global interface dof numbering gamma (ascending global)
  std::vector<int64_t> gam_of(P.n_glob, -1);
  std::vector<int> mult(P.n_glob, 0);
  for (int s = 0; s < ns; ++s)
    for (int t = 0; t < L.nG[s]; ++t) mult[P.subs[s].gdof[L.nI[s] + t]]++;
  std::vector<int64_t> gamma_gdof;
  for (int64_t g = 0; g < P.n_glob; ++g)
    if (mult[g] > 0) {
      gam_of[g] = (int64_t)gamma_gdof.size();
      gamma_gdof.push_back(g);
    }
  L.n_gamma = (int64_t)gamma_gdof.size();
  std::vector<int64_t> ifc_gamma(L.sumG), ifc_gdof(L.sumG), int_gdof(L.sumI);
  std::vector<double> ifc_delta(L.sumG);
  std::vector<int> gptr(L.n_gamma + 1, 0);
  for (int s = 0; s < ns; ++s)
    for (int t = 0; t < L.nG[s]; ++t) {
      const int64_t g = P.subs[s].gdof[L.nI[s] + t];
      ifc_gamma[L.offG[s] + t] = gam_of[g];
      ifc_gdof[L.offG[s] + t] = g;
      ifc_delta[L.offG[s] + t] = P.subs[s].delta[t];
      gptr[gam_of[g] + 1]++;
    }
  for (int64_t k = 0; k < L.n_gamma; ++k) gptr[k + 1] += gptr[k];
  std::vector<int64_t> gcopies(gptr[L.n_gamma]);
  {
    std::vector<int> fill(gptr.begin(), gptr.end() - 1);
    for (int s = 0; s < ns; ++s)  // substructures ascending: fixed summation order
      for (int t = 0; t < L.nG[s]; ++t) gcopies[fill[ifc_gamma[L.offG[s] + t]]++] = L.offG[s] + t;
  }
  for (int s = 0; s < ns; ++s)
    for (int t = 0; t < L.nI[s]; ++t) int_gdof[L.offI[s] + t] = P.subs[s].gdof[t];
  d_ifc_gamma = upload(alloc, st, ifc_gamma);
  d_ifc_gdof = upload(alloc, st, ifc_gdof);
  d_ifc_delta = upload(alloc, st, ifc_delta);
  d_gamma_ptr = upload(alloc, st, gptr);
  d_gamma_copies = upload(alloc, st, gcopies);
  d_gamma_gdof = upload(alloc, st, gamma_gdof);
  d_int_gdof = upload(alloc, st, int_gdof);
  std::vector<MatDesc> dGG(ns);
  for (int s = 0; s < ns; ++s) dGG[s] = MatDesc{L.offGG[s], 0, L.nG[s], 0, std::max(1, L.nG[s]), 1};
  h_descGG = dGG;
  d_descGG = upload(alloc, st, dGG);
  d_S = alloc0(alloc, st, sizeof(double) * (size_t)L.sGG);
  d_W = alloc0(alloc, st, sizeof(double) * (size_t)L.sGG);
  const size_t R = kMaxRhs;
  d_vG = alloc0(alloc, st, sizeof(double) * L.sumG * R);
  d_vG2 = alloc0(alloc, st, sizeof(double) * L.sumG * R);
  {
    // partial sums of the symmetric Schur products: n - 64 (J+1) rows per
    // column block J below its diagonal block
    std::vector<int64_t> off(ns);
    int64_t tot = 0;
    bytes_S_sym = 0;
    for (int s = 0; s < ns; ++s) {
      off[s] = tot;
      const int64_t n = L.nG[s], nb = (n + 63) / 64;
      for (int64_t j = 0; j < nb; ++j) {
        tot += std::max<int64_t>(0, n - 64 * (j + 1));
        // the panel read: rows 64j.. of its columns (diagonal block whole)
        bytes_S_sym += 8.0 * (double)std::min<int64_t>(64, n - 64 * j) * (double)(n - 64 * j);
      }
    }
    symv_parts = (double)tot;
    d_symv_part = alloc0(alloc, st, sizeof(double) * std::max<int64_t>(1, tot) * R);
    d_symv_off = upload(alloc, st, off);
  }
  d_vI = alloc0(alloc, st, sizeof(double) * L.sumI * R);
  d_vI2 = alloc0(alloc, st, sizeof(double) * L.sumI * R);
  d_gam_r = alloc0(alloc, st, sizeof(double) * L.n_gamma * R);
  d_gam_z = alloc0(alloc, st, sizeof(double) * L.n_gamma * R);
  d_gam_p = alloc0(alloc, st, sizeof(double) * L.n_gamma * R);
  d_gam_q = alloc0(alloc, st, sizeof(double) * L.n_gamma * R);
  d_gam_x = alloc0(alloc, st, sizeof(double) * L.n_gamma * R);
  d_sc = alloc0(alloc, st, sizeof(double) * kScStride * R);
  d_part = alloc0(alloc, st, sizeof(double) * DOT_BLOCKS * R);
  d_alphas = alloc0(alloc, st, sizeof(double) * (kMaxIt + 1) * R);
  d_betas = alloc0(alloc, st, sizeof(double) * (kMaxIt + 1) * R);
  d_pcg_ctl = alloc0(alloc, st, sizeof(int) * (kCtl0 + 4 * R));
  d_pcg_hist = alloc0(alloc, st, sizeof(double) * (kMaxIt + 2) * R);
  d_true_r = alloc0(alloc, st, sizeof(double) * std::max<int64_t>(1, L.n_glob));
  d_true_d = alloc0(alloc, st, sizeof(double) * std::max<int64_t>(1, L.n_glob));
  d_abs_I = alloc0(alloc, st, sizeof(double) * std::max<int64_t>(1, L.sumI));
  d_abs_G = alloc0(alloc, st, sizeof(double) * std::max<int64_t>(1, L.sumG));
  // interior elimination
  mf.setup(P, L.offI, alloc, st);
}

// Dirichlet factors of A_II (multifrontal) and Schur complements S_i
// (original basis); independent of the constraints.
void Solver::factor_schur() {
  hipStream_t st = stream;
  const int ns = L.nsub;
  HIPCHK(hipMemsetAsync(d_status.p, 0, d_status.bytes, st));
  HIPCHK(hipMemsetAsync(d_S.p, 0, d_S.bytes, st));
  scatter_gg_kernel<<<nblocks(n_rows), TPB, 0, st>>>(
      d_row_sub.as<int>(), d_row_loc.as<int>(), d_rowptr.as<int64_t>(), d_col.as<int>(),
      d_val.as<double>(), n_rows, d_nI.as<int>(), d_nG.as<int>(), d_offGG.as<int64_t>(),
      d_S.as<double>());
  HIPCHK(hipGetLastError());
  timer.begin(st, "factor_interior_schur", 8.0 * (mf.sym.l_entries + (double)mf.sym.c_size), mf.sym.flops);
  mf.factor(st, d_val.as<double>(), nnz, d_S.as<double>(), d_offGG.as<int64_t>(), d_nG.as<int>(),
            L.max_nG, ns);
  timer.end(st);
  HIPCHK(symmetrize_lower<double>(st, d_S.as<double>(), d_descGG.as<MatDesc>(), ns, L.max_nG,
                                  h_descGG.data()));
  check_status(false);
  schur_ready = true;
}

void Solver::factor() {
  hipStream_t st = stream;
  const int ns = L.nsub;
  auto t0 = std::chrono::steady_clock::now();
  const bool did_interior = !schur_ready;
  if (schur_ready) {
    HIPCHK(hipMemsetAsync(d_status.p, 0, d_status.bytes, st));
  } else {
    factor_schur();
  }
  // one factor consumes the Schur complements: the next factor (or adapt)
  // recomputes them from the substructure matrices
  schur_ready = false;
  int *status = d_status.as<int>();
  double fl_rr = 0;
  for (int s = 0; s < ns; ++s) fl_rr += (double)L.nr[s] * L.nr[s] * L.nr[s] / 3;
  // transformed Schur complements Sbar = T^T S T in the work pool
  HIPCHK(hipMemcpyAsync(d_W.p, d_S.p, sizeof(double) * L.sGG, hipMemcpyDeviceToDevice, st));
  if (n_gx > 0 && L.max_nG > 0) {
    DBuf scrS;
    scrS.bytes = sizeof(double) * (size_t)scrS_elems;
    scrS.p = alloc.get(scrS.bytes);
    for (int rows = 0; rows < 2; ++rows) {
      xform_copy_pivots_kernel<<<dim3(nblocks(L.max_nG), n_gx), TPB, 0, st>>>(
          d_W.as<double>(), d_offGG.as<int64_t>(), d_nG.as<int>(), d_gx.as<GlobXf>(), n_gx,
          d_pos.as<int>(), d_offG.as<int64_t>(), scrS.as<double>(), rows);
      HIPCHK(hipGetLastError());
      if (!rows)
        HIPCHK(DenseOps<double>::gemm_scatter(st, scrS.as<double>(), d_wmat.as<double>(),
                                              d_W.as<double>(), d_xf_cols.as<GemmDesc>(),
                                              d_xf_map.as<int>(), d_xf_map_off.as<int64_t>(), false,
                                              n_gx, L.max_nG, xf_max_ng, h_xf_cols.data()));
      else
        HIPCHK(DenseOps<double>::gemm_scatter(st, d_wmat.as<double>(), scrS.as<double>(),
                                              d_W.as<double>(), d_xf_rows.as<GemmDesc>(),
                                              d_xf_map.as<int>(), d_xf_map_off.as<int64_t>(), true,
                                              n_gx, xf_max_ng, L.max_nG, h_xf_rows.data()));
    }
    HIPCHK(hipStreamSynchronize(st));
    release(scrS);
  }
  // split into rr, r-pi, pi-pi
  auto gather = [&](DBuf &dst, const DBuf &dstoff, const DBuf &ldd, const DBuf &ri, const DBuf &rio,
                    const DBuf &nrow, const DBuf &ci, const DBuf &cio, const DBuf &ncol,
                    const std::vector<int64_t> &h_boff, const DBuf &boff, double scale) {
    if (h_boff.back() <= 0) return;
    gather_block_kernel<<<(unsigned)h_boff.back(), TPB, 0, st>>>(
        d_W.as<double>(), d_offGG.as<int64_t>(), d_nG.as<int>(), dst.as<double>(),
        dstoff.as<int64_t>(), ldd.as<int>(), ri.as<int>(), rio.as<int64_t>(), nrow.as<int>(),
        ci.as<int>(), cio.as<int64_t>(), ncol.as<int>(), scale, boff.as<int64_t>(), ns);
    HIPCHK(hipGetLastError());
  };
  gather(d_Lrr, d_offRR, d_nr, d_ridx, d_ridx_off, d_nr, d_ridx, d_ridx_off, d_nr, h_gb_rr, d_gb_rr, 1.0);
  gather(d_Phi, d_offRP, d_nr, d_ridx, d_ridx_off, d_nr, d_pidx, d_pidx_off, d_np, h_gb_rp, d_gb_rp, 1.0);
  gather(d_Spi, d_offPP, d_np, d_pidx, d_pidx_off, d_np, d_pidx, d_pidx_off, d_np, h_gb_pp, d_gb_pp, 1.0);
  // constrained local factor and coarse basis (FP64, or FP32 local factors
  // with an FP64 Galerkin coarse matrix: factor_local_fp32); all substructures
  // in each launch sequence, or with per_substructure_launches one sequence
  // per substructure (the dense operations follow per_entry_launches)
  const MatDesc *dRR = d_descRR.as<MatDesc>();
  const int64_t *dio = d_dinv_rr_off.as<int64_t>();
  fp32_fallbacks = 0;
  if (factor_precision == 32) {
    factor_local_fp32(status);
  } else {
    timer.begin(st, "factor_potrf_local", 8.0 * L.sRR, fl_rr);
    HIPCHK(DenseOps<double>::potrf(st, d_Lrr.as<double>(), dRR, h_descRR.data(), ns, status + ns,
                                   d_dinv_rr.as<double>(), dio));
    timer.end(st);
    HIPCHK(DenseOps<double>::trsm(st, d_Lrr.as<double>(), d_Phi.as<double>(), dRR, h_descRR.data(), ns,
                                  false, d_dinv_rr.as<double>(), dio));
    HIPCHK(DenseOps<double>::gemm(st, d_Phi.as<double>(), d_Phi.as<double>(), d_Spi.as<double>(),
                                  d_spi_desc.as<GemmDesc>(), ns, L.max_np, L.max_np, true, false, -1.0,
                                  1.0, false, h_spi.data()));
    HIPCHK(DenseOps<double>::trsm(st, d_Lrr.as<double>(), d_Phi.as<double>(), dRR, h_descRR.data(), ns,
                                  true, d_dinv_rr.as<double>(), dio));
    if (L.sRP > 0) {
      axpby_kernel<<<nblocks(L.sRP), TPB, 0, st>>>(d_Phi.as<double>(), d_Phi.as<double>(), 0.0, -1.0,
                                                   L.sRP);
      HIPCHK(hipGetLastError());
    }
    // L_rr^T beside L_rr: the backward solves read it row-coalesced
    HIPCHK(transpose_batched<double>(st, d_Lrr.as<double>(), d_Urr.as<double>(),
                                     d_descRRT.as<MatDesc>(), ns, L.max_nr, h_descRR.data()));
  }
  // coarse problem
  const int64_t nc = L.n_coarse;
  if (nc > 0) {
    coarse_assemble_kernel<<<nblocks(nc * nc), TPB, 0, st>>>(
        (int)nc, d_c_ptr.as<int>(), d_c_sub.as<int>(), d_c_loc.as<int>(), d_offPP.as<int64_t>(),
        d_np.as<int>(), d_Spi.as<double>(), d_sub_cids.as<int>(), d_offP.as<int64_t>(),
        d_Lc.as<double>());
    HIPCHK(hipGetLastError());
    HIPCHK(DenseOps<double>::potrf(st, d_Lc.as<double>(), d_descC.as<MatDesc>(), h_descC.data(), 1,
                                   status + 2 * ns, d_dinv_c.as<double>(),
                                   d_dinv_c_off.as<int64_t>()));
    HIPCHK(transpose_batched<double>(st, d_Lc.as<double>(), d_Uc.as<double>(), d_descC.as<MatDesc>(), 1,
                                     (int)nc, h_descC.data()));
  }
  check_status(true);
  auto t1 = std::chrono::steady_clock::now();
  factor_seconds = std::chrono::duration<double>(t1 - t0).count();
  // flops executed by this call (the interior elimination only when it was
  // not reused from bddc_adapt)
  double fl = did_interior ? mf.sym.flops : 0.0;
  for (int s = 0; s < ns; ++s) {
    const double nr = L.nr[s], np = L.np[s];
    fl += nr * nr * nr / 3 + 2 * nr * nr * np + nr * np * np;
  }
  fl += (double)nc * nc * nc / 3;
  factor_flops = fl;
  factored = true;
}

// The constrained local factorization in FP32 on the matrix cores (FP32
// accumulate): K_rr is scaled symmetrically, S K_rr S with S = diag(K_rr)^-1/2,
// converted and factored, Lt Lt^T = S K_rr S.  A substructure whose FP32
// factorization meets a non-positive pivot is factored again in FP64 from
// the unscaled K_rr (kept in FP64) and stored rounded with unit scaling; the
// count is reported.  The coarse basis runs through the FP32 factor, Phi =
// -S Lt^-T Lt^-1 S K_r,pi (FP32 TRSMs) with one FP64-residual refinement
// step, and S_pi is its Galerkin product in FP64 (below).  The coarse matrix
// and its factor stay FP64.
void Solver::factor_local_fp32(int *status) {
  hipStream_t st = stream;
  const int ns = L.nsub;
  const MatDesc *dRR = d_descRR.as<MatDesc>();
  const int64_t *dio = d_dinv_rr_off.as<int64_t>();
  double *sc = d_rscale.as<double>();
  float *L32 = d_Lrr32.as<float>(), *P32 = d_Phi32.as<float>();
  if (L.max_nr == 0) return;
  rscale_kernel<<<dim3(nblocks(L.max_nr), ns), TPB, 0, st>>>(d_Lrr.as<double>(), d_offRR.as<int64_t>(),
                                                             d_nr.as<int>(), d_offR.as<int64_t>(), sc);
  scale_f32_kernel<<<dim3(nblocks((int64_t)L.max_nr * L.max_nr), ns), TPB, 0, st>>>(
      d_Lrr.as<double>(), L32, d_offRR.as<int64_t>(), d_nr.as<int>(), d_nr.as<int>(), sc, sc,
      d_offR.as<int64_t>());
  HIPCHK(hipGetLastError());
  double fl = 0;
  for (int q = 0; q < ns; ++q) fl += (double)L.nr[q] * L.nr[q] * L.nr[q] / 3;
  timer.begin(st, "factor_potrf_local", 4.0 * L.sRR, fl);
  HIPCHK(DenseOps<float>::potrf(st, L32, dRR, h_descRR.data(), ns, status + ns,
                                d_dinv_rr32.as<float>(), dio));
  timer.end(st);
  std::vector<int> hs(ns);
  HIPCHK(hipMemcpyAsync(hs.data(), status + ns, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int q = 0; q < ns; ++q) {
    if (!hs[q]) continue;
    // FP64 fallback for this substructure: its pivot flag is cleared first,
    // so that a failure here is reported as NOT_SPD
    ++fp32_fallbacks;
    HIPCHK(hipMemsetAsync(status + ns + q, 0, sizeof(int), st));
    const int64_t n = L.nr[q], nb = (n + NB - 1) / NB;
    const int64_t o = h_descRR[q].a_off;
    // the FP64 factorization runs in place; K_rr itself is kept aside and put
    // back afterwards, since the Galerkin product below needs it unfactored
    const size_t kbytes = sizeof(double) * (size_t)(n * n);
    void *keep = alloc.get(kbytes);
    HIPCHK(hipMemcpyAsync(keep, d_Lrr.as<double>() + o, kbytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(DenseOps<double>::potrf(st, d_Lrr.as<double>(), dRR + q, &h_descRR[q], 1, status + ns + q,
                                   d_dinv_rr.as<double>(), dio + q));
    convert_kernel<double, float><<<nblocks(n * n), TPB, 0, st>>>(d_Lrr.as<double>() + o, L32 + o,
                                                                   n * n, 1.0);
    convert_kernel<double, float><<<nblocks(nb * NB * NB), TPB, 0, st>>>(
        d_dinv_rr.as<double>() + h_dinv_rr_off[q], d_dinv_rr32.as<float>() + h_dinv_rr_off[q],
        nb * NB * NB, 1.0);
    fill_kernel<<<nblocks(n), TPB, 0, st>>>(sc + L.offR[q], 1.0, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(d_Lrr.as<double>() + o, keep, kbytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    alloc.put(keep, kbytes);
  }
  if (L.max_np > 0) {
    double *PhiF = d_PhiF.as<double>(), *Krp = d_Phi.as<double>();
    const int64_t mx = (int64_t)L.max_nr * L.max_np;
    // K_rr^-1 X ~ S Lt^-T Lt^-1 S X in FP32: PhiF (+)= alpha of that, X in Krp
    auto solve32 = [&](double alpha, int accumulate) {
      scale_f32_kernel<<<dim3(nblocks(mx), ns), TPB, 0, st>>>(Krp, P32, d_offRP.as<int64_t>(),
                                                              d_nr.as<int>(), d_np.as<int>(), sc,
                                                              nullptr, d_offR.as<int64_t>());
      HIPCHK(hipGetLastError());
      HIPCHK(DenseOps<float>::trsm(st, L32, P32, dRR, h_descRR.data(), ns, false,
                                   d_dinv_rr32.as<float>(), dio));
      HIPCHK(DenseOps<float>::trsm(st, L32, P32, dRR, h_descRR.data(), ns, true,
                                   d_dinv_rr32.as<float>(), dio));
      unscale_f64_kernel<<<dim3(nblocks(mx), ns), TPB, 0, st>>>(P32, PhiF, d_offRP.as<int64_t>(),
                                                                d_nr.as<int>(), d_np.as<int>(), sc,
                                                                d_offR.as<int64_t>(), alpha, accumulate);
      HIPCHK(hipGetLastError());
    };
    // Krp = K_r,pi (again) and Krp += K_rr PhiF: the FP64 residual of K_rr Phi = -K_r,pi
    auto residual = [&]() {
      if (h_gb_rp.back() > 0)
        gather_block_kernel<<<(unsigned)h_gb_rp.back(), TPB, 0, st>>>(
            d_W.as<double>(), d_offGG.as<int64_t>(), d_nG.as<int>(), Krp, d_offRP.as<int64_t>(),
            d_nr.as<int>(), d_ridx.as<int>(), d_ridx_off.as<int64_t>(), d_nr.as<int>(), d_pidx.as<int>(),
            d_pidx_off.as<int64_t>(), d_np.as<int>(), 1.0, d_gb_rp.as<int64_t>(), ns);
      HIPCHK(hipGetLastError());
      HIPCHK(DenseOps<double>::gemm(st, d_Lrr.as<double>(), PhiF, Krp, d_krrphi_desc.as<GemmDesc>(),
                                    ns, L.max_nr, L.max_np, false, false, 1.0, 1.0, false,
                                    h_krrphi.data()));
    };
    // Phi_0 = -K_rr^-1 K_r,pi by the FP32 factor; one step of refinement with
    // the FP64 residual W_0 = K_r,pi + K_rr Phi_0: Phi_1 = Phi_0 - K_rr^-1 W_0
    solve32(-1.0, 0);
    residual();
    solve32(-1.0, 1);
    // S_pi as the Galerkin product [Phi; I]^T K [Phi; I] in FP64 (K_rr, K_r,pi
    // and K_pi,pi unrounded): symmetric positive definite for any basis, and
    // off the exact Schur complement only by (Phi - Phi_exact)^T K_rr (Phi -
    // Phi_exact).  The shorter form K_pi,pi - K_pi,r K_rr^-1 K_r,pi with an
    // FP32 solve loses its small eigenvalues to cancellation at high
    // coefficient contrast (an indefinite coarse matrix at the 64^3 k-means
    // size; without the refinement step the basis costs 76 PCG iterations
    // there instead of 30).  S_pi += K_pi,r Phi; W = K_r,pi + K_rr Phi;
    // S_pi += Phi^T W.
    if (h_gb_rp.back() > 0)
      gather_block_kernel<<<(unsigned)h_gb_rp.back(), TPB, 0, st>>>(
          d_W.as<double>(), d_offGG.as<int64_t>(), d_nG.as<int>(), Krp, d_offRP.as<int64_t>(),
          d_nr.as<int>(), d_ridx.as<int>(), d_ridx_off.as<int64_t>(), d_nr.as<int>(), d_pidx.as<int>(),
          d_pidx_off.as<int64_t>(), d_np.as<int>(), 1.0, d_gb_rp.as<int64_t>(), ns);
    HIPCHK(hipGetLastError());
    HIPCHK(DenseOps<double>::gemm(st, Krp, PhiF, d_Spi.as<double>(), d_spi_desc.as<GemmDesc>(), ns,
                                  L.max_np, L.max_np, true, false, 1.0, 1.0, false, h_spi.data()));
    HIPCHK(DenseOps<double>::gemm(st, d_Lrr.as<double>(), PhiF, Krp, d_krrphi_desc.as<GemmDesc>(), ns,
                                  L.max_nr, L.max_np, false, false, 1.0, 1.0, false, h_krrphi.data()));
    HIPCHK(DenseOps<double>::gemm(st, PhiF, Krp, d_Spi.as<double>(), d_spi_desc.as<GemmDesc>(), ns,
                                  L.max_np, L.max_np, true, false, 1.0, 1.0, false, h_spi.data()));
    HIPCHK(hipMemcpyAsync(Krp, PhiF, sizeof(double) * L.sRP, hipMemcpyDeviceToDevice, st));
  }
  HIPCHK(transpose_batched<float>(st, L32, d_Urr32.as<float>(), d_descRRT.as<MatDesc>(), ns, L.max_nr,
                                  h_descRR.data()));
}

void Solver::check_status(bool all) {
  const int ns = L.nsub;
  std::vector<int> hs(2 * ns + 2, 0);
  HIPCHK(hipMemcpyAsync(hs.data(), d_status.p, sizeof(int) * (2 * ns + 2), hipMemcpyDeviceToHost,
                        stream));
  HIPCHK(hipStreamSynchronize(stream));
  timer.collect();
  for (int s = 0; s < ns; ++s) {
    if (hs[s])
      throw NotSpdError("substructure " + std::to_string(s) +
                        ": interior (Dirichlet) matrix, non-positive pivot at column " +
                        std::to_string(hs[s] - 1) + " of " + std::to_string(L.nI[s]));
    if (all && hs[ns + s])
      throw NotSpdError("substructure " + std::to_string(s) +
                        ": constrained interface matrix, non-positive pivot at column " +
                        std::to_string(hs[ns + s] - 1) + " of " + std::to_string(L.nr[s]));
  }
  if (all && hs[2 * ns])
    throw SingularCoarseError("coarse problem: non-positive pivot at column " +
                              std::to_string(hs[2 * ns] - 1) + " of " + std::to_string(L.n_coarse));
}

// ---------------------------------------------------------------------------
// preconditioner and PCG (one right-hand side per call of the internals)

void Solver::trsv(const TrsvPlan &plan, const DBuf &A, const DBuf &desc, const DBuf &dinv,
                  const DBuf &dinv_off, double *x, bool upper, const ApplyWork &w, int m,
                  int64_t ldx) {
  // the substructures' local solves one at a time (per_sub_launches)
  if (&plan == &plan_rr && !sub_plans.empty()) {
    for (const TrsvPlan &pq : sub_plans)
      HIPCHK(trsv_blocked<double>(stream, A.as<double>(), x, desc.as<MatDesc>(), pq, upper,
                                  dinv.as<double>(), dinv_off.as<int64_t>(), w.trsv_work, w.err, m,
                                  ldx));
    return;
  }
  HIPCHK(trsv_blocked<double>(stream, A.as<double>(), x, desc.as<MatDesc>(), plan, upper,
                              dinv.as<double>(), dinv_off.as<int64_t>(), w.trsv_work, w.err, m, ldx));
}
void Solver::trsv32(const TrsvPlan &plan, const DBuf &A, const DBuf &desc, const DBuf &dinv,
                    const DBuf &dinv_off, float *x, bool upper, const ApplyWork &w, int m,
                    int64_t ldx) {
  if (&plan == &plan_rr && !sub_plans.empty()) {
    for (const TrsvPlan &pq : sub_plans)
      HIPCHK(trsv_blocked<float>(stream, A.as<float>(), x, desc.as<MatDesc>(), pq, upper,
                                 dinv.as<float>(), dinv_off.as<int64_t>(), w.trsv_work, w.err, m,
                                 ldx));
    return;
  }
  HIPCHK(trsv_blocked<float>(stream, A.as<float>(), x, desc.as<MatDesc>(), plan, upper,
                             dinv.as<float>(), dinv_off.as<int64_t>(), w.trsv_work, w.err, m, ldx));
}

ApplyWork Solver::own_work() {
  ApplyWork w;
  w.vI = d_vI.as<double>();
  w.vG = d_vG.as<double>();
  w.vG2 = d_vG2.as<double>();
  w.gr = d_gam_r.as<double>();
  w.gz = d_gam_z.as<double>();
  w.vR = d_vR.as<double>();
  w.vR2 = d_vR2.as<double>();
  w.vP = d_vP.as<double>();
  w.vc = d_vc.as<double>();
  w.scr = d_scr.as<double>();
  w.vR32 = d_vR32.as<float>();
  w.mf_upd = nullptr;  // the interior elimination's own vectors
  w.mf_zp = nullptr;
  w.trsv_work = d_work_i.as<int>();
  w.err = d_status.as<int>() + 2 * L.nsub + 1;
  w.cols = kMaxRhs;
  return w;
}

namespace {
constexpr int kWorkSegments = 15;
// segment sizes of a work set in the order of ApplyWork's members, in bytes,
// each rounded up to 256
std::vector<size_t> work_segments(const Layout &L, int64_t scr, int64_t trsv_ints, int64_t upd,
                                  int64_t zp, bool fp32) {
  auto al = [](size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; };
  const size_t d = sizeof(double);
  return {al(d * L.sumI), al(d * L.sumG), al(d * L.sumG), al(d * L.n_gamma), al(d * L.n_gamma),
          al(d * L.sumR), al(d * L.sumR), al(d * L.sumP), al(d * L.n_coarse), al(d * scr),
          al(fp32 ? sizeof(float) * L.sumR : 0), al(d * upd), al(d * zp),
          al(sizeof(int) * trsv_ints), al(sizeof(int))};
}
}  // namespace

size_t Solver::work_bytes() const {
  size_t t = 0;
  for (size_t b : work_segments(L, scr_elems,
                                (int64_t)(d_work_i.bytes / sizeof(int)), mf.upd_elems(),
                                mf.zp_elems(), factor_precision == 32))
    t += b;
  return t;
}

ApplyWork Solver::carve_work(void *base) const {
  const auto seg = work_segments(L, scr_elems,
                                 (int64_t)(d_work_i.bytes / sizeof(int)), mf.upd_elems(),
                                 mf.zp_elems(), factor_precision == 32);
  char *p = (char *)base;
  void *q[kWorkSegments];
  for (int k = 0; k < kWorkSegments; ++k) {
    q[k] = p;
    p += seg[k];
  }
  ApplyWork w;
  w.vI = (double *)q[0];
  w.vG = (double *)q[1];
  w.vG2 = (double *)q[2];
  w.gr = (double *)q[3];
  w.gz = (double *)q[4];
  w.vR = (double *)q[5];
  w.vR2 = (double *)q[6];
  w.vP = (double *)q[7];
  w.vc = (double *)q[8];
  w.scr = (double *)q[9];
  w.vR32 = (float *)q[10];
  w.mf_upd = (double *)q[11];
  w.mf_zp = (double *)q[12];
  w.trsv_work = (int *)q[13];
  w.err = (int *)q[14];
  w.cols = 1;
  return w;
}

// interface residuals (gamma vectors, m columns at stride n_gamma) -> z on
// gamma.  Interior values are not produced here.
void Solver::apply_gamma(const double *r, double *z, int m) {
  const ApplyWork w = own_work();
  gather_kernel<<<nblocks(L.sumG), TPB, 0, stream>>>(r, L.n_gamma, d_ifc_gamma.as<int64_t>(),
                                                     d_ifc_delta.as<double>(), w.vG, L.sumG, L.sumG, m);
  HIPCHK(hipGetLastError());
  apply_local(w.vG, z, w, m);
}

void Solver::apply_Tt_vec(double *b, double *scr, int m) {
  if (!n_gx) return;
  vec_pivots_kernel<<<dim3(nblocks(n_gx), m), TPB, 0, stream>>>(b, d_gx.as<GlobXf>(), n_gx, d_pos.as<int>(),
                                                                scr, L.sumG, scr_elems);
  apply_Tt_kernel<<<dim3(nblocks((int64_t)n_gx * 64), m), TPB, 0, stream>>>(
      b, d_gx.as<GlobXf>(), n_gx, d_wmat.as<double>(), d_pos.as<int>(), scr, L.sumG, scr_elems);
  HIPCHK(hipGetLastError());
}

void Solver::apply_T_vec(double *x, double *scr, int m) {
  if (!n_gx) return;
  apply_T_dots_kernel<<<dim3(nblocks((int64_t)n_gk * 64), m), TPB, 0, stream>>>(
      x, d_gx.as<GlobXf>(), d_gk_glob.as<int>(), d_gk_k.as<int>(), n_gk, d_trow.as<double>(),
      d_pos.as<int>(), scr, L.sumG, scr_elems);
  apply_T_store_kernel<<<dim3(nblocks(n_gk), m), TPB, 0, stream>>>(
      x, d_gx.as<GlobXf>(), d_gk_glob.as<int>(), d_gk_k.as<int>(), n_gk, d_pos.as<int>(), scr,
      L.sumG, scr_elems);
  HIPCHK(hipGetLastError());
}

namespace {
// kernel instance for m columns: the smallest of 1, 2, 4, 8 that holds them
inline int col_tile(int m) { return m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : 8; }

template <int M>
void symv_launch(dim3 grid, hipStream_t st, const double *S, const int64_t *offGG, const int *nG,
                 const double *x, const int64_t *offG, int64_t ldx, double *y, double *part,
                 const int64_t *poff, int64_t ldp, int s0, int m) {
  symv_panel_kernel<M><<<grid, SYMV_NT, 0, st>>>(S, offGG, nG, x, offG, ldx, y, part, poff, ldp, s0, m);
}
template <int M>
void gemv_launch(bool trans, dim3 grid, hipStream_t st, const double *A, const int64_t *aoff,
                 const int *rows, const int *cols, const double *x, const int64_t *xoff,
                 int64_t ldx, double *y, const int64_t *yoff, int64_t ldy, int m) {
  if (trans)
    gemv_t_kernel<M><<<grid, TPB, 0, st>>>(A, aoff, rows, cols, x, xoff, ldx, y, yoff, ldy, 1.0, 1.0, m);
  else
    gemv_n_kernel<M><<<grid, TPB, 0, st>>>(A, aoff, rows, cols, x, xoff, ldx, y, yoff, ldy, 1.0, 1.0, m);
}
}  // namespace

// q = sum_i R_i^T S_i R_i p on gamma vectors (m columns at stride n_gamma)
void Solver::schur_gamma(const double *p, double *q, int m) {
  hipStream_t st = stream;
  double *vG = d_vG.as<double>(), *vG2 = d_vG2.as<double>();
  gather_kernel<<<nblocks(L.sumG), TPB, 0, st>>>(p, L.n_gamma, d_ifc_gamma.as<int64_t>(), nullptr, vG,
                                                 L.sumG, L.sumG, m);
  if (L.max_nG > 0) {
    // lower triangle of each S_s (read once for all columns), the partial
    // sums for its upper triangle written and read once per column, x read
    // per panel and y written
    const int64_t ldp = (int64_t)symv_parts;
    const double by = bytes_S_sym + m * (2.0 * 8.0 * symv_parts + 16.0 * L.sumG);
    timer.begin(st, "schur_symv", by, 2.0 * (double)L.sGG * m);
    // all substructures in one launch, or (per_sub_launches) one at a time
    const int groups = per_sub_launches ? L.nsub : 1, gsz = per_sub_launches ? 1 : L.nsub;
    for (int g = 0; g < groups; ++g) {
      const int mg = per_sub_launches ? L.nG[g] : L.max_nG;
      if (mg == 0) continue;
      {
        LaunchScope ls(st, "symv_kernel", bytes_S_sym + m * (8.0 * symv_parts + 16.0 * L.sumG),
                       2.0 * (double)L.sGG * m);
        const dim3 grid((mg + 63) / 64, gsz);
        const double *S = d_S.as<double>();
        const int64_t *offGG = d_offGG.as<int64_t>(), *offG = d_offG.as<int64_t>();
        const int *nG = d_nG.as<int>();
        double *part = d_symv_part.as<double>();
        const int64_t *poff = d_symv_off.as<int64_t>();
        switch (col_tile(m)) {
          case 1: symv_launch<1>(grid, st, S, offGG, nG, vG, offG, L.sumG, vG2, part, poff, ldp, g * gsz, m); break;
          case 2: symv_launch<2>(grid, st, S, offGG, nG, vG, offG, L.sumG, vG2, part, poff, ldp, g * gsz, m); break;
          case 4: symv_launch<4>(grid, st, S, offGG, nG, vG, offG, L.sumG, vG2, part, poff, ldp, g * gsz, m); break;
          default: symv_launch<8>(grid, st, S, offGG, nG, vG, offG, L.sumG, vG2, part, poff, ldp, g * gsz, m);
        }
      }
      {
        LaunchScope ls(st, "symv_reduce_kernel", m * (8.0 * symv_parts + 16.0 * L.sumG),
                       (double)symv_parts * m);
        symv_reduce_kernel<<<dim3(nblocks(mg), gsz, m), TPB, 0, st>>>(
            d_nG.as<int>(), d_offG.as<int64_t>(), L.sumG, vG2, d_symv_part.as<double>(),
            d_symv_off.as<int64_t>(), ldp, g * gsz);
      }
    }
    timer.end(st);
  }
  reduce_copies_kernel<<<nblocks(L.n_gamma), TPB, 0, st>>>(vG2, L.sumG, d_gamma_ptr.as<int>(),
                                                           d_gamma_copies.as<int64_t>(), nullptr, q,
                                                           L.n_gamma, L.n_gamma, m, 1.0, 0.0);
  HIPCHK(hipGetLastError());
}

// out[q kScStride] = (a_q, b_q) for the m columns (at strides lda, ldb)
void Solver::dot(const double *a, const double *b, int64_t n, double *out, int m, int64_t lda,
                 int64_t ldb) {
  dot_partial_kernel<<<dim3(DOT_BLOCKS, m), TPB, 0, stream>>>(a, b, n, lda, ldb, d_part.as<double>());
  dot_final_kernel<<<m, TPB, 0, stream>>>(d_part.as<double>(), DOT_BLOCKS, out);
  HIPCHK(hipGetLastError());
}

// interior Dirichlet solve in every substructure: vI <- A_II^-1 vI (m
// columns at stride sumI)
void Solver::interior_solve(double *vI, const ApplyWork *w, int m) {
  mf.solve(stream, vI, w ? w->mf_upd : nullptr, w ? w->mf_zp : nullptr, m, L.sumI);
}

// z = M r for global vectors (Algorithm 2): the interior part of r enters
// through E^T, i.e. the substructure right-hand side has b_I = r_I, which is
// condensed onto the interface before the interface solve; the result is
// extended harmonically.  m <= w.cols columns (r, z at strides ldr, ldz)
// share every read of the factors; a column gets the same bits for every m.
void Solver::apply_global(const double *r, double *z) { apply_global(r, z, own_work()); }

void Solver::apply_global(const double *r, double *z, const ApplyWork &w) {
  apply_global(r, L.n_glob, z, L.n_glob, 1, w);
}

void Solver::apply_global(const double *r, int64_t ldr, double *z, int64_t ldz, int m,
                          const ApplyWork &w) {
  if (!factored) throw StateError("bddc_apply before bddc_factor");
  if (m < 1 || m > w.cols) throw ArgError("apply: more columns than the work vectors hold");
  hipStream_t st = stream;
  double *vI = w.vI, *vG = w.vG;
  double *gr = w.gr, *gz = w.gz;
  // condensation of the interior right-hand side: r_G - sum A_GI A_II^-1 r_I
  gather_kernel<<<nblocks(L.sumI), TPB, 0, st>>>(r, ldr, d_int_gdof.as<int64_t>(), nullptr, vI,
                                                 L.sumI, L.sumI, m);
  interior_solve(vI, &w, m);
  spmv_coupling_kernel<<<nblocks(n_rows), TPB, 0, st>>>(
      d_row_sub.as<int>(), d_row_loc.as<int>(), d_rowptr.as<int64_t>(), d_col.as<int>(),
      d_val.as<double>(), n_rows, d_nI.as<int>(), d_offI.as<int64_t>(), d_offG.as<int64_t>(), vI,
      nullptr, nullptr, vG, 0, m, L.sumI, L.sumG);
  // gamma residual: r_gamma - sum over copies of (A_GI A_II^-1 r_I), where
  // the interior part enters through E^T with weight 1 in its substructure and
  // the condensed part is weighted like the interface entries
  gather_kernel<<<nblocks(L.n_gamma), TPB, 0, st>>>(r, ldr, d_gamma_gdof.as<int64_t>(), nullptr, gr,
                                                    L.n_gamma, L.n_gamma, m);
  HIPCHK(hipGetLastError());
  apply_gamma_condensed(gr, vG, gz, w, m);
  harmonic_extension(gz, z, ldz, w, m);
}

// as apply_gamma, but the local right-hand sides receive the condensed
// interior contribution -A_GI A_II^-1 r_I (already in vG_cond, unweighted)
void Solver::apply_gamma_condensed(const double *r, const double *vG_cond, double *z,
                                   const ApplyWork &w, int m) {
  hipStream_t st = stream;
  // vG2 = delta . R_i r - vG_cond
  double *vG2 = w.vG2;
  gather_kernel<<<nblocks(L.sumG), TPB, 0, st>>>(r, L.n_gamma, d_ifc_gamma.as<int64_t>(),
                                                 d_ifc_delta.as<double>(), vG2, L.sumG, L.sumG, m);
  axpby_kernel<<<nblocks(L.sumG * m), TPB, 0, st>>>(vG2, vG_cond, -1.0, 1.0, L.sumG * m);
  HIPCHK(hipGetLastError());
  apply_local(vG2, z, w, m);
}

// everything of apply_gamma after the weighted gather; b (sum-nG stacks, m
// columns) is consumed
void Solver::apply_local(double *b, double *z, const ApplyWork &w, int m) {
  hipStream_t st = stream;
  const int ns = L.nsub;
  double *vG = b, *vR = w.vR, *vR2 = w.vR2;
  double *vP = w.vP, *vc = w.vc;
  apply_Tt_vec(vG, w.scr, m);
  gather32_kernel<<<nblocks(L.sumR), TPB, 0, st>>>(vG, L.sumG, d_rabs.as<int>(), vR, L.sumR, L.sumR, m);
  gather32_kernel<<<nblocks(L.sumP), TPB, 0, st>>>(vG, L.sumG, d_pabs.as<int>(), vP, L.sumP, L.sumP, m);
  HIPCHK(hipGetLastError());
  if (L.max_np > 0) {
    LaunchScope ls(st, "gemv_t_kernel", 8.0 * ((double)L.sRP + m * (L.sumR + 2.0 * L.sumP)),
                   2.0 * (double)L.sRP * m);
    const dim3 grid(nblocks((int64_t)L.max_np * 64), ns);
    const double *Phi = d_Phi.as<double>();
    const int64_t *offRP = d_offRP.as<int64_t>(), *offR = d_offR.as<int64_t>(), *offP = d_offP.as<int64_t>();
    const int *nr = d_nr.as<int>(), *np = d_np.as<int>();
    switch (col_tile(m)) {
      case 1: gemv_launch<1>(true, grid, st, Phi, offRP, nr, np, vR, offR, L.sumR, vP, offP, L.sumP, m); break;
      case 2: gemv_launch<2>(true, grid, st, Phi, offRP, nr, np, vR, offR, L.sumR, vP, offP, L.sumP, m); break;
      case 4: gemv_launch<4>(true, grid, st, Phi, offRP, nr, np, vR, offR, L.sumR, vP, offP, L.sumP, m); break;
      default: gemv_launch<8>(true, grid, st, Phi, offRP, nr, np, vR, offR, L.sumR, vP, offP, L.sumP, m);
    }
  }
  copy_kernel<<<nblocks(L.sumR * m), TPB, 0, st>>>(vR2, vR, L.sumR * m);
  if (factor_precision == 32) {
    // K_rr solves in FP32 with the scaled factor (K_rr = S^-1 Lt Lt^T S^-1):
    // the vector enters and leaves in FP64, scaled by S on both sides
    float *x32 = w.vR32;
    const double *rsc = d_rscale.as<double>();
    convert_scaled_kernel<double, float><<<dim3(nblocks(L.sumR), m), TPB, 0, st>>>(vR2, x32, rsc, L.sumR);
    HIPCHK(hipGetLastError());
    timer.begin(st, "trsv_local_fwd", bytes_Lrr_tri + 8.0 * L.sumR * m, (double)L.sRR * m);
    trsv32(plan_rr, d_Lrr32, d_descRRvec, d_dinv_rr32, d_dinv_rr_off, x32, false, w, m, L.sumR);
    timer.end(st);
    timer.begin(st, "trsv_local_bwd", bytes_Lrr_tri + 8.0 * L.sumR * m, (double)L.sRR * m);
    trsv32(plan_rr, d_Urr32, d_descRRvec, d_dinv_rr32, d_dinv_rr_off, x32, true, w, m, L.sumR);
    timer.end(st);
    convert_scaled_kernel<float, double><<<dim3(nblocks(L.sumR), m), TPB, 0, st>>>(x32, vR2, rsc, L.sumR);
    HIPCHK(hipGetLastError());
  } else {
    timer.begin(st, "trsv_local_fwd", bytes_Lrr_tri + 16.0 * L.sumR * m, (double)L.sRR * m);
    trsv(plan_rr, d_Lrr, d_descRRvec, d_dinv_rr, d_dinv_rr_off, vR2, false, w, m, L.sumR);
    timer.end(st);
    timer.begin(st, "trsv_local_bwd", bytes_Lrr_tri + 16.0 * L.sumR * m, (double)L.sRR * m);
    trsv(plan_rr, d_Urr, d_descRRvec, d_dinv_rr, d_dinv_rr_off, vR2, true, w, m, L.sumR);
    timer.end(st);
  }
  if (L.n_coarse > 0) {
    reduce_copies_kernel<<<nblocks(L.n_coarse), TPB, 0, st>>>(vP, L.sumP, d_c_ptr.as<int>(),
                                                              d_c_copies.as<int64_t>(), nullptr, vc,
                                                              L.n_coarse, L.n_coarse, m, 1.0, 0.0);
    timer.begin(st, "trsv_coarse", 8.0 * (double)L.n_coarse * L.n_coarse,
                2.0 * L.n_coarse * L.n_coarse * m);
    trsv(plan_c, d_Lc, d_descCvec, d_dinv_c, d_dinv_c_off, vc, false, w, m, L.n_coarse);
    trsv(plan_c, d_Uc, d_descCvec, d_dinv_c, d_dinv_c_off, vc, true, w, m, L.n_coarse);
    timer.end(st);
    gather32_kernel<<<nblocks(L.sumP), TPB, 0, st>>>(vc, L.n_coarse, d_pcid.as<int>(), vP, L.sumP,
                                                     L.sumP, m);
    if (L.max_nr > 0) {
      LaunchScope ls(st, "gemv_n_kernel", 8.0 * ((double)L.sRP + m * (L.sumP + 2.0 * L.sumR)),
                     2.0 * (double)L.sRP * m);
      const dim3 grid(nblocks(L.max_nr), ns);
      const double *Phi = d_Phi.as<double>();
      const int64_t *offRP = d_offRP.as<int64_t>(), *offR = d_offR.as<int64_t>(), *offP = d_offP.as<int64_t>();
      const int *nr = d_nr.as<int>(), *np = d_np.as<int>();
      switch (col_tile(m)) {
        case 1: gemv_launch<1>(false, grid, st, Phi, offRP, nr, np, vP, offP, L.sumP, vR2, offR, L.sumR, m); break;
        case 2: gemv_launch<2>(false, grid, st, Phi, offRP, nr, np, vP, offP, L.sumP, vR2, offR, L.sumR, m); break;
        case 4: gemv_launch<4>(false, grid, st, Phi, offRP, nr, np, vP, offP, L.sumP, vR2, offR, L.sumR, m); break;
        default: gemv_launch<8>(false, grid, st, Phi, offRP, nr, np, vP, offP, L.sumP, vR2, offR, L.sumR, m);
      }
    }
  }
  scatter32_kernel<<<nblocks(L.sumR), TPB, 0, st>>>(vR2, L.sumR, d_rabs.as<int>(), vG, L.sumG, L.sumR, m);
  scatter32_kernel<<<nblocks(L.sumP), TPB, 0, st>>>(vP, L.sumP, d_pabs.as<int>(), vG, L.sumG, L.sumP, m);
  apply_T_vec(vG, w.scr, m);
  reduce_copies_kernel<<<nblocks(L.n_gamma), TPB, 0, st>>>(vG, L.sumG, d_gamma_ptr.as<int>(),
                                                           d_gamma_copies.as<int64_t>(),
                                                           d_ifc_delta.as<double>(), z, L.n_gamma,
                                                           L.n_gamma, m, 1.0, 0.0);
  HIPCHK(hipGetLastError());
}

// global z from interface values zg: z_G = zg, z_I = -A_II^-1 A_IG zg
void Solver::harmonic_extension(const double *zg, double *z, int64_t ldz, const ApplyWork &w, int m) {
  hipStream_t st = stream;
  double *vI = w.vI, *vG = w.vG;
  scatter_gamma(zg, z, ldz, m);
  gather_kernel<<<nblocks(L.sumG), TPB, 0, st>>>(zg, L.n_gamma, d_ifc_gamma.as<int64_t>(), nullptr, vG,
                                                 L.sumG, L.sumG, m);
  spmv_coupling_kernel<<<nblocks(n_rows), TPB, 0, st>>>(
      d_row_sub.as<int>(), d_row_loc.as<int>(), d_rowptr.as<int64_t>(), d_col.as<int>(),
      d_val.as<double>(), n_rows, d_nI.as<int>(), d_offI.as<int64_t>(), d_offG.as<int64_t>(),
      nullptr, vG, vI, nullptr, 1, m, L.sumI, L.sumG);
  HIPCHK(hipGetLastError());
  interior_solve(vI, &w, m);
  axpby_kernel<<<nblocks(L.sumI * m), TPB, 0, st>>>(vI, vI, 0.0, -1.0, L.sumI * m);
  scatter_interior(vI, z, ldz, m);
}

void Solver::scatter_gamma(const double *zg, double *z, int64_t ldz, int m) {
  // z[gamma_gdof[k]] = zg[k]
  scatter64(zg, L.n_gamma, d_gamma_gdof.as<int64_t>(), L.n_gamma, z, ldz, m);
}

void Solver::scatter_interior(const double *vI, double *z, int64_t ldz, int m) {
  scatter64(vI, L.sumI, d_int_gdof.as<int64_t>(), L.sumI, z, ldz, m);
}

namespace {
__global__ void scatter64_kernel(const double *src, int64_t lds, const int64_t *idx, int64_t n,
                                 double *dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i] + blockIdx.y * ldd] = src[i + blockIdx.y * lds];
}
}  // namespace

void Solver::scatter64(const double *src, int64_t lds, const int64_t *idx, int64_t n, double *dst,
                       int64_t ldd, int m) {
  if (n <= 0) return;
  scatter64_kernel<<<dim3(nblocks(n), m), TPB, 0, stream>>>(src, lds, idx, n, dst, ldd);
  HIPCHK(hipGetLastError());
}

// PCG on the reduced problem (Remark after Lemma 1: zero interface start,
// interior Dirichlet solves, residuals vanish in the interiors).
// One PCG iteration on the interface for m columns in lock step, all scalars
// on the device (see pcg_check_kernel); launched eagerly or captured as a
// graph.
void Solver::pcg_iteration(int m) {
  hipStream_t st = stream;
  const int64_t ng = L.n_gamma;
  double *r = d_gam_r.as<double>(), *z = d_gam_z.as<double>(), *p = d_gam_p.as<double>();
  double *q = d_gam_q.as<double>(), *x = d_gam_x.as<double>();
  double *sc = d_sc.as<double>();
  int *ctl = d_pcg_ctl.as<int>();
  schur_gamma(p, q, m);
  dot(p, q, ng, sc + 1, m, ng, ng);
  pcg_alpha_kernel<<<1, 64, 0, st>>>(sc, d_alphas.as<double>(), ctl, m);
  pcg_update_kernel<<<dim3(nblocks(ng), m), TPB, 0, st>>>(x, r, p, q, sc, ctl, ng);
  dot(r, r, ng, sc + 2, m, ng, ng);
  pcg_check_kernel<<<1, 64, 0, st>>>(sc, ctl, d_pcg_hist.as<double>(), m);
  const int flexible = factor_precision == 32 ? 1 : 0;
  if (flexible) dot(r, z, ng, sc + 11, m, ng, ng);
  apply_gamma(r, z, m);
  dot(r, z, ng, sc + 5, m, ng, ng);
  pcg_beta_kernel<<<1, 64, 0, st>>>(sc, d_betas.as<double>(), ctl, flexible, m);
  pcg_dir_kernel<<<dim3(nblocks(ng), m), TPB, 0, st>>>(p, z, sc, ctl, ng);
  HIPCHK(hipGetLastError());
}

double Solver::true_residual(const double *f, const double *u, double *rt, double *floor) {
  hipStream_t st = stream;
  double *vI = d_vI.as<double>(), *vI2 = d_vI2.as<double>();
  double *vG = d_vG.as<double>(), *vG2 = d_vG2.as<double>();
  gather_kernel<<<nblocks(L.sumI), TPB, 0, st>>>(u, L.n_glob, d_int_gdof.as<int64_t>(), nullptr, vI,
                                                 L.sumI, L.sumI, 1);
  gather_kernel<<<nblocks(L.sumG), TPB, 0, st>>>(u, L.n_glob, d_ifc_gdof.as<int64_t>(), nullptr, vG,
                                                 L.sumG, L.sumG, 1);
  {
    LaunchScope ls(st, "spmv_local_kernel", 12.0 * (double)nnz + 8.0 * (double)n_rows * 3.0,
                   2.0 * (double)nnz);
    spmv_local_kernel<<<nblocks(n_rows), TPB, 0, st>>>(
        d_row_sub.as<int>(), d_row_loc.as<int>(), d_rowptr.as<int64_t>(), d_col.as<int>(),
        d_val.as<double>(), n_rows, d_nI.as<int>(), d_offI.as<int64_t>(), d_offG.as<int64_t>(), vI,
        vG, vI2, vG2, d_abs_I.as<double>(), d_abs_G.as<double>());
  }
  residual_interior_kernel<<<nblocks(L.sumI), TPB, 0, st>>>(f, d_int_gdof.as<int64_t>(), vI2, rt,
                                                            L.sumI);
  residual_gamma_kernel<<<nblocks(L.n_gamma), TPB, 0, st>>>(
      f, d_gamma_gdof.as<int64_t>(), d_gamma_ptr.as<int>(), d_gamma_copies.as<int64_t>(), vG2, rt,
      L.n_gamma);
  HIPCHK(hipGetLastError());
  double *sc = d_sc.as<double>();
  dot(rt, rt, L.n_glob, sc + 8);
  // the rounding scale of the product: | |A| |u| | over the free dofs, the
  // interface rows summed over their copies (PCG's q is free here)
  double *aG = d_gam_q.as<double>();
  reduce_copies_kernel<<<nblocks(L.n_gamma), TPB, 0, st>>>(d_abs_G.as<double>(), L.sumG,
                                                           d_gamma_ptr.as<int>(),
                                                           d_gamma_copies.as<int64_t>(), nullptr,
                                                           aG, L.n_gamma, L.n_gamma, 1, 1.0, 0.0);
  HIPCHK(hipGetLastError());
  dot(d_abs_I.as<double>(), d_abs_I.as<double>(), L.sumI, sc + 9);
  dot(aG, aG, L.n_gamma, sc + 10);
  double h[3];
  HIPCHK(hipMemcpyAsync(h, sc + 8, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (floor) *floor = std::numeric_limits<double>::epsilon() * std::sqrt(h[1] + h[2]);
  return std::sqrt(h[0]);
}

// PCG to ||r_k|| <= rtol ||r_0|| (Sec. 7), on the interface with the explicit
// Schur complements; then the residual of the assembled system R^T A R u =
// R^T f is computed once with the substructure matrices A_i, with the
// rounding scale of that product, eps || |A| |u| ||: a residual at that
// level is as small as FP64 evaluation can show (with a coefficient contrast
// of 1e6 it exceeds 1e-8 ||r_0|| even for the exact solution rounded to
// FP64).  The explicit operator carries the rounding of the Schur
// complements, so the true residual can sit above the recursive one; while it
// exceeds both rtol ||r_0|| and twice that rounding scale, and keeps halving,
// a correction A d = f - A u is solved by the same PCG to half the absolute
// tolerance and added to u.  Below twice the rounding scale the computed
// residual is mostly the rounding of the product itself, and a correction
// solved from it adds that noise to the solution (measured: at 48^3 with
// contrast 1e6 one such correction moved the solution from 7e-9 to 1.2e-8 of
// the oracle's).
PcgResult Solver::pcg(const double *f, double *u, double rtol, int maxit) {
  std::vector<PcgResult> r = pcg_block(f, L.n_glob, u, L.n_glob, 1, rtol, maxit);
  return r[0];
}

// m right-hand sides (f, u at strides ldf, ldu) solved together: one block
// PCG in lock step (every application of the operator and the preconditioner
// reads the factors once for all columns), then the true-residual check and
// the correction solves column by column.  A column's result has the same
// bits as when solved alone.
std::vector<PcgResult> Solver::pcg_block(const double *f, int64_t ldf, double *u, int64_t ldu,
                                         int m, double rtol, int maxit) {
  auto t0 = std::chrono::steady_clock::now();
  std::vector<double> rt_in(m, rtol), abs_in(m, 0.0);
  std::vector<PcgResult> out = pcg_once(f, ldf, u, ldu, m, rt_in.data(), maxit, abs_in.data());
  double *rt = d_true_r.as<double>(), *du = d_true_d.as<double>();
  for (int c = 0; c < m; ++c) {
    PcgResult &res = out[c];
    if (res.r0 == 0.0) continue;
    const double *fc = f + c * ldf;
    double *uc = u + c * ldu;
    double fl = 0;
    double rn = true_residual(fc, uc, rt, &fl);
    res.true_relres = rn / res.r0;
    res.residual_floor = fl / res.r0;
    const double target = rtol * res.r0;
    while (res.converged && rn > target && rn > 2.0 * fl && res.refinements < kMaxRefine) {
      // half the target, so that the rounding of the update leaves room
      const double half = 0.5 * target;
      PcgResult cr = pcg_once(rt, L.n_glob, du, L.n_glob, 1, &rtol, maxit, &half)[0];
      ++res.refinements;
      res.refine_iters += cr.iters;
      axpby_kernel<<<nblocks(L.n_glob), TPB, 0, stream>>>(uc, du, 1.0, 1.0, L.n_glob);
      HIPCHK(hipGetLastError());
      const double rn_new = true_residual(fc, uc, rt, &fl);
      const bool stalled = rn_new > 0.5 * rn;
      rn = rn_new;
      res.true_relres = rn / res.r0;
      res.residual_floor = fl / res.r0;
      if (stalled) break;
    }
  }
  last_history = out[0].history;
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (PcgResult &res : out) res.seconds = sec;
  return out;
}

std::vector<PcgResult> Solver::pcg_once(const double *f, int64_t ldf, double *u, int64_t ldu, int m,
                                        const double *rtol_in, int maxit, const double *abs_tol) {
  if (!factored) throw StateError("bddc_pcg_solve before bddc_factor");
  if (m < 1 || m > kMaxRhs) throw ArgError("pcg: bad number of columns");
  maxit = std::min(maxit, kMaxIt);
  hipStream_t st = stream;
  auto t0 = std::chrono::steady_clock::now();
  const int64_t ng = L.n_gamma;
  double *vI = d_vI.as<double>(), *vG = d_vG.as<double>();
  double *r = d_gam_r.as<double>(), *z = d_gam_z.as<double>(), *p = d_gam_p.as<double>();
  double *x = d_gam_x.as<double>();
  double *sc = d_sc.as<double>();
  int *ctl = d_pcg_ctl.as<int>();
  // u0: interior solves with zero interface
  gather_kernel<<<nblocks(L.sumI), TPB, 0, st>>>(f, ldf, d_int_gdof.as<int64_t>(), nullptr, vI,
                                                 L.sumI, L.sumI, m);
  interior_solve(vI, nullptr, m);
  // r0 = f_G - sum A_GI u0_I
  spmv_coupling_kernel<<<nblocks(n_rows), TPB, 0, st>>>(
      d_row_sub.as<int>(), d_row_loc.as<int>(), d_rowptr.as<int64_t>(), d_col.as<int>(),
      d_val.as<double>(), n_rows, d_nI.as<int>(), d_offI.as<int64_t>(), d_offG.as<int64_t>(), vI,
      nullptr, nullptr, vG, 0, m, L.sumI, L.sumG);
  gather_kernel<<<nblocks(ng), TPB, 0, st>>>(f, ldf, d_gamma_gdof.as<int64_t>(), nullptr, r, ng,
                                             ng, m);
  reduce_copies_kernel<<<nblocks(ng), TPB, 0, st>>>(vG, L.sumG, d_gamma_ptr.as<int>(),
                                                    d_gamma_copies.as<int64_t>(), nullptr, r, ng, ng,
                                                    m, -1.0, 1.0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * ng * m, st));
  dot(r, r, ng, sc + 2, m, ng, ng);
  std::vector<double> hsc((size_t)kScStride * m);
  HIPCHK(hipMemcpyAsync(hsc.data(), sc, sizeof(double) * hsc.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<PcgResult> out(m);
  PcgInit init{};
  bool any = false;
  for (int c = 0; c < m; ++c) {
    const double r0 = std::sqrt(hsc[(size_t)c * kScStride + 2]);
    out[c].r0 = r0;
    out[c].history.push_back(1.0);
    init.r0[c] = r0;
    init.rtol[c] = (abs_tol[c] > 0 && r0 > 0) ? abs_tol[c] / r0 : rtol_in[c];
    if (r0 > 0) any = true;
  }
  std::vector<int> its(m, 0), convs(m, 0);
  for (int c = 0; c < m; ++c) convs[c] = out[c].r0 == 0.0;
  if (any && maxit > 0) {
    apply_gamma(r, z, m);
    copy_kernel<<<nblocks(ng * m), TPB, 0, st>>>(p, z, ng * m);
    dot(r, z, ng, sc + 0, m, ng, ng);
    pcg_init_kernel<<<1, 64, 0, st>>>(sc, ctl, init, m, maxit);
    HIPCHK(hipGetLastError());
    // per-launch timing records events around launches: then run eagerly
    const bool graphs = use_graphs && timer.mode == 0;
    hipGraphExec_t &exec = pcg_exec[m];
    if (graphs && !exec) {
      // capture one iteration on a private stream (the caller's stream may
      // be the legacy default stream, which cannot be captured)
      if (!cap_stream) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      stream = cap_stream;
      HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
      try {
        pcg_iteration(m);
      } catch (...) {
        hipStreamEndCapture(cap_stream, &g);
        if (g) hipGraphDestroy(g);
        stream = st;
        throw;
      }
      stream = st;
      HIPCHK(hipStreamEndCapture(cap_stream, &g));
      const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      HIPCHK(e);
    }
    if (graphs) {
      if (!pcg_pin) HIPCHK(hipHostMalloc((void **)&pcg_pin, sizeof(int) * 8, hipHostMallocDefault));
      for (hipEvent_t &e : pcg_ev)
        if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      // the host checks iteration k while iteration k + 1 runs (word 0:
      // every column stopped)
      for (int k = 0; k < maxit; ++k) {
        HIPCHK(hipGraphLaunch(exec, st));
        HIPCHK(hipMemcpyAsync(pcg_pin + 4 * (k & 1), ctl, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(pcg_ev[k & 1], st));
        if (k > 0) {
          HIPCHK(hipEventSynchronize(pcg_ev[(k - 1) & 1]));
          if (pcg_pin[4 * ((k - 1) & 1)]) break;
        }
      }
    } else {
      for (int k = 0; k < maxit; ++k) {
        pcg_iteration(m);
        int h = 0;
        HIPCHK(hipMemcpyAsync(&h, ctl, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (h) break;
      }
    }
    std::vector<int> h((size_t)kCtl0 + 4 * m);
    HIPCHK(hipMemcpyAsync(h.data(), ctl, sizeof(int) * h.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int c = 0; c < m; ++c) {
      its[c] = h[kCtl0 + 4 * c + 1];
      convs[c] = h[kCtl0 + 4 * c + 2] != 0;
      const int it = its[c];
      if (it > 0) {
        std::vector<double> hist(it + 1);
        HIPCHK(hipMemcpyAsync(hist.data(), d_pcg_hist.as<double>() + (size_t)c * (kMaxIt + 2),
                              sizeof(double) * (it + 1), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int k = 1; k <= it; ++k) out[c].history.push_back(hist[k]);
        out[c].relres = hist[it];
      }
    }
  }
  // u: interface from x, interiors A_II^-1 (f_I - A_IG x)
  scatter_gamma(x, u, ldu, m);
  gather_kernel<<<nblocks(L.sumG), TPB, 0, st>>>(x, ng, d_ifc_gamma.as<int64_t>(), nullptr, vG, L.sumG,
                                                 L.sumG, m);
  spmv_coupling_kernel<<<nblocks(n_rows), TPB, 0, st>>>(
      d_row_sub.as<int>(), d_row_loc.as<int>(), d_rowptr.as<int64_t>(), d_col.as<int>(),
      d_val.as<double>(), n_rows, d_nI.as<int>(), d_offI.as<int64_t>(), d_offG.as<int64_t>(),
      nullptr, vG, d_vI2.as<double>(), nullptr, 1, m, L.sumI, L.sumG);
  gather_kernel<<<nblocks(L.sumI), TPB, 0, st>>>(f, ldf, d_int_gdof.as<int64_t>(), nullptr, vI,
                                                 L.sumI, L.sumI, m);
  axpby_kernel<<<nblocks(L.sumI * m), TPB, 0, st>>>(vI, d_vI2.as<double>(), -1.0, 1.0, L.sumI * m);
  HIPCHK(hipGetLastError());
  interior_solve(vI, nullptr, m);
  scatter_interior(vI, u, ldu, m);
  // Lanczos coefficients
  for (int c = 0; c < m; ++c) {
    PcgResult &res = out[c];
    const int it = its[c];
    const bool conv = convs[c] != 0;
    const int na = conv ? it : std::max(0, it - 1);
    res.alphas.resize(na);
    res.betas.resize(std::max(0, na - 1));
    if (na > 0)
      HIPCHK(hipMemcpyAsync(res.alphas.data(), d_alphas.as<double>() + (size_t)c * (kMaxIt + 1),
                            sizeof(double) * na, hipMemcpyDeviceToHost, st));
    if (na > 1)
      HIPCHK(hipMemcpyAsync(res.betas.data(), d_betas.as<double>() + (size_t)c * (kMaxIt + 1),
                            sizeof(double) * (na - 1), hipMemcpyDeviceToHost, st));
    res.iters = it;
    res.converged = conv;
  }
  int herr[2];
  HIPCHK(hipMemcpyAsync(herr, d_status.as<int>() + 2 * L.nsub + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (herr[0]) throw DeviceError("triangular solve wait bound exceeded");
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (PcgResult &res : out) {
    lanczos_extremes(res.alphas, res.betas, res.lmin, res.lmax);
    res.seconds = sec;
  }
  last_history = out[0].history;
  timer.collect();
  return out;
}

double Solver::apply_bytes() const {
  double b = 0;
  for (int s = 0; s < L.nsub; ++s) {
    const double nr = L.nr[s], np = L.np[s], ng = L.nG[s];
    const double fb = factor_precision == 32 ? 4.0 : 8.0;
    b += fb * nr * nr + 8.0 * 2 * nr * np + 8.0 * 6 * ng;  // two triangle sweeps, Phi twice, vectors
  }
  b += 8.0 * (double)L.n_coarse * L.n_coarse;
  return b;
}

double Solver::iter_bytes() const {
  // the Schur operator reads the lower triangles (diagonal blocks whole) and
  // writes and reads its partial sums once
  return apply_bytes() + bytes_S_sym + 16.0 * symv_parts;
}

// extreme eigenvalues of the CG-Lanczos tridiagonal matrix by Sturm
// bisection: diag_j = 1/a_j + b_{j-1}/a_{j-1}, off_j = sqrt(b_j)/a_j
void lanczos_extremes(const std::vector<double> &a, const std::vector<double> &b, double &lmin,
                      double &lmax) {
  const int k = (int)a.size();
  if (k == 0) {
    lmin = lmax = NAN;
    return;
  }
  std::vector<double> d(k), e2(k, 0.0);
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / a[j] + (j > 0 ? b[j - 1] / a[j - 1] : 0.0);
    if (j < k - 1) {
      const double o = std::sqrt(b[j]) / a[j];
      e2[j] = o * o;
    }
  }
  double lo = d[0], hi = d[0];
  for (int j = 0; j < k; ++j) {
    const double r = (j > 0 ? std::sqrt(e2[j - 1]) : 0) + (j < k - 1 ? std::sqrt(e2[j]) : 0);
    lo = std::min(lo, d[j] - r);
    hi = std::max(hi, d[j] + r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int j = 1; j < k; ++j) {
      if (q == 0) q = 1e-300;
      q = d[j] - x - e2[j - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  auto kth = [&](int idx) {  // idx-th smallest (0-based)
    double a0 = lo, b0 = hi;
    for (int it = 0; it < 200 && b0 - a0 > 1e-15 * std::max(std::fabs(a0), std::fabs(b0)); ++it) {
      const double m = 0.5 * (a0 + b0);
      if (count_below(m) > idx)
        b0 = m;
      else
        a0 = m;
    }
    return 0.5 * (a0 + b0);
  };
  lmin = kth(0);
  lmax = kth(k - 1);
}

}  // namespace bddc
