// Multifrontal elimination of the substructure interiors on the device
// (structure in multifrontal.h / multifrontal.cpp).
//
// Factorization, deepest fronts first, all substructures batched per depth:
//   assemble   U <- the rows of the substructure matrices owned by each front
//   pull       U, C += the children's contribution blocks (each parent entry
//              sums its children in a fixed order: deterministic, no atomics)
//   potrf      F11 = L11 L11^T                     (MFMA, dense.hip)
//   trsm       F12 <- L11^-1 F12                    (MFMA)
//   gemm       C <- C - F12^T F12, lower triangle   (MFMA)
// and at the top the interface Schur complements S_i pull the contributions
// of their top fronts.  Solves run front by front: forward (deepest first)
// with update vectors pulled by the parents, backward (top first) reading
// the already solved ancestors.
#include "multifrontal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "solver.h"

namespace bddc {

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess)                                                            \
      throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));             \
  } while (0)

namespace {

constexpr int TPB = 256;
constexpr int TB = 64;  // block size of the in-front triangular solves

// one-sided symmetric read of a contribution block stored in its lower triangle
__device__ __forceinline__ double csym(const double *C, int b, int i, int j) {
  return i >= j ? C[i + (int64_t)j * b] : C[j + (int64_t)i * b];
}

__global__ void mf_assemble_kernel(const int64_t *dst, const double *val, int64_t nnz, double *U) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int64_t d = dst[k];
  if (d >= 0) U[d] = val[k];
}

// Fronts ids[f] of a depth: U += the children's contributions (U holds the
// assembled rows already); the lower triangle of C = the children's
// contributions (zero for a leaf), so C needs no clearing.  A flat launch:
// front f owns the blocks [boff[f], boff[f+1]) (offsets relative to the
// depth's list, block b of the launch is b + base), PULL_CHUNK elements of its
// U and C blocks per launch block.
constexpr int PULL_ITEMS = 4;
constexpr int PULL_CHUNK = TPB * PULL_ITEMS;
__global__ void mf_pull_kernel(const MfFront *F, const int *ids, const int *child_ids,
                               const int *pmap, double *U, double *C, const int64_t *boff, int nf,
                               int64_t base) {
  const int64_t blk = blockIdx.x + base;
  int lo = 0, hi = nf;  // boff[lo] <= blk < boff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= blk)
      lo = mid;
    else
      hi = mid;
  }
  const MfFront f = F[ids[lo]];
  const int p = f.p, b = f.b, fs = p + b;
  // a front's blocks hold well under 2^31 entries: 32-bit index arithmetic
  // (a 64-bit division costs several times a 32-bit one)
  const int nu = f.n_child > 0 ? p * fs : 0, ntot = nu + b * b;
  const int e0 = (int)(blk - boff[lo]) * PULL_CHUNK + threadIdx.x;
  // the items' positions first, then per child all their index loads and
  // then all their value loads, so that a thread's loads are in flight
  // together (the sum over the children keeps its order)
  int pr[PULL_ITEMS], pc[PULL_ITEMS];
  bool ok[PULL_ITEMS];
#pragma unroll
  for (int it = 0; it < PULL_ITEMS; ++it) {
    const int e = e0 + it * TPB;
    ok[it] = e < ntot;
    pr[it] = pc[it] = 0;
    if (!ok[it]) continue;
    if (e < nu) {
      pr[it] = e % p;
      pc[it] = e / p;
    } else {
      const int e2 = e - nu;
      const int r = e2 % b, c = e2 / b;
      ok[it] = r >= c;
      pr[it] = p + r;
      pc[it] = p + c;
    }
  }
  double acc[PULL_ITEMS];
#pragma unroll
  for (int it = 0; it < PULL_ITEMS; ++it) acc[it] = 0;
  for (int ci = 0; ci < f.n_child; ++ci) {
    const MfFront ch = F[child_ids[f.child_ptr + ci]];
    const int *pm = pmap + ch.pmap_off;
    const double *Cc = C + ch.c_off;
    int ii[PULL_ITEMS], jj[PULL_ITEMS];
#pragma unroll
    for (int it = 0; it < PULL_ITEMS; ++it) {
      ii[it] = ok[it] ? pm[pr[it]] : -1;
      jj[it] = ok[it] ? pm[pc[it]] : -1;
    }
    double v[PULL_ITEMS];
#pragma unroll
    for (int it = 0; it < PULL_ITEMS; ++it)
      v[it] = (ii[it] >= 0 && jj[it] >= 0) ? csym(Cc, ch.b, ii[it], jj[it]) : 0.0;
#pragma unroll
    for (int it = 0; it < PULL_ITEMS; ++it)
      if (ii[it] >= 0 && jj[it] >= 0) acc[it] += v[it];
  }
#pragma unroll
  for (int it = 0; it < PULL_ITEMS; ++it) {
    const int e = e0 + it * TPB;
    if (!ok[it]) continue;
    if (e < nu)
      U[f.u_off + e] += acc[it];
    else
      C[f.c_off + (e - nu)] = acc[it];
  }
}

// S_s (lower) += the contributions of substructure s's top fronts
__global__ void mf_root_pull_kernel(const MfFront *F, const int *root_ptr, const int *root_ids,
                                    const int *pmap, const double *C, double *S,
                                    const int64_t *offGG, const int *nG, int s0) {
  const int s = blockIdx.y + s0;
  const int ng = nG[s];
  const int r0 = root_ptr[s], r1 = root_ptr[s + 1];
  if (r0 == r1) return;
  const int nn = ng * ng;  // interface blocks hold well under 2^31 entries
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += gridDim.x * blockDim.x) {
    const int r = e % ng, c = e / ng;
    if (r < c) continue;
    double acc = 0;
    for (int ri = r0; ri < r1; ++ri) {
      const MfFront ch = F[root_ids[ri]];
      const int i = pmap[ch.pmap_off + r], j = pmap[ch.pmap_off + c];
      if (i >= 0 && j >= 0) acc += csym(C + ch.c_off, ch.b, i, j);
    }
    S[offGG[s] + e] += acc;
  }
}

// z <- L^-1 z, L (n x n lower, column-major, ld) in global memory, z in LDS;
// Di: inverses of L's TB x TB diagonal blocks (block k at Di + k TB^2, ld TB).
// Per block: the diagonal block is applied through its inverse (a product,
// no sequential substitution), then the rows below are updated.
__device__ void lower_solve(const double *L, int ld, int n, const double *Di, double *z,
                            double *tmp) {
  const int tid = threadIdx.x;
  for (int jb = 0, kb = 0; jb < n; jb += TB, ++kb) {
    const int nb = min(TB, n - jb);
    const double *D = Di + (int64_t)kb * TB * TB;
    if (tid < nb) {
      double y = 0;
      for (int c = 0; c <= tid; ++c) y += D[tid + c * TB] * z[jb + c];
      tmp[tid] = y;
    }
    __syncthreads();
    if (tid < nb) z[jb + tid] = tmp[tid];
    __syncthreads();
    for (int r = jb + nb + tid; r < n; r += blockDim.x) {
      double acc = 0;
      for (int k = 0; k < nb; ++k) acc += L[r + (int64_t)(jb + k) * ld] * z[jb + k];
      z[r] -= acc;
    }
    __syncthreads();
  }
}

// x <- L^-T x (same storage)
__device__ void upper_solve(const double *L, int ld, int n, const double *Di, double *x,
                            double *tmp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  const int nblk = (n + TB - 1) / TB;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int jb = bi * TB, nb = min(TB, n - jb);
    // rows of the block minus the contributions of the solved rows below it
    for (int i = wave; i < nb; i += nwave) {
      double acc = 0;
      const double *col = L + (int64_t)(jb + i) * ld;
      for (int m = jb + nb + lane; m < n; m += 64) acc += col[m] * x[m];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (lane == 0) x[jb + i] -= acc;
    }
    __syncthreads();
    // x_block = D^-T x_block
    const double *D = Di + (int64_t)bi * TB * TB;
    if (tid < nb) {
      double y = 0;
      for (int c = tid; c < nb; ++c) y += D[c + tid * TB] * x[jb + c];
      tmp[tid] = y;
    }
    __syncthreads();
    if (tid < nb) x[jb + tid] = tmp[tid];
    __syncthreads();
  }
}

// Several right-hand sides: work-group -> (logical block b, column q).  The
// m columns of a logical block are consecutive logical ids; with m > 1 the
// grid is padded to a multiple of 8 and logical ids are laid out so that
// consecutive ones run on one XCD (work-groups go to the 8 XCDs in turn), so
// the columns of a front read its factor through one L2.  Column q's vectors
// sit at vI + q ldI, upd + q upd_n, zp + q zp_n.
__device__ __forceinline__ bool col_block(int nlog, int m, int &b, int &q) {
  int id = blockIdx.x;
  if (m > 1) id = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  if (id >= nlog * m) return false;
  b = id / m;
  q = id % m;
  return true;
}

// forward solve of one depth, pivots: one work-group per front; the
// right-hand side at the pivots (plus the children's updates) goes through
// L11^-1 and the result z is written to the pivots of vI and to zp
// (p values per front at piv_off)
__global__ __launch_bounds__(256) void mf_fwd_kernel(const MfFront *F, const int *ids,
                                                     const int *child_ids, const int *pmap,
                                                     const int64_t *piv, const double *U,
                                                     const double *dinv, const int64_t *dinv_off,
                                                     const double *upd, double *vI, double *zp,
                                                     int nf, int m, int64_t ldI, int64_t upd_n,
                                                     int64_t zp_n) {
  extern __shared__ double z[];
  __shared__ double tmp[TB];
  int fi, q;
  if (!col_block(nf, m, fi, q)) return;
  upd += q * upd_n;
  vI += q * ldI;
  zp += q * zp_n;
  const MfFront f = F[ids[fi]];
  const int p = f.p, tid = threadIdx.x;
  for (int j = tid; j < p; j += blockDim.x) {
    double v = vI[piv[f.piv_off + j]];
    for (int ci = 0; ci < f.n_child; ++ci) {
      const MfFront ch = F[child_ids[f.child_ptr + ci]];
      const int k = pmap[ch.pmap_off + j];
      if (k >= 0) v += upd[ch.upd_off + k];
    }
    z[j] = v;
  }
  __syncthreads();
  if (p > 0) lower_solve(U + f.u_off, p, p, dinv + dinv_off[ids[fi]], z, tmp);
  for (int j = tid; j < p; j += blockDim.x) {
    vI[piv[f.piv_off + j]] = z[j];
    zp[f.piv_off + j] = z[j];
  }
}

// forward solve of one depth, boundary: the update each front passes to its
// parent, its children's updates at the boundary minus F12^T z; work-group
// (front, 64-column chunk of the boundary), four columns per wave step
__global__ __launch_bounds__(256) void mf_fupd_kernel(const MfFront *F, const int *ids, int nchunk,
                                                      const int *child_ids, const int *pmap,
                                                      const double *U, const double *zp,
                                                      double *upd, int nf, int m, int64_t upd_n,
                                                      int64_t zp_n) {
  extern __shared__ double z[];
  int lb, q;
  if (!col_block(nf * nchunk, m, lb, q)) return;
  upd += q * upd_n;
  zp += q * zp_n;
  const int fi = lb / nchunk, i_lo = (lb % nchunk) * 64;
  const MfFront f = F[ids[fi]];
  const int p = f.p, b = f.b, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (i_lo >= b) return;
  for (int j = tid; j < p; j += blockDim.x) z[j] = zp[f.piv_off + j];
  __syncthreads();
  const double *Uf = U + f.u_off;
  const int i_hi = min(b, i_lo + 64);
  for (int i0 = i_lo + 4 * wave; i0 < i_hi; i0 += 16) {
    double acc[4] = {0, 0, 0, 0};
    for (int j = lane; j < p; j += 64) {
      const double zj = z[j];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (i0 + t < i_hi) acc[t] += Uf[j + (int64_t)(p + i0 + t) * p] * zj;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      for (int off = 32; off > 0; off >>= 1) acc[t] += __shfl_xor(acc[t], off, 64);
    if (lane < 4 && i0 + lane < i_hi) {
      const int i = i0 + lane;
      double v = -(lane == 0 ? acc[0] : lane == 1 ? acc[1] : lane == 2 ? acc[2] : acc[3]);
      for (int ci = 0; ci < f.n_child; ++ci) {
        const MfFront ch = F[child_ids[f.child_ptr + ci]];
        const int k = pmap[ch.pmap_off + p + i];
        if (k >= 0) v += upd[ch.upd_off + k];
      }
      upd[f.upd_off + i] = v;
    }
  }
}

// backward solve of one depth, boundary product: zp <- y_p - F12 x_b for the
// pivot rows of each front (interface boundary values are zero: pure
// interior solve); work-group (front, 64-row chunk), lane = row, the four
// waves take quarters of the boundary and are summed in a fixed order
__global__ __launch_bounds__(256) void mf_bprod_kernel(const MfFront *F, const int *ids, int nchunk,
                                                       const int64_t *piv, const int64_t *bnd,
                                                       const double *U, const double *vI,
                                                       double *zp, int nf, int m, int64_t ldI,
                                                       int64_t zp_n) {
  extern __shared__ double xb[];
  __shared__ double part[4][64];
  int lb, col;
  if (!col_block(nf * nchunk, m, lb, col)) return;
  vI += col * ldI;
  zp += col * zp_n;
  const int fi = lb / nchunk, j_lo = (lb % nchunk) * 64;
  const MfFront f = F[ids[fi]];
  const int p = f.p, b = f.b, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (j_lo >= p) return;
  for (int i = tid; i < b; i += blockDim.x) {
    const int64_t g = bnd[f.bnd_off + i];
    xb[i] = g >= 0 ? vI[g] : 0.0;
  }
  __syncthreads();
  const double *Uf = U + f.u_off;
  const int j = j_lo + lane;
  const int q = (b + 3) / 4, i_lo = wave * q, i_hi = min(b, i_lo + q);
  double a0 = 0, a1 = 0;
  if (j < p) {
    int i = i_lo;
    for (; i + 1 < i_hi; i += 2) {
      a0 += Uf[j + (int64_t)(p + i) * p] * xb[i];
      a1 += Uf[j + (int64_t)(p + i + 1) * p] * xb[i + 1];
    }
    if (i < i_hi) a0 += Uf[j + (int64_t)(p + i) * p] * xb[i];
  }
  part[wave][lane] = a0 + a1;
  __syncthreads();
  if (wave == 0 && j < p)
    zp[f.piv_off + j] =
        vI[piv[f.piv_off + j]] - ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]));
}

// backward solve of one depth, pivots: x_p = L11^-T zp (zp from
// mf_bprod_kernel); one work-group per front
__global__ __launch_bounds__(256) void mf_bwd_kernel(const MfFront *F, const int *ids,
                                                     const int64_t *piv, const double *U,
                                                     const double *dinv, const int64_t *dinv_off,
                                                     const double *zp, double *vI, int nf, int m,
                                                     int64_t ldI, int64_t zp_n) {
  extern __shared__ double x[];
  __shared__ double tmp[TB];
  int fi, q;
  if (!col_block(nf, m, fi, q)) return;
  zp += q * zp_n;
  vI += q * ldI;
  const MfFront f = F[ids[fi]];
  const int p = f.p, tid = threadIdx.x;
  for (int j = tid; j < p; j += blockDim.x) x[j] = zp[f.piv_off + j];
  __syncthreads();
  if (p > 0) upper_solve(U + f.u_off, p, p, dinv + dinv_off[ids[fi]], x, tmp);
  for (int j = tid; j < p; j += blockDim.x) vI[piv[f.piv_off + j]] = x[j];
}

template <class T>
DBuf upload(DevAlloc &A, hipStream_t st, const std::vector<T> &v) {
  DBuf b;
  b.bytes = std::max<size_t>(v.size() * sizeof(T), 8);
  b.p = A.get(b.bytes);
  if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return b;
}

DBuf zeros(DevAlloc &A, hipStream_t st, size_t bytes) {
  DBuf b;
  b.bytes = std::max<size_t>(bytes, 8);
  b.p = A.get(b.bytes);
  HIPCHK(hipMemsetAsync(b.p, 0, b.bytes, st));
  return b;
}

inline unsigned nblocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TPB - 1) / TPB); }

}  // namespace

void MfDevice::release(DevAlloc &A) {
  for (DBuf *b : {&d_fronts_, &d_child_, &d_piv_, &d_bnd_, &d_pmap_, &d_asm_, &d_root_ptr_,
                  &d_root_ids_, &d_U_, &d_C_, &d_upd_, &d_status_, &d_level_ids_, &d_dinv_,
                  &d_dinv_front_, &d_zp_}) {
    if (b->p) A.put(b->p, b->bytes);
    *b = DBuf();
  }
  h_pull_off_.clear();
  for (auto *v : {&d_potrf_, &d_trsm_, &d_gemm_, &d_dinv_off_, &d_dinv_toff_, &d_pull_off_}) {
    for (DBuf &b : *v)
      if (b.p) A.put(b.p, b.bytes);
    v->clear();
  }
  ready = false;
}

size_t MfDevice::bytes() const {
  size_t t = 0;
  for (const DBuf *b : {&d_fronts_, &d_child_, &d_piv_, &d_bnd_, &d_pmap_, &d_asm_, &d_root_ptr_,
                        &d_root_ids_, &d_U_, &d_C_, &d_upd_, &d_status_, &d_level_ids_, &d_dinv_,
                        &d_dinv_front_, &d_zp_})
    t += b->bytes;
  return t;
}

void MfDevice::setup(const Problem &P, const std::vector<int64_t> &offI, DevAlloc &A, hipStream_t st) {
  release(A);
  sym = mf_analyze(P, offI);
  const MfSymbolic &M = sym;
  nnz_ = (int64_t)M.asm_dst.size();
  d_fronts_ = upload(A, st, M.fronts);
  d_child_ = upload(A, st, M.child_ids);
  d_piv_ = upload(A, st, M.piv);
  d_bnd_ = upload(A, st, M.bnd);
  d_pmap_ = upload(A, st, M.pmap);
  d_asm_ = upload(A, st, M.asm_dst);
  d_root_ptr_ = upload(A, st, M.root_ptr);
  d_root_ids_ = upload(A, st, M.root_ids);
  d_U_ = zeros(A, st, sizeof(double) * (size_t)M.u_size);
  d_C_ = zeros(A, st, sizeof(double) * (size_t)M.c_size);
  upd_n_ = std::max<int64_t>(1, M.upd_size);
  d_upd_ = zeros(A, st, sizeof(double) * (size_t)upd_n_ * kMaxCols);
  d_status_ = zeros(A, st, sizeof(int) * (M.fronts.size() + 1));
  // per-depth front lists and batched descriptors
  const int D = M.max_depth;
  std::vector<int> ids;
  level_off_.assign(D + 2, 0);
  h_potrf_.assign(D + 1, {});
  h_trsm_.assign(D + 1, {});
  h_gemm_.assign(D + 1, {});
  max_f_.assign(D + 1, 0);
  max_pb_.assign(D + 1, 0);
  max_p_.assign(D + 1, 0);
  max_b_.assign(D + 1, 0);
  for (int d = 0; d <= D; ++d) {
    level_off_[d] = (int64_t)ids.size();
    for (int t : M.levels[d]) {
      ids.push_back(t);
      const MfFront &f = M.fronts[t];
      max_f_[d] = std::max<int64_t>(max_f_[d], (int64_t)f.p * (f.p + f.b) + (int64_t)f.b * f.b);
      // the extend-add kernels index a front's blocks with 32-bit integers
      if (max_f_[d] >= ((int64_t)1 << 31))
        throw ArgError("a front holds 2^31 entries or more");
      max_pb_[d] = std::max(max_pb_[d], f.p + f.b);
      max_p_[d] = std::max(max_p_[d], f.p);
      max_b_[d] = std::max(max_b_[d], f.b);
      if (f.p == 0) continue;
      h_potrf_[d].push_back(MatDesc{f.u_off, 0, f.p, 0, f.p, f.p});
      if (f.b == 0) continue;
      h_trsm_[d].push_back(MatDesc{f.u_off, f.u_off + (int64_t)f.p * f.p, f.p, f.b, f.p, f.p});
      h_gemm_[d].push_back(GemmDesc{f.u_off + (int64_t)f.p * f.p, f.u_off + (int64_t)f.p * f.p,
                                    f.c_off, f.b, f.b, f.p, f.p, f.p, f.b});
    }
  }
  level_off_[D + 1] = (int64_t)ids.size();
  d_level_ids_ = upload(A, st, ids);
  // per-substructure ranges of every depth's lists
  nsub_ = (int)P.subs.size();
  lvl_lo_.assign(D + 1, std::vector<int>(nsub_ + 1, 0));
  pot_lo_ = lvl_lo_;
  trs_lo_ = lvl_lo_;
  for (int d = 0; d <= D; ++d) {
    std::vector<int> nl(nsub_, 0), npo(nsub_, 0), ntr(nsub_, 0);
    int last = -1;
    for (int t : M.levels[d]) {
      const MfFront &f = M.fronts[t];
      if (f.sub < last) throw ArgError("interior elimination: fronts of a depth not ordered by substructure");
      last = f.sub;
      nl[f.sub]++;
      if (f.p > 0) npo[f.sub]++;
      if (f.p > 0 && f.b > 0) ntr[f.sub]++;
    }
    for (int q = 0; q < nsub_; ++q) {
      lvl_lo_[d][q + 1] = lvl_lo_[d][q] + nl[q];
      pot_lo_[d][q + 1] = pot_lo_[d][q] + npo[q];
      trs_lo_[d][q + 1] = trs_lo_[d][q] + ntr[q];
    }
  }
  // inverses of the diagonal blocks of every front's L11, per depth
  std::vector<std::vector<int64_t>> doff(D + 1);
  int64_t dtot = 0;
  for (int d = 0; d <= D; ++d) {
    const int64_t t = dinv_layout(h_potrf_[d].data(), (int)h_potrf_[d].size(), doff[d]);
    for (auto &o : doff[d]) o += dtot;
    dtot += t;
  }
  d_dinv_ = zeros(A, st, sizeof(double) * (size_t)dtot);
  // trsm entries are the potrf entries with b > 0: their inverse offsets
  for (int d = 0; d <= D; ++d) {
    std::vector<int64_t> toff;
    size_t e = 0;
    for (int t : M.levels[d]) {
      const MfFront &f = M.fronts[t];
      if (f.p == 0) continue;
      if (f.b > 0) toff.push_back(doff[d][e]);
      ++e;
    }
    {
      std::vector<int64_t> bo(M.levels[d].size() + 1, 0);
      for (size_t k = 0; k < M.levels[d].size(); ++k) {
        const MfFront &f = M.fronts[M.levels[d][k]];
        const int64_t ntot = (f.n_child > 0 ? (int64_t)f.p * (f.p + f.b) : 0) + (int64_t)f.b * f.b;
        bo[k + 1] = bo[k] + (ntot + PULL_CHUNK - 1) / PULL_CHUNK;
      }
      if (bo.back() > INT32_MAX) throw ArgError("extend-add: a depth needs 2^31 blocks or more");
      d_pull_off_.push_back(upload(A, st, bo));
      h_pull_off_.push_back(std::move(bo));
    }
    d_potrf_.push_back(upload(A, st, h_potrf_[d]));
    d_trsm_.push_back(upload(A, st, h_trsm_[d]));
    d_gemm_.push_back(upload(A, st, h_gemm_[d]));
    d_dinv_off_.push_back(upload(A, st, doff[d]));
    d_dinv_toff_.push_back(upload(A, st, toff));
  }
  // per front (global id): offset of its diagonal-block inverses (0 if p = 0)
  {
    std::vector<int64_t> fo(M.fronts.size(), 0);
    for (int d = 0; d <= D; ++d) {
      size_t e = 0;
      for (int t : M.levels[d])
        if (M.fronts[t].p > 0) fo[t] = doff[d][e++];
    }
    d_dinv_front_ = upload(A, st, fo);
  }
  // z of every front's pivots between the two launches of a depth
  zp_n_ = std::max<int64_t>(1, (int64_t)M.piv.size());
  d_zp_ = zeros(A, st, sizeof(double) * (size_t)zp_n_ * kMaxCols);
  // the in-front solves keep p values (boundary products: b values) in LDS
  int max_lds = 0;
  for (int d = 1; d <= D; ++d) max_lds = std::max(max_lds, std::max(max_p_[d], max_b_[d]));
  if ((size_t)max_lds * sizeof(double) > 150 * 1024)
    throw ArgError("a front of the interior elimination exceeds the LDS of one work-group");
  if ((size_t)max_lds * sizeof(double) > 64 * 1024)
    for (const void *k : {(const void *)mf_bwd_kernel, (const void *)mf_fwd_kernel,
                          (const void *)mf_fupd_kernel, (const void *)mf_bprod_kernel})
      HIPCHK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(max_lds * sizeof(double))));
  HIPCHK(hipStreamSynchronize(st));
  ready = true;
}

void MfDevice::factor(hipStream_t st, const double *val, int64_t nnz, double *S, const int64_t *offGG,
                      const int *nG, int max_nG, int nsub) {
  if (!ready) throw StateError("interior elimination not set up");
  if (nnz != nnz_) throw ArgError("interior elimination: matrix size changed");
  const MfSymbolic &M = sym;
  double *U = d_U_.as<double>(), *C = d_C_.as<double>();
  const MfFront *F = d_fronts_.as<MfFront>();
  const int *ids = d_level_ids_.as<int>();
  HIPCHK(hipMemsetAsync(d_U_.p, 0, d_U_.bytes, st));
  HIPCHK(hipMemsetAsync(d_status_.p, 0, d_status_.bytes, st));
  {
    LaunchScope ls(st, "mf_assemble_kernel", 20.0 * (double)nnz, 0);
    mf_assemble_kernel<<<nblocks(nnz), TPB, 0, st>>>(d_asm_.as<int64_t>(), val, nnz, U);
    HIPCHK(hipGetLastError());
  }
  int *status = d_status_.as<int>();
  // one depth of fronts: level entries [l0, l1), potrf entries [p0, p1), trsm /
  // gemm entries [t0, t1)
  auto depth = [&](int d, int l0, int l1, int p0, int p1, int t0, int t1) {
    const int nf = l1 - l0;
    if (nf == 0) return;
    const int *lid = ids + level_off_[d] + l0;
    {
      double by = 0;
      if (launch_timing())
        for (int k = l0; k < l1; ++k) {
          const MfFront &f = M.fronts[M.levels[d][k]];
          by += 8.0 * ((double)f.p * (f.p + f.b) + 0.5 * (double)f.b * f.b);
          for (int ci = 0; ci < f.n_child; ++ci) by += 4.0 * M.fronts[M.child_ids[f.child_ptr + ci]].b * 0.5 * M.fronts[M.child_ids[f.child_ptr + ci]].b;
        }
      LaunchScope ls(st, "mf_pull_kernel", by, 0);
      const std::vector<int64_t> &bo = h_pull_off_[d];
      const int64_t nb = bo[l1] - bo[l0];
      if (nb > 0)
        mf_pull_kernel<<<(unsigned)nb, TPB, 0, st>>>(F, lid, d_child_.as<int>(), d_pmap_.as<int>(), U, C,
                                                     d_pull_off_[d].as<int64_t>() + l0, nf, bo[l0]);
      HIPCHK(hipGetLastError());
    }
    const int np = p1 - p0;
    if (np > 0)
      HIPCHK(DenseOps<double>::potrf(st, U, d_potrf_[d].as<MatDesc>() + p0, h_potrf_[d].data() + p0, np,
                                     status + level_off_[d] + p0, d_dinv_.as<double>(),
                                     d_dinv_off_[d].as<int64_t>() + p0));
    const int nt = t1 - t0;
    if (nt > 0) {
      HIPCHK(DenseOps<double>::trsm(st, U, U, d_trsm_[d].as<MatDesc>() + t0, h_trsm_[d].data() + t0, nt,
                                    false, d_dinv_.as<double>(), d_dinv_toff_[d].as<int64_t>() + t0));
      int maxb = 0;
      for (int k = t0; k < t1; ++k) maxb = std::max(maxb, h_gemm_[d][k].M);
      HIPCHK(DenseOps<double>::gemm(st, U, U, C, d_gemm_[d].as<GemmDesc>() + t0, nt, maxb, maxb, true,
                                    false, -1.0, 1.0, true, h_gemm_[d].data() + t0));
    }
  };
  auto root_pull = [&](int s0, int count) {
    if (max_nG <= 0 || count <= 0) return;
    if ((int64_t)max_nG * max_nG >= ((int64_t)1 << 31))  // 32-bit indices in mf_root_pull_kernel
      throw ArgError("an interface of 46341 dofs or more");
    const unsigned gx = (unsigned)std::min<int64_t>(4096, ((int64_t)max_nG * max_nG + TPB - 1) / TPB);
    LaunchScope ls(st, "mf_root_pull_kernel", 0, 0);
    mf_root_pull_kernel<<<dim3(std::max(1u, gx), count), TPB, 0, st>>>(
        F, d_root_ptr_.as<int>(), d_root_ids_.as<int>(), d_pmap_.as<int>(), C, S, offGG, nG, s0);
    HIPCHK(hipGetLastError());
  };
  if (per_entry_launches() && nsub > 1) {
    // unbatched: one substructure at a time, its fronts of a depth batched
    PerEntryOff off;
    for (int q = 0; q < nsub; ++q) {
      for (int d = M.max_depth; d >= 1; --d)
        depth(d, lvl_lo_[d][q], lvl_lo_[d][q + 1], pot_lo_[d][q], pot_lo_[d][q + 1], trs_lo_[d][q],
              trs_lo_[d][q + 1]);
      root_pull(q, 1);
    }
  } else {
    for (int d = M.max_depth; d >= 1; --d)
      depth(d, 0, (int)M.levels[d].size(), 0, (int)h_potrf_[d].size(), 0, (int)h_trsm_[d].size());
    root_pull(0, nsub);
  }
  // pivots
  std::vector<int> hs(M.fronts.size() + 1);
  HIPCHK(hipMemcpyAsync(hs.data(), d_status_.p, sizeof(int) * hs.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int d = 1; d <= M.max_depth; ++d)
    for (size_t e = 0; e < h_potrf_[d].size(); ++e)
      if (hs[level_off_[d] + e]) {
        // batch entry e of depth d: find its front
        int k = 0;
        for (int t : M.levels[d]) {
          if (M.fronts[t].p == 0) continue;
          if (k++ == (int)e)
            throw NotSpdError("interior elimination: non-positive pivot in substructure " +
                              std::to_string(M.fronts[t].sub));
        }
      }
}

void MfDevice::solve(hipStream_t st, double *vI, double *upd_w, double *zp_w, int m, int64_t ldI) {
  if (!ready) throw StateError("interior elimination not set up");
  if (m < 1 || m > kMaxCols) throw ArgError("interior solve: bad number of columns");
  // grid of n logical blocks times m columns (padded to a multiple of 8)
  auto grid = [m](int64_t n) {
    const int64_t g = n * m;
    return (unsigned)(m > 1 ? (g + 7) / 8 * 8 : g);
  };
  const MfSymbolic &M = sym;
  const MfFront *F = d_fronts_.as<MfFront>();
  const int *ids = d_level_ids_.as<int>();
  const double *U = d_U_.as<double>();
  double *upd = upd_w ? upd_w : d_upd_.as<double>();
  // bytes of the pivot (triangle) and boundary (F12) parts of a depth
  auto tri_bytes = [&](int d) {
    double by = 0;
    for (int t : M.levels[d]) {
      const MfFront &f = M.fronts[t];
      by += 8.0 * (0.5 * (double)f.p * (f.p + 1) + 3.0 * f.p);
    }
    return by;
  };
  auto f12_bytes = [&](int d) {
    double by = 0;
    for (int t : M.levels[d]) {
      const MfFront &f = M.fronts[t];
      by += 8.0 * ((double)f.p * f.b + f.p + 2.0 * f.b);
    }
    return by;
  };
  const bool tm = launch_timing() != nullptr;
  double *zp = zp_w ? zp_w : d_zp_.as<double>();
  // forward and backward sweeps over the fronts [l0, l1) of each depth
  auto fwd = [&](int d, int l0, int l1) {
    const int nf = l1 - l0;
    if (nf == 0) return;
    const int *lid = ids + level_off_[d] + l0;
    {
      LaunchScope ls(st, "mf_fwd_kernel", tm ? tri_bytes(d) : 0, 0);
      mf_fwd_kernel<<<grid(nf), TPB, sizeof(double) * std::max(1, max_p_[d]), st>>>(
          F, lid, d_child_.as<int>(), d_pmap_.as<int>(), d_piv_.as<int64_t>(), U,
          d_dinv_.as<double>(), d_dinv_front_.as<int64_t>(), upd, vI, zp, nf, m, ldI, upd_n_,
          zp_n_);
    }
    const int nc = (max_b_[d] + 63) / 64;
    if (nc > 0) {
      LaunchScope ls(st, "mf_fupd_kernel", tm ? f12_bytes(d) : 0, 0);
      mf_fupd_kernel<<<grid((int64_t)nf * nc), TPB, sizeof(double) * std::max(1, max_p_[d]), st>>>(
          F, lid, nc, d_child_.as<int>(), d_pmap_.as<int>(), U, zp, upd, nf, m, upd_n_, zp_n_);
    }
    HIPCHK(hipGetLastError());
  };
  auto bwd = [&](int d, int l0, int l1) {
    const int nf = l1 - l0;
    if (nf == 0) return;
    const int *lid = ids + level_off_[d] + l0;
    const int nc = (max_p_[d] + 63) / 64;
    if (nc > 0) {
      LaunchScope ls(st, "mf_bprod_kernel", tm ? f12_bytes(d) : 0, 0);
      mf_bprod_kernel<<<grid((int64_t)nf * nc), TPB, sizeof(double) * std::max(1, max_b_[d]), st>>>(
          F, lid, nc, d_piv_.as<int64_t>(), d_bnd_.as<int64_t>(), U, vI, zp, nf, m, ldI, zp_n_);
    }
    {
      LaunchScope ls(st, "mf_bwd_kernel", tm ? tri_bytes(d) : 0, 0);
      mf_bwd_kernel<<<grid(nf), TPB, sizeof(double) * std::max(1, max_p_[d]), st>>>(
          F, lid, d_piv_.as<int64_t>(), U, d_dinv_.as<double>(), d_dinv_front_.as<int64_t>(), zp,
          vI, nf, m, ldI, zp_n_);
    }
    HIPCHK(hipGetLastError());
  };
  if (per_entry_launches() && nsub_ > 1) {
    // unbatched: one substructure at a time
    for (int q = 0; q < nsub_; ++q) {
      for (int d = M.max_depth; d >= 1; --d) fwd(d, lvl_lo_[d][q], lvl_lo_[d][q + 1]);
      for (int d = 1; d <= M.max_depth; ++d) bwd(d, lvl_lo_[d][q], lvl_lo_[d][q + 1]);
    }
  } else {
    for (int d = M.max_depth; d >= 1; --d) fwd(d, 0, (int)M.levels[d].size());
    for (int d = 1; d <= M.max_depth; ++d) bwd(d, 0, (int)M.levels[d].size());
  }
}

}  // namespace bddc
