// Batched dense kernels for the substructure factors (gfx950).
//
// GEMM tiles run on the matrix cores: v_mfma_f64_16x16x4f64 in FP64 and
// v_mfma_f32_16x16x4f32 in FP32 (FP32 accumulate).  A work-group of 256
// lanes (4 wave64) owns a 64x64, 128x64, 64x128 or 128x128 tile of C; each
// wave owns a quadrant of 16x16 MFMA blocks.  Operand tiles are staged
// through LDS in K-steps of 16, the next step loaded into registers while the
// current one is multiplied.
// A launch holds only the tiles each entry has (tile maps); in batches too
// large for a map, work-group ids are remapped so that the tiles of one batch
// entry stay on one XCD (consecutive hardware ids are dealt round-robin to the
// 8 XCDs).
//
// Cholesky and multi-RHS triangular solves are blocked with NB = 64 in panels
// of PB block columns: within a panel each block column is updated
// (short-K GEMM), its 64x64 diagonal block factored (one wave) or applied
// through its inverse, and the rest of the panel solved; then one large-K
// GEMM updates everything outside the panel.  The Cholesky runs either one
// launch per step or as one fused launch (tasks with per-entry counters).
// The few-RHS triangular solve used in every preconditioner application is a
// single launch per direction: one work-group per 64-row block, ordered by an
// atomic ticket, waiting on per-block completion flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>

#include <map>
#include <mutex>
#include <tuple>
#include "dense.h"
#include "device.h"

namespace bddc {

namespace {

constexpr int BK = 16;  // K-step of the GEMM tiles
constexpr int NXCD = 8;
constexpr int PB = 8;   // block columns per panel of the blocked Cholesky and TRSM

template <class T>
struct Mfma;
// Output layout of the 16x16x4 MFMA: lane l, item t holds D[row][l % 16] with
// row = (l / 16) + 4 t for FP64 and row = 4 (l / 16) + t for FP32 (A and B:
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] for both).
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int t) { return (lane >> 4) + 4 * t; }
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int t) { return 4 * (lane >> 4) + t; }
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Linear work-group id -> (entry, tile) with all tiles of one entry on the
// same XCD when the grid is a multiple of NXCD.
// Returns false for the padding work-groups past the last entry.
__device__ __forceinline__ bool xcd_remap(int nwg, int tiles_per_entry, int batch, int &entry,
                                          int &tile) {
  int b = blockIdx.x;
  int logical = b;
  if ((nwg % NXCD) == 0) logical = (b % NXCD) * (nwg / NXCD) + (b / NXCD);
  entry = logical / tiles_per_entry;
  tile = logical % tiles_per_entry;
  return entry < batch;
}

// tile (ti, tj), tj <= ti, of the lower triangle from a linear index
__device__ __forceinline__ void lower_tile(int t, int &ti, int &tj) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// Only the tiles each entry has: the host sums every entry's tile count into
// off[0..n] (passed by value with the launch), and work-group ids are split at
// those offsets.  A batch of uneven entries then launches no empty
// work-groups.  Logical tiles are dealt to the XCDs in chunks of kXcdChunk
// consecutive tiles (consecutive hardware ids go round-robin to the 8 XCDs;
// the grid is a multiple of 8 kXcdChunk): a chunk's tiles share operand
// panels in one L2, and every XCD gets a fine-grained mix of all entries, so
// entries whose tiles differ in cost (K) do not leave some XCDs idle at the
// end of a launch (keeping each entry on one XCD measured 4% slower on the
// adaptive selection at the 64^3 size; chunks of 1 to 16 tiles measured the
// same).
// n = 0: not used (the caller falls back to a grid sized by its largest entry).
constexpr int kMaxMapEntries = 480;
struct TileMap {
  int n;
  int off[kMaxMapEntries + 1];
  // xb[NXCD] > 0: XCD x takes the logical tiles [xb[x], xb[x+1]) (split by
  // cost, xcd_balance), the grid being NXCD times the largest share
  int xb[NXCD + 1];
};
constexpr int kXcdChunk = 8;
__device__ __forceinline__ bool map_tile(const TileMap &m, int nwg, int &entry, int &tile) {
  const int b = blockIdx.x;
  int logical = b;
  if (m.xb[NXCD] > 0) {
    const int x = b % NXCD;
    logical = m.xb[x] + b / NXCD;
    if (logical >= m.xb[x + 1]) return false;
  } else if (kXcdChunk > 1 && nwg % (NXCD * kXcdChunk) == 0) {
    const int x = b % NXCD, i = b / NXCD;
    logical = ((i / kXcdChunk) * NXCD + x) * kXcdChunk + (i % kXcdChunk);
  }
  if (logical >= m.off[m.n]) return false;
  int lo = 0, hi = m.n;  // off[lo] <= logical < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (m.off[mid] <= logical)
      lo = mid;
    else
      hi = mid;
  }
  entry = lo;
  tile = logical - m.off[lo];
  return true;
}

// C[m0:m0+TM, n0:n0+TN] = beta*C + alpha*op(A)*op(B), bounds-checked, with
// TM = 32 MT and TN = 32 NT: in each group of four waves, the waves own 2 x 2
// quadrants of MT x NT MFMA blocks of 16 x 16.  Operands go through two LDS
// buffers per group in K-steps of BK: the next step's operands are loaded
// into registers while the current step is multiplied from one buffer, then
// stored into the other, so one barrier per step suffices.  With KS > 1 the
// work-group has KS groups (256 KS threads) that take every KS-th K-step of
// the same tile; their partial products are summed through LDS in group
// order (deterministic) -- more waves per tile where a launch has few tiles
// and long K.  A or B may alias C (in-place products of one tile): every
// operand element a work-group reads lies in its own C tile or is read before
// the tile is written.
// With KS = 1 the epilogue stages C through the operand buffers: a caller
// that uses the LDS again after gemm_tile must synchronize first.
// TAG tells the callers apart: each kernel uses instantiations of its own, so
// that no LDS array is reached from two kernels (such an array is addressed
// through a per-kernel lookup table, which costs registers).
// rmap / cmap (optional): C's row i is row rmap[i] of the storage, column j
// is column cmap[j].  LW: only entries with row >= column are written.
// gemm_tile_s is the same product with its LDS given by the caller (smem,
// gemm_tile_lds<T, MT, NT, KS>() elements), so that one kernel can run tiles
// of several shapes in one buffer.  COH: every global load and store of the
// operands and of C is a device-coherent (agent-scope) access, for products
// whose operands were written by other work-groups of the same launch (the
// fused factorization); otherwise plain accesses.
template <bool COH, class T>
__device__ __forceinline__ T gld(const T *p) {
  if constexpr (COH)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
template <bool COH, class T>
__device__ __forceinline__ void gst(T *p, T v) {
  if constexpr (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

template <class T, int MT, int NT, int KS>
constexpr int gemm_tile_lds() {
  constexpr int TM = 32 * MT, TN = 32 * NT;
  constexpr int SA = BK * (TM + 2), SB = BK * (TN + 2);
  constexpr int PART = 256 * MT * NT * 4;
  constexpr int SOPS = KS * 2 * (SA + SB), SRED = (KS - 1) * PART;
  return SOPS > SRED ? SOPS : SRED;
}

template <class T, bool TA, bool TB, int MT, int NT, int KS = 1, bool LW = false, bool COH = false>
__device__ __forceinline__ void gemm_tile_s(T *smem, const T *A, const T *B, T *C, int M, int N,
                                            int K, int lda, int ldb, int ldc, T alpha, T beta,
                                            int m0, int n0, const int *rmap = nullptr,
                                            const int *cmap = nullptr) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int TM = 32 * MT, TN = 32 * NT;
  constexpr int LA = TM * BK / 256, LB = TN * BK / 256;
  constexpr int SA = BK * (TM + 2), SB = BK * (TN + 2);      // one buffer of A / B
  constexpr int PART = 256 * MT * NT * 4;                     // one group's partial tile
  constexpr int SOPS = KS * 2 * (SA + SB);
  static_assert(KS > 1 || SOPS >= 4 * (16 * MT + 1) * 16, "epilogue staging exceeds the operand buffers");
  const int tid = threadIdx.x % 256, g = threadIdx.x / 256;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  T *As = smem + g * 2 * SA, *Bs = smem + KS * 2 * SA + g * 2 * SB;
  v4 acc[MT][NT];
#pragma unroll
  for (int x = 0; x < MT; ++x)
#pragma unroll
    for (int y = 0; y < NT; ++y) acc[x][y] = v4{0, 0, 0, 0};
  T ra[LA], rb[LB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int it = 0; it < LA; ++it) {
      const int e = tid + it * 256;
      const int r = TA ? e / BK : e % TM, kk = TA ? e % BK : e / TM;
      const int gr = m0 + r, gk = k0 + kk;
      ra[it] = (gr < M && gk < K) ? gld<COH>(TA ? &A[gk + (int64_t)gr * lda] : &A[gr + (int64_t)gk * lda])
                                  : T(0);
    }
#pragma unroll
    for (int it = 0; it < LB; ++it) {
      const int e = tid + it * 256;
      const int c = TB ? e % TN : e / BK, kk = TB ? e / TN : e % BK;
      const int gc = n0 + c, gk = k0 + kk;
      rb[it] = (gc < N && gk < K) ? gld<COH>(TB ? &B[gc + (int64_t)gk * ldb] : &B[gk + (int64_t)gc * ldb])
                                  : T(0);
    }
  };
  auto lstore = [&](int buf) {
    T *as = As + buf * SA, *bs = Bs + buf * SB;
#pragma unroll
    for (int it = 0; it < LA; ++it) {
      const int e = tid + it * 256;
      as[(TA ? e % BK : e / TM) * (TM + 2) + (TA ? e / BK : e % TM)] = ra[it];
    }
#pragma unroll
    for (int it = 0; it < LB; ++it) {
      const int e = tid + it * 256;
      bs[(TB ? e / TN : e % BK) * (TN + 2) + (TB ? e % TN : e / BK)] = rb[it];
    }
  };
  const int nsteps = (K + BK - 1) / BK, rounds = (nsteps + KS - 1) / KS;
  int step = g;  // this group's K-steps: g, g + KS, ...
  if (step < nsteps) {
    gload(step * BK);
    lstore(0);
  }
  __syncthreads();
  int buf = 0;
  for (int it = 0; it < rounds; ++it, step += KS) {
    const bool more = step + KS < nsteps;
    if (more) gload((step + KS) * BK);
    if (step < nsteps) {
      const T *as = As + buf * SA, *bs = Bs + buf * SB;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int k = kk + (lane >> 4), l16 = lane & 15;
        T a[MT], b[NT];
#pragma unroll
        for (int x = 0; x < MT; ++x) a[x] = as[k * (TM + 2) + wr * 16 * MT + 16 * x + l16];
#pragma unroll
        for (int y = 0; y < NT; ++y) b[y] = bs[k * (TN + 2) + wc * 16 * NT + 16 * y + l16];
#pragma unroll
        for (int x = 0; x < MT; ++x)
#pragma unroll
          for (int y = 0; y < NT; ++y) acc[x][y] = Mfma<T>::op(a[x], b[y], acc[x][y]);
      }
    }
    // the other buffer was last read before the previous barrier
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (KS > 1) {
    // partial tiles of groups 1.. through LDS (operand buffers are free now)
    auto ridx = [&](int x, int y, int j) { return (((wave * MT + x) * NT + y) * 4 + j) * 64 + lane; };
    if (g > 0) {
#pragma unroll
      for (int x = 0; x < MT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y)
#pragma unroll
          for (int j = 0; j < 4; ++j) smem[(g - 1) * PART + ridx(x, y, j)] = acc[x][y][j];
    }
    __syncthreads();
    if (g > 0) return;
    for (int q = 0; q < KS - 1; ++q)
#pragma unroll
      for (int x = 0; x < MT; ++x)
#pragma unroll
        for (int y = 0; y < NT; ++y)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[x][y][j] += smem[q * PART + ridx(x, y, j)];
  }
  if (KS == 1) {
    // each wave stages one 16-column strip of its quadrant at a time in LDS
    // (its own slot; the operand buffers are free after the last barrier)
    // and writes C a column at a time: lanes on consecutive rows, so every
    // access covers whole cache lines of the column-major C (the MFMA layout
    // spreads a register over 16 columns)
    constexpr int SR = 16 * MT + 1;  // strip rows + pad
    T *stg = smem + wave * SR * 16;
    const int r0 = m0 + wr * 16 * MT;
#pragma unroll
    for (int y = 0; y < NT; ++y) {
      const int c0 = n0 + wc * 16 * NT + 16 * y;
      // the strip's C values are all requested before the accumulators are
      // staged, so their latencies overlap each other and the staging instead
      // of one load-then-store round trip per element
      T cv[MT * 4];
#pragma unroll
      for (int it = 0; it < MT * 4; ++it) {
        const int i = lane + 64 * it, r = i % (16 * MT), c = i / (16 * MT);
        const int row = r0 + r, col = c0 + c;
        cv[it] = (beta != T(0) && row < M && col < N)
                     ? gld<COH>(&C[(rmap ? rmap[row] : row) + (int64_t)(cmap ? cmap[col] : col) * ldc])
                     : T(0);
      }
#pragma unroll
      for (int x = 0; x < MT; ++x)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          stg[16 * x + Mfma<T>::row(lane, j) + (lane & 15) * SR] = alpha * acc[x][y][j];
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
#pragma unroll
      for (int it = 0; it < MT * 4; ++it) {
        const int i = lane + 64 * it, r = i % (16 * MT), c = i / (16 * MT);
        const int row = r0 + r, col = c0 + c;
        if (row < M && col < N && (!LW || row >= col)) {
          T *cp = &C[(rmap ? rmap[row] : row) + (int64_t)(cmap ? cmap[col] : col) * ldc];
          const T v = stg[r + c * SR];
          gst<COH>(cp, (beta == T(0)) ? v : v + beta * cv[it]);
        }
      }
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
    }
  } else {
#pragma unroll
    for (int x = 0; x < MT; ++x)
#pragma unroll
      for (int y = 0; y < NT; ++y)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = m0 + wr * 16 * MT + 16 * x + Mfma<T>::row(lane, j);
          const int col = n0 + wc * 16 * NT + 16 * y + (lane & 15);
          if (row < M && col < N && (!LW || row >= col)) {
            T *c = &C[(rmap ? rmap[row] : row) + (int64_t)(cmap ? cmap[col] : col) * ldc];
            const T v = alpha * acc[x][y][j];
            gst<COH>(c, (beta == T(0)) ? v : v + beta * gld<COH>(c));
          }
        }
  }
}

// gemm_tile_s with an LDS array of its own per instantiation (TAG tells the
// kernels apart, see above)
template <class T, bool TA, bool TB, int MT, int NT, int KS = 1, int TAG = 0, bool LW = false>
__device__ __forceinline__ void gemm_tile(const T *A, const T *B, T *C, int M, int N, int K, int lda,
                                          int ldb, int ldc, T alpha, T beta, int m0, int n0,
                                          const int *rmap = nullptr, const int *cmap = nullptr) {
  __shared__ T smem[gemm_tile_lds<T, MT, NT, KS>()];
  gemm_tile_s<T, TA, TB, MT, NT, KS, LW, false>(smem, A, B, C, M, N, K, lda, ldb, ldc, alpha, beta,
                                                m0, n0, rmap, cmap);
}

// map.n > 0: the entry's own tiles only (lower: its lower-triangle tiles,
// TM = TN and M = N for every entry)
template <class T, bool TA, bool TB, int MT, int NT>
__global__ __launch_bounds__(256) void gemm_kernel(const T *A, const T *B, T *C,
                                                   const GemmDesc *desc, int tm, int tn, T alpha,
                                                   T beta, int lower, int batch, const TileMap map) {
  constexpr int TM = 32 * MT, TN = 32 * NT;
  int e, t, ti, tj;
  if (map.n > 0) {
    if (!map_tile(map, gridDim.x, e, t)) return;
    if (lower) {
      lower_tile(t, ti, tj);
    } else {
      const int tme = (desc[e].M + TM - 1) / TM;
      ti = t % tme;
      tj = t / tme;
    }
  } else {
    if (!xcd_remap(gridDim.x, tm * tn, batch, e, t)) return;
    ti = t % tm;
    tj = t / tm;
  }
  const GemmDesc d = desc[e];
  const int m0 = ti * TM, n0 = tj * TN;
  if (m0 >= d.M || n0 >= d.N) return;
  if (lower && m0 + TM - 1 < n0) return;
  gemm_tile<T, TA, TB, MT, NT, 1, 0>(A + d.a_off, B + d.b_off, C + d.c_off, d.M, d.N, d.K, d.lda,
                                     d.ldb, d.ldc, alpha, beta, m0, n0);
}

// C[map rows or columns] += A B^T per entry (TAG 5: instantiations of its own)
template <class T, int MT, int NT>
__global__ __launch_bounds__(256) void gemm_scatter_kernel(const T *A, const T *B, T *C,
                                                           const GemmDesc *desc, const int *map,
                                                           const int64_t *map_off, int map_rows,
                                                           int tm, int tn, int batch,
                                                           const TileMap tmap) {
  constexpr int TM = 32 * MT, TN = 32 * NT;
  int e, t, ti, tj;
  if (tmap.n > 0) {
    if (!map_tile(tmap, gridDim.x, e, t)) return;
    const int tme = (desc[e].M + TM - 1) / TM;
    ti = t % tme;
    tj = t / tme;
  } else {
    if (!xcd_remap(gridDim.x, tm * tn, batch, e, t)) return;
    ti = t % tm;
    tj = t / tm;
  }
  const GemmDesc d = desc[e];
  const int m0 = ti * TM, n0 = tj * TN;
  if (m0 >= d.M || n0 >= d.N) return;
  const int *mp = map + map_off[e];
  gemm_tile<T, false, true, MT, NT, 1, 5>(A + d.a_off, B + d.b_off, C + d.c_off, d.M, d.N, d.K, d.lda,
                                          d.ldb, d.ldc, T(1), T(1), m0, n0, map_rows ? mp : nullptr,
                                          map_rows ? nullptr : mp);
}

// --- Cholesky -------------------------------------------------------------

// The steps of the blocked Cholesky, one tile each, shared by the launch per
// step (chol_*_kernel) and the fused launch (potrf_fused_kernel).  COH: the
// matrix, the inverse blocks and the factor are accessed device-coherently
// (the fused launch, where other work-groups of the same launch wrote them).

// A[kb:, kb:kb+w] -= A[kb:, c0:kb] A[kb:kb+w, c0:kb]^T with c0 = k0 NB (the
// panel's first column; the columns before it were applied by the panel
// updates, chol_syrk_tile), row tile t of 32 MT rows.
template <class T, int MT, bool COH>
__device__ __forceinline__ void chol_update_tile(T *smem, T *pool, const MatDesc &d, int k, int k0,
                                                 int t) {
  constexpr int TM = 32 * MT;
  const int kb = k * NB, c0 = k0 * NB;
  if (kb >= d.n || k <= k0) return;
  const int M = d.n - kb, N = min(NB, d.n - kb), K = kb - c0;
  if (t * TM >= M) return;
  T *A = pool + d.a_off;
  const T *P = A + kb + (int64_t)c0 * d.lda;
  gemm_tile_s<T, false, true, MT, 2, 1, false, COH>(smem, P, P, A + kb + (int64_t)kb * d.lda, M, N,
                                                    K, d.lda, d.lda, d.lda, T(-1), T(1), t * TM, 0);
}

// Trailing update after a factored panel of columns [p0, p1):
// A[p1:, p1:] -= L[p1:, p0:p1] L[p1:, p0:p1]^T, lower triangle only, 128 x 128
// tiles (tile t = the pair tj <= ti of lower_tile); the diagonal tiles write
// only their lower part.
template <class T, bool COH>
__device__ __forceinline__ void chol_syrk_tile(T *smem, T *pool, const MatDesc &d, int p0, int p1,
                                               int t) {
  if (p1 >= d.n) return;
  int ti, tj;
  lower_tile(t, ti, tj);
  const int M = d.n - p1;
  if (ti * 128 >= M) return;
  T *A = pool + d.a_off;
  const T *P = A + p1 + (int64_t)p0 * d.lda;
  gemm_tile_s<T, false, true, 4, 4, 1, true, COH>(smem, P, P, A + p1 + (int64_t)p1 * d.lda, M, M,
                                                  p1 - p0, d.lda, d.lda, d.lda, T(-1), T(1),
                                                  ti * 128, tj * 128);
}

// Row tiles below the diagonal of block column k (tile t: rows
// kb + (t + 1) NB ..): X <- X L_kk^{-T} = X (L_kk^{-1})^T, an MFMA tile product
// with the inverse written by chol_diag_block (in place: the tile is read
// whole before it is written).
template <class T, bool COH>
__device__ __forceinline__ void chol_panel_tile(T *smem, T *pool, const MatDesc &d, int k, int t,
                                                const T *Di) {
  const int kb = k * NB;
  if (kb >= d.n) return;
  const int w = min(NB, d.n - kb);
  const int r0 = kb + (t + 1) * NB;
  if (r0 >= d.n) return;
  const int nr = min(NB, d.n - r0);
  T *X = pool + d.a_off + r0 + (int64_t)kb * d.lda;
  gemm_tile_s<T, false, true, 2, 2, 1, false, COH>(smem, X, Di, X, nr, w, w, d.lda, NB, d.lda, T(1),
                                                   T(0), 0, 0);
}

// value of v in lane l (l uniform over the wave)
__device__ __forceinline__ double readlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Factor the diagonal block of block column k in place and write the inverse
// of the factored block to out (NB x NB, ld NB, zero outside the w x w
// block).  Wave 0 computes; every thread of the work-group must call (the
// barriers), and all of them copy the inverse out.  Lane r holds row r of the
// block in registers.  The columns are taken in sub-blocks of DSB: within a
// sub-block, column c is eliminated right-looking (l_rc = a_rc / sqrt(a_cc),
// a_rs -= l_rc l_sc for the sub-block's later columns s, the l_sc broadcast
// from their lanes by readlane: no barrier, no LDS traffic); the columns after
// the sub-block then take the rank-DSB update A22 -= L21 L21^T of their lower
// 16 x 16 tiles as matrix-core products, the panel staged in Y and the
// products in D (one wave: its LDS accesses complete in order).  The inverse
// is formed by lane j taking column j by forward substitution against the
// rows of L broadcast from LDS (D).  *status receives (column+1) of the first
// non-positive pivot.
constexpr int DSB = 16;
static_assert(DSB == 16 && NB % DSB == 0, "the trailing update works on 16 x 16 tiles");
// orders one wave's LDS accesses across lanes: the hardware completes a wave's
// LDS operations in issue order, so only the compiler must not move them
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }
template <class T, bool COH>
__device__ void chol_diag_block(T *pool, const MatDesc &d, int k, int *status, T *out,
                                T (*D)[NB + 1], T (*Y)[NB + 1]) {
  const int kb = k * NB;
  if (kb >= d.n) return;  // uniform
  const int w = min(NB, d.n - kb);
  T *A = pool + d.a_off;
  const int64_t lda = d.lda;
  const int r = threadIdx.x;
  if (r < 64) {
    T row[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      row[c] = (r < w && c < w && r >= c) ? gld<COH>(&A[(kb + r) + (int64_t)(kb + c) * lda]) : T(0);
    int fail = 0;
#pragma unroll
    for (int c0 = 0; c0 < NB; c0 += DSB) {
      if (c0 < w) {  // uniform
#pragma unroll
        for (int c = c0; c < c0 + DSB; ++c) {
          if (c < w) {  // uniform
            T piv = readlane(row[c], c);
            if (!(piv > T(0))) {
              if (fail == 0) fail = kb + c + 1;
              piv = T(1);
            }
            const T lcc = sqrt(piv);
            const T l = r == c ? lcc : row[c] / lcc;
            row[c] = l;
            // rows r > c: a_rs -= l_rc l_sc for the sub-block's columns
            // c < s <= r (entries above the diagonal, s > r, are updated too
            // and never read)
#pragma unroll
            for (int sc = c + 1; sc < c0 + DSB; ++sc) row[sc] -= l * readlane(l, sc);
          }
        }
        if (c0 + DSB < w) {  // uniform: the trailing columns' lower tiles
          const int l16 = r & 15, kq = r >> 4;
          wave_lds_order();
#pragma unroll
          for (int q = 0; q < DSB; ++q) Y[r][q] = row[c0 + q];
          wave_lds_order();
#pragma unroll
          for (int tj = c0 / 16 + 1; tj < NB / 16; ++tj) {
#pragma unroll
            for (int ti = tj; ti < NB / 16; ++ti) {
              typename Mfma<T>::v4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
              for (int q = 0; q < DSB; q += 4)
                acc = Mfma<T>::op(Y[16 * ti + l16][q + kq], Y[16 * tj + l16][q + kq], acc);
#pragma unroll
              for (int t = 0; t < 4; ++t) D[16 * ti + Mfma<T>::row(r, t)][16 * tj + l16] = acc[t];
            }
          }
          wave_lds_order();
          // lane r: a_rs -= (L21 L21^T)_rs for the tiles at or below the
          // diagonal (s / 16 <= r / 16); D is stale elsewhere and not read
#pragma unroll
          for (int sc = c0 + DSB; sc < NB; ++sc) {
            const T u = D[r][sc];
            row[sc] -= (sc >> 4) <= (r >> 4) ? u : T(0);
          }
          wave_lds_order();
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (r < w && c < w && r >= c) gst<COH>(&A[(kb + r) + (int64_t)(kb + c) * lda], row[c]);
      // the factor, and the identity outside the w x w block, for the inverse
      D[r][c] = (r < w && c < w) ? (r >= c ? row[c] : T(0)) : (r == c ? T(1) : T(0));
    }
    if (r == 0 && fail && status) atomicCAS(status, 0, fail);
  }
  __syncthreads();
  if (r < 64) {
    const int j = r;
    T y[NB];
#pragma unroll
    for (int rr = 0; rr < NB; ++rr) {
      T s0 = rr == j ? T(1) : T(0), s1 = T(0);
#pragma unroll
      for (int m = 0; m + 1 < rr; m += 2) {
        s0 -= D[rr][m] * y[m];
        s1 -= D[rr][m + 1] * y[m + 1];
      }
      if (rr & 1) s0 -= D[rr][rr - 1] * y[rr - 1];
      y[rr] = (s0 + s1) / D[rr][rr];
    }
#pragma unroll
    for (int rr = 0; rr < NB; ++rr) Y[rr][j] = (rr < w && j < w) ? y[rr] : T(0);
  }
  __syncthreads();
  for (int i = r; i < NB * NB; i += blockDim.x) gst<COH>(&out[i], Y[i % NB][i / NB]);
}

// One launch per step of the blocked Cholesky (DenseOps::potrf without the
// fused launch): every entry's tiles of the step.
// MT = 4: 128-row tiles; MT = 2: 64-row tiles (launches with few tiles); the
// sums are the same for both.
template <class T, int MT>
__global__ __launch_bounds__(256) void chol_update_kernel(T *pool, const MatDesc *desc, int k, int k0,
                                                          int tm, int batch, const TileMap map) {
  __shared__ T smem[gemm_tile_lds<T, MT, 2, 1>()];
  int e, t;
  if (map.n > 0 ? !map_tile(map, gridDim.x, e, t) : !xcd_remap(gridDim.x, tm, batch, e, t)) return;
  chol_update_tile<T, MT, false>(smem, pool, desc[e], k, k0, t);
}

template <class T>
__global__ __launch_bounds__(256) void chol_syrk_kernel(T *pool, const MatDesc *desc, int p0, int p1,
                                                        int tm, int batch, const TileMap map) {
  __shared__ T smem[gemm_tile_lds<T, 4, 4, 1>()];
  int e, t;
  if (map.n > 0 ? !map_tile(map, gridDim.x, e, t) : !xcd_remap(gridDim.x, tm * (tm + 1) / 2, batch, e, t))
    return;
  chol_syrk_tile<T, false>(smem, pool, desc[e], p0, p1, t);
}

// one wave per entry
template <class T>
__global__ __launch_bounds__(64) void chol_diag_kernel(T *pool, const MatDesc *desc, int k,
                                                       int *status, int batch, T *dinv,
                                                       const int64_t *dinv_off) {
  __shared__ T D[NB][NB + 1];
  __shared__ T Y[NB][NB + 1];
  const int e = blockIdx.x;
  if (e >= batch) return;
  chol_diag_block<T, false>(pool, desc[e], k, status ? status + e : nullptr,
                            dinv + dinv_off[e] + (int64_t)k * NB * NB, D, Y);
}

template <class T>
__global__ __launch_bounds__(256) void chol_panel_kernel(T *pool, const MatDesc *desc, int k,
                                                         int tm, int batch, const T *dinv,
                                                         const int64_t *dinv_off, const TileMap map) {
  __shared__ T smem[gemm_tile_lds<T, 2, 2, 1>()];
  int e, t;
  if (map.n > 0 ? !map_tile(map, gridDim.x, e, t) : !xcd_remap(gridDim.x, tm, batch, e, t)) return;
  chol_panel_tile<T, false>(smem, pool, desc[e], k, t, dinv + dinv_off[e] + (int64_t)k * NB * NB);
}

// --- multi-RHS triangular solves -------------------------------------------

// Within a panel of block rows [p0, p1) (columns of L):
// forward: B[kb:kb+w, :] -= L[kb:kb+w, p0:kb] B[p0:kb, :]
// backward: B[kb:kb+w, :] -= L[kb+w:q1, kb:kb+w]^T B[kb+w:q1, :], q1 = min(p1, n)
// (the rows outside the panel were applied by trsm_gemm_kernel).
// NT = 4, KS = 1: 128-column tiles; NT = 1, KS = 2: 32-column tiles with two
// groups of waves splitting K (few right-hand sides)
template <class T, bool BWD, int NT, int KS>
__global__ __launch_bounds__(256 * KS) void trsm_update_kernel(const T *apool, T *bpool,
                                                               const MatDesc *desc, int k, int p0,
                                                               int p1, int tn, int batch,
                                                               const TileMap map) {
  constexpr int TN = 32 * NT;
  int e, t;
  if (map.n > 0 ? !map_tile(map, gridDim.x, e, t) : !xcd_remap(gridDim.x, tn, batch, e, t)) return;
  const MatDesc d = desc[e];
  const int kb = k * NB;
  if (kb >= d.n) return;
  const int w = min(NB, d.n - kb);
  if (t * TN >= d.nrhs) return;
  const T *L = apool + d.a_off;
  T *B = bpool + d.b_off;
  if (!BWD) {
    if (kb <= p0) return;
    gemm_tile<T, false, false, 2, NT, KS, 3>(L + kb + (int64_t)p0 * d.lda, B + p0, B + kb, w, d.nrhs,
                                             kb - p0, d.lda, d.ldb, d.ldb, T(-1), T(1), 0, t * TN);
  } else {
    const int K = min(p1, d.n) - kb - w;
    if (K <= 0) return;
    gemm_tile<T, true, false, 2, NT, KS, 3>(L + (kb + w) + (int64_t)kb * d.lda, B + kb + w, B + kb,
                                            w, d.nrhs, K, d.lda, d.ldb, d.ldb, T(-1), T(1), 0,
                                            t * TN);
  }
}

// B[kb:kb+w, tile t] <- L_kk^{-1} B (forward) or L_kk^{-T} B (backward): an MFMA
// tile product with the inverse of the diagonal block (in place: each
// work-group reads its column tile whole before writing it).
template <class T, bool BWD>
__global__ __launch_bounds__(256) void trsm_diag_kernel(const T *apool, T *bpool,
                                                        const MatDesc *desc, int k, int tn,
                                                        int batch, const T *dinv,
                                                        const int64_t *dinv_off, const TileMap map) {
  int e, t;
  if (map.n > 0 ? !map_tile(map, gridDim.x, e, t) : !xcd_remap(gridDim.x, tn, batch, e, t)) return;
  const MatDesc d = desc[e];
  const int kb = k * NB;
  if (kb >= d.n) return;
  const int w = min(NB, d.n - kb);
  const int c0 = t * NB;
  if (c0 >= d.nrhs) return;
  T *B = bpool + d.b_off + kb;
  const T *Di = dinv + dinv_off[e] + (int64_t)k * NB * NB;
  gemm_tile<T, BWD, false, 2, 2, 1, 4>(Di, B, B, w, d.nrhs, w, NB, d.ldb, d.ldb, T(1), T(0), 0, c0);
}

// Block row k in one launch (128-column tiles): the update by the panel's
// solved rows as in trsm_update_kernel<NT = 4>, then, after a barrier, the
// product with the inverse diagonal block as in trsm_diag_kernel, on the
// same columns; the same sums in the same order as the two launches.
template <class T, bool BWD>
__global__ __launch_bounds__(256) void trsm_step_kernel(const T *apool, T *bpool, const MatDesc *desc,
                                                        int k, int p0, int p1, int tu, int batch,
                                                        const T *dinv, const int64_t *dinv_off,
                                                        const TileMap map) {
  __shared__ T smem[gemm_tile_lds<T, 2, 4, 1>()];
  int e, t;
  if (map.n > 0 ? !map_tile(map, gridDim.x, e, t) : !xcd_remap(gridDim.x, tu, batch, e, t)) return;
  const MatDesc d = desc[e];
  const int kb = k * NB;
  if (kb >= d.n) return;
  const int w = min(NB, d.n - kb);
  const int c0 = t * 128;
  if (c0 >= d.nrhs) return;
  const T *L = apool + d.a_off;
  T *B = bpool + d.b_off;
  if (!BWD) {
    if (kb > p0) {
      gemm_tile_s<T, false, false, 2, 4>(smem, L + kb + (int64_t)p0 * d.lda, B + p0, B + kb, w, d.nrhs,
                                         kb - p0, d.lda, d.ldb, d.ldb, T(-1), T(1), 0, c0);
      __syncthreads();
    }
  } else {
    const int K = min(p1, d.n) - kb - w;
    if (K > 0) {
      gemm_tile_s<T, true, false, 2, 4>(smem, L + (kb + w) + (int64_t)kb * d.lda, B + kb + w, B + kb,
                                        w, d.nrhs, K, d.lda, d.ldb, d.ldb, T(-1), T(1), 0, c0);
      __syncthreads();
    }
  }
  const T *Di = dinv + dinv_off[e] + (int64_t)k * NB * NB;
  gemm_tile_s<T, BWD, false, 2, 4>(smem, Di, B + kb, B + kb, w, d.nrhs, w, NB, d.ldb, d.ldb, T(1), T(0),
                                   0, c0);
}

// Update of the rows outside a solved panel of block rows [p0, p1):
// forward: B[p1:n, :] -= L[p1:n, p0:p1] B[p0:p1, :]
// backward: B[0:p0, :] -= L[p0:q1, 0:p0]^T B[p0:q1, :], q1 = min(p1, n)
// 128-row tiles (tm for the largest entry) by 32 NT-column tiles (tn).
template <class T, bool BWD, int NT>
__global__ __launch_bounds__(256) void trsm_gemm_kernel(const T *apool, T *bpool, const MatDesc *desc,
                                                        int p0, int p1, int tm, int tn, int batch,
                                                        const TileMap map) {
  constexpr int TN = 32 * NT;
  int e, t, ti, tj;
  if (map.n > 0) {
    if (!map_tile(map, gridDim.x, e, t)) return;
    // the entry's own row tiles: below the panel (forward) or above it
    const MatDesc q = desc[e];
    const int rows = BWD ? (p0 < min(p1, q.n) ? p0 : 0) : max(0, q.n - p1);
    const int tme = max(1, (rows + 127) / 128);
    ti = t % tme;
    tj = t / tme;
  } else {
    if (!xcd_remap(gridDim.x, tm * tn, batch, e, t)) return;
    ti = t % tm;
    tj = t / tm;
  }
  const MatDesc d = desc[e];
  if (tj * TN >= d.nrhs) return;
  const T *L = apool + d.a_off;
  T *B = bpool + d.b_off;
  if (!BWD) {
    if (p1 >= d.n) return;
    const int M = d.n - p1;
    if (ti * 128 >= M) return;
    gemm_tile<T, false, false, 4, NT, 1, 7>(L + p1 + (int64_t)p0 * d.lda, B + p0, B + p1, M, d.nrhs,
                                            p1 - p0, d.lda, d.ldb, d.ldb, T(-1), T(1), ti * 128,
                                            tj * TN);
  } else {
    const int q1 = min(p1, d.n);
    if (p0 >= q1 || ti * 128 >= p0) return;
    gemm_tile<T, true, false, 4, NT, 1, 7>(L + p0, B + p0, B, p0, d.nrhs, q1 - p0, d.lda, d.ldb,
                                           d.ldb, T(-1), T(1), ti * 128, tj * TN);
  }
}

// Upper triangle <- lower triangle, by 32 x 32 tiles through LDS so that
// both the reads and the writes run down columns: work-group (bi, bj), bi <=
// bj, writes tile (bi, bj) from the transpose of tile (bj, bi) (on the
// diagonal only the entries above it).
// With a tile map (map.n > 0) only each entry's own tile pairs are launched:
// tile t of entry e is the pair (bi, bj) = (tj, ti) of lower_tile(t).
template <class T>
__global__ __launch_bounds__(256) void symmetrize_kernel(T *pool, const MatDesc *desc, int nt,
                                                         const TileMap map) {
  __shared__ T tl[32][33];
  int e, bi, bj;
  if (map.n > 0) {
    int t;
    if (!map_tile(map, gridDim.x, e, t)) return;
    lower_tile(t, bj, bi);
  } else {
    bi = blockIdx.x % nt;
    bj = blockIdx.x / nt;
    e = blockIdx.y;
    if (bi > bj) return;
  }
  const MatDesc d = desc[e];
  const int n = d.n;
  if (32 * bj >= n) return;
  T *A = pool + d.a_off;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 32 * bj + tx, c = 32 * bi + ty + 8 * q;  // lower tile (bj, bi)
    if (r < n && c < n) tl[ty + 8 * q][tx] = A[r + (int64_t)c * d.lda];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = 32 * bi + tx, c = 32 * bj + ty + 8 * q;  // upper tile (bi, bj)
    if (r < n && c < n && r < c) A[r + (int64_t)c * d.lda] = tl[tx][ty + 8 * q];
  }
}

// --- one-RHS blocked triangular solve with completion flags -----------------

template <class T>
__device__ __forceinline__ T ld_coherent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_coherent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Completion flags of the one-right-hand-side solves.  Everything that
// crosses work-groups in those kernels (the flags and the solved entries of x)
// is read and written with device-coherent atomic accesses, so a flag needs
// only ordering, not cache maintenance: the producer waits for its x stores
// to complete before the flag store (workgroup-scope release: a store-counter
// wait), and the consumer's x loads are issued after the flag load returned
// (workgroup-scope acquire).  Agent-scope fences would write back and
// invalidate the whole L2 of the XCD at every block, evicting the cached
// factor tiles of every other work-group.
// (called by a lane of the wave that stored the entries: s_waitcnt vmcnt(0),
// encoded for gfx9 with expcnt and lgkmcnt left at their maxima, waits until
// those device-coherent stores are acknowledged)
__device__ __forceinline__ void flag_publish(int *flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded spin on a completion flag: the block waited on holds a smaller
// ticket, so it is resident or done; the bound only guards against an earlier
// fault.
__device__ bool wait_flag(int *flag, int *err) {
  for (long it = 0; it < (1L << 26); ++it) {
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  atomicExch(err, 1);
  return false;
}

__device__ __forceinline__ bool flag_set(int *flag) {
  if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return true;
}


// One work-group per 64-row block k of one entry, taken in ticket order
// (lower: blocks upwards, upper: downwards), so every block waited on holds a
// smaller ticket.  The work-group accumulates the products of its block row
// with the solution blocks as they complete: each round takes every block
// already solved (up to 32); block j always goes to wave j mod 4 and every
// wave adds its blocks in order, so the sums do not depend on timing.  A lane
// owns one row and reads its row of each 64 x 64 tile with coalesced loads.
// The tile of the block solved last (on the critical path) is loaded into
// registers, a quarter per wave, before waiting.  The diagonal block is
// applied through its precomputed inverse (staged in LDS before waiting).
// The upper variant solves U x = b for an upper triangular U stored
// column-major, so that L^T x = b runs on an explicit transpose of L with the
// same coalesced access.
// Several right-hand sides (m <= M columns of x, column stride ldx) share
// every load of the factor: each tile element is multiplied into all columns
// while in registers.  The operations on one column, and their order, are
// the same for every M, so a column solved in a block has the bits it has
// when solved alone.
template <class T, bool UPPER, int M>
__global__ __launch_bounds__(256) void trsv_kernel(const T *apool, T *xpool, const MatDesc *desc,
                                                   const T *dinv, const int64_t *dinv_off,
                                                   const int *order, const int *flag_off,
                                                   int total, int *work, int *err, int m,
                                                   int64_t ldx) {
  __shared__ int s_ticket, s_ok, s_end;
  __shared__ T D[NB][NB + 1];
  __shared__ T part[4][M][NB];
  __shared__ T vs[M][NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    s_ticket = atomicAdd(&work[0], 1);
    s_ok = 1;
  }
  __syncthreads();
  const int tk = s_ticket;
  if (tk >= total) return;
  const int e = order[2 * tk], k = order[2 * tk + 1];
  const MatDesc d = desc[e];
  const T *L = apool + d.a_off;
  T *x = xpool + d.b_off;
  const int64_t lda = d.lda;
  const int nblk = (d.n + NB - 1) / NB;
  const int r0 = k * NB, w = min(NB, d.n - r0);
  const int rl = r0 + min(lane, w - 1);  // row read by this lane (clamped)
  int *flags = work + 1 + flag_off[e];
  const int step = UPPER ? -1 : 1;
  const int last = k - step;                        // block solved just before this one
  const bool has_last = UPPER ? last < nblk : last >= 0;
  // critical-path tile: columns 16 wave .. 16 wave + 15 of block `last`
  T pf[16];
  int wl = 0;
  if (has_last) {
    const int c0 = last * NB;
    wl = min(NB, d.n - c0);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int c = wave * 16 + i;
      pf[i] = c < wl ? L[rl + (int64_t)(c0 + c) * lda] : T(0);
    }
  }
  // inverse of the diagonal block of L (of L^T's transpose for the upper
  // variant)
  const T *Di = dinv + dinv_off[e] + (int64_t)k * NB * NB;
  for (int i = tid; i < NB * NB; i += 256) {
    const int r = i % NB, c = i / NB;
    D[r][c] = (r < w && c < w && r >= c) ? Di[r + c * NB] : T(0);
  }
  // right-hand sides of this block (only this work-group overwrites them)
  for (int i = tid; i < M * NB; i += 256) {
    const int q = i / NB, l = i % NB;
    vs[q][l] = (q < m && l < w) ? x[r0 + l + q * ldx] : T(0);
  }
  T acc[M];
#pragma unroll
  for (int q = 0; q < M; ++q) acc[q] = T(0);
  // blocks before `last`, in rounds
  int next = UPPER ? nblk - 1 : 0;
  while (UPPER ? next > last : next < last) {
    if (tid == 0) {
      if (!wait_flag(&flags[next], err)) s_ok = 0;
      int end = next + step;
      for (int c = 1; c < 32 && (UPPER ? end > last : end < last) && flag_set(&flags[end]); ++c)
        end += step;
      s_end = end;
    }
    __syncthreads();
    const int end = s_end;
    for (int jb = next; jb != end; jb += step) {
      const int owner = UPPER ? (nblk - 1 - jb) & 3 : jb & 3;
      if (owner != wave) continue;
      const int c0 = jb * NB, wc = min(NB, d.n - c0);
      T xv[M];
#pragma unroll
      for (int q = 0; q < M; ++q) xv[q] = (q < m && lane < wc) ? ld_coherent(&x[c0 + lane + q * ldx]) : T(0);
      const T *row = L + rl + (int64_t)c0 * lda;
      if (wc == NB) {
        // four independent partial sums per column, added in a fixed order
        T a0[M], a1[M], a2[M], a3[M];
#pragma unroll
        for (int q = 0; q < M; ++q) a0[q] = a1[q] = a2[q] = a3[q] = T(0);
#pragma unroll
        for (int c = 0; c < NB; c += 4) {
          const T l0 = row[(int64_t)c * lda], l1 = row[(int64_t)(c + 1) * lda];
          const T l2 = row[(int64_t)(c + 2) * lda], l3 = row[(int64_t)(c + 3) * lda];
#pragma unroll
          for (int q = 0; q < M; ++q) {
            a0[q] += l0 * readlane(xv[q], c);
            a1[q] += l1 * readlane(xv[q], c + 1);
            a2[q] += l2 * readlane(xv[q], c + 2);
            a3[q] += l3 * readlane(xv[q], c + 3);
          }
        }
#pragma unroll
        for (int q = 0; q < M; ++q) acc[q] += (a0[q] + a1[q]) + (a2[q] + a3[q]);
      } else {
#pragma unroll
        for (int q = 0; q < M; ++q) {
          T a = T(0);
          for (int c = 0; c < wc; ++c) a += row[(int64_t)c * lda] * readlane(xv[q], c);
          acc[q] += a;
        }
      }
    }
    next = end;
    __syncthreads();
  }
  if (has_last) {
    if (tid == 0 && !wait_flag(&flags[last], err)) s_ok = 0;
    __syncthreads();
    const int c0 = last * NB;
#pragma unroll
    for (int q = 0; q < M; ++q) {
      const T xv = (q < m && lane < wl) ? ld_coherent(&x[c0 + lane + q * ldx]) : T(0);
      T a0 = T(0), a1 = T(0);
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        a0 += pf[i] * readlane(xv, wave * 16 + i);
        a1 += pf[i + 1] * readlane(xv, wave * 16 + i + 1);
      }
      acc[q] += a0 + a1;
    }
  }
#pragma unroll
  for (int q = 0; q < M; ++q) part[wave][q][lane] = acc[q];
  __syncthreads();
  for (int i = tid; i < M * NB; i += 256) {
    const int q = i / NB, l = i % NB;
    vs[q][l] = l < w ? vs[q][l] - (part[0][q][l] + part[1][q][l] + part[2][q][l] + part[3][q][l])
                     : T(0);
  }
  __syncthreads();
  // x_k = D^-1 v (lower) or D^-T v (upper), D^-1 lower triangular (D is zero
  // outside its lower triangle and v beyond w: full-length sums with four
  // partial sums); column q on wave q mod 4
  for (int q = wave; q < M; q += 4) {
    T y0 = T(0), y1 = T(0), y2 = T(0), y3 = T(0);
#pragma unroll 4
    for (int c = 0; c < NB; c += 4) {
      if (!UPPER) {
        y0 += D[lane][c] * vs[q][c];
        y1 += D[lane][c + 1] * vs[q][c + 1];
        y2 += D[lane][c + 2] * vs[q][c + 2];
        y3 += D[lane][c + 3] * vs[q][c + 3];
      } else {
        y0 += D[c][lane] * vs[q][c];
        y1 += D[c + 1][lane] * vs[q][c + 1];
        y2 += D[c + 2][lane] * vs[q][c + 2];
        y3 += D[c + 3][lane] * vs[q][c + 3];
      }
    }
    const T y = (y0 + y1) + (y2 + y3);
    if (q < m && lane < w) st_coherent(&x[r0 + lane + q * ldx], y);
  }
  // every wave that stored waits for its stores before the barrier, so the
  // flag below is published after all of them
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (tid == 0) {
    flag_publish(&flags[k]);
    if (!s_ok) atomicExch(err, 1);
  }
}

// Inverse of every NB x NB diagonal block of the lower triangular L of each
// entry: block kb of entry e goes to inv + inv_off[e] + kb NB^2 (column-major,
// ld NB, upper part zero).  One work-group per block; thread j solves for
// column j of the inverse.
template <class T>
__global__ __launch_bounds__(64) void diag_inv_kernel(const T *pool, const MatDesc *desc, T *inv,
                                                      const int64_t *inv_off) {
  __shared__ T D[NB][NB + 1];
  __shared__ T Y[NB][NB + 1];  // Y[i][j]: row i of column j of the inverse
  const MatDesc d = desc[blockIdx.y];
  const int kb = blockIdx.x, r0 = kb * NB;
  if (r0 >= d.n) return;
  const int w = min(NB, d.n - r0), j = threadIdx.x;
  const T *A = pool + d.a_off;
  for (int c = 0; c < w; ++c)
    if (j < w) D[j][c] = (j >= c) ? A[(r0 + j) + (int64_t)(r0 + c) * d.lda] : T(0);
  for (int i = 0; i < NB; ++i) Y[i][j] = T(0);
  __syncthreads();
  if (j < w) {
    for (int i = j; i < w; ++i) {
      T sacc = (i == j) ? T(1) : T(0);
      for (int m = j; m < i; ++m) sacc -= D[i][m] * Y[m][j];
      Y[i][j] = sacc / D[i][i];
    }
  }
  __syncthreads();
  T *out = inv + inv_off[blockIdx.y] + (int64_t)kb * NB * NB;
  for (int c = 0; c < NB; ++c) out[j + (int64_t)c * NB] = Y[j][c];
}

// B <- A^T for every entry (n x n, lda / ldb); used to keep L^T beside L
// With a tile map (map.n > 0) only each entry's own nt x nt tiles are
// launched (tile t: column tile t % nt, row tile t / nt, nt = ceil(n / 32)).
template <class T>
__global__ void transpose_kernel(const T *apool, T *bpool, const MatDesc *desc, const TileMap map) {
  int e, c0, r0;
  if (map.n > 0) {
    int t;
    if (!map_tile(map, gridDim.x, e, t)) return;
    const int nt = (desc[e].n + 31) / 32;
    c0 = (t % nt) * 32;
    r0 = (t / nt) * 32;
  } else {
    e = blockIdx.z;
    c0 = blockIdx.x * 32;
    r0 = blockIdx.y * 32;
  }
  const MatDesc d = desc[e];
  if (c0 >= d.n || r0 >= d.n) return;
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + tx, c = c0 + j;
    tile[j][tx] = (r < d.n && c < d.n) ? apool[d.a_off + r + (int64_t)c * d.lda] : T(0);
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = c0 + tx, c = r0 + j;
    if (r < d.n && c < d.n) bpool[d.b_off + r + (int64_t)c * d.ldb] = tile[tx][j];
  }
}

// --- fused Cholesky: one launch for every step of every entry -------------
//
// The tasks are the tiles of the steps above, grouped in levels: per panel of
// PB block columns, for each column k of the panel the update (except the
// panel's first column), the diagonal factor and the panel solve, then the
// trailing update.  An entry's tasks of one level need all of its tasks of the
// earlier levels (the order of the launch-per-step sequence, kept per entry
// instead of over the whole batch), and run the same tile code on the same
// data, so the factor is bitwise the launch-per-step one.  A ticket counter
// hands out the tasks in chunks (the tasks of one entry at one level, in
// an order chosen by the host that keeps every entry's levels in sequence); a
// work-group waits until its entry has completed all its tasks of the earlier
// levels (a per-entry counter).  Every task waited on holds a smaller ticket,
// so it is running or done: the launch cannot deadlock whatever the number of
// resident work-groups.  Matrix data that crosses work-groups is read and
// written device-coherently; a task's counter increment follows the
// completion of all its stores (store-counter wait and barrier), and its reads
// follow the counter load.  The waits are bounded: past the bound (a guard
// against an earlier fault only) the launch sets err and every work-group
// leaves.
struct FusedPlan {
  const int *base;  // [C + 1] first ticket of each chunk
  const int *code;  // [C] level of the chunk: panel * 3 PB + step in the panel
  const int *ent;   // [C] batch entry of the chunk
  const int *need;  // [C] tasks of the entry in its earlier levels
  int C, total;
  int mt_update;    // row tile of the update step: 32 mt_update rows
};
constexpr int kFusedCtl = 4;  // ctl[0] ticket counter, ctl[1] abort flag, then B counters
constexpr long long kFusedWaitTicks = 400000000LL;  // wall-clock ticks (100 MHz: 4 s)

// largest j in [0, n) with a[j] <= key (a ascending, a[0] <= key); called by
// all lanes of one wave: 64-ary search, one load per lane and step
__device__ int wave_floor(const int *a, int n, int key) {
  const int lane = threadIdx.x & 63;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int step = (hi - lo + 63) / 64;
    const int idx = lo + lane * step;
    const bool ok = idx < hi && a[idx] <= key;
    const int cnt = __popcll(__ballot(ok));  // a prefix of the lanes (a ascending); lane 0 holds
    lo = lo + (cnt - 1) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// bounded wait until *cnt >= need; false (the launch is aborted) past the bound
// or when another work-group aborted
__device__ bool fused_wait(int *cnt, int need, int *abort, int *err) {
  const long long t0 = wall_clock64();
  for (int it = 0;; ++it) {
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
    if ((it & 31) == 31) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
      if (wall_clock64() - t0 > kFusedWaitTicks) {
        atomicExch(abort, 1);
        atomicExch(err, 1);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

template <class T>
constexpr int fused_lds() {
  return gemm_tile_lds<T, 4, 4, 1>() > 2 * NB * (NB + 1) ? gemm_tile_lds<T, 4, 4, 1>()
                                                         : 2 * NB * (NB + 1);
}

// One task per work-group: the work-group takes the next ticket (not its
// block index), so every task it waits on holds a smaller ticket, taken by a
// work-group that is running or done.
template <class T>
__global__ __launch_bounds__(256) void potrf_fused_kernel(T *pool, const MatDesc *desc, int *status,
                                                          T *dinv, const int64_t *dinv_off,
                                                          const FusedPlan plan, int *ctl, int *err) {
  static_assert(gemm_tile_lds<T, 4, 2, 1>() <= fused_lds<T>() &&
                gemm_tile_lds<T, 2, 2, 1>() <= fused_lds<T>(), "LDS of the fused launch");
  __shared__ T smem[fused_lds<T>()];
  __shared__ int s_task[4];
  int *done = ctl + kFusedCtl;
  constexpr int LPP = 3 * PB;
  if (threadIdx.x < 64) {  // wave 0: take a ticket, decode it, wait for the entry
    int ticket = 0;
    if (threadIdx.x == 0) ticket = atomicAdd(&ctl[0], 1);
    ticket = __shfl(ticket, 0);
    int ch = 0, tile = 0, stop = 1;
    if (ticket < plan.total &&
        __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      ch = wave_floor(plan.base, plan.C, ticket);
      tile = ticket - plan.base[ch];
      if (threadIdx.x == 0)
        stop = fused_wait(&done[plan.ent[ch]], plan.need[ch], &ctl[1], err) ? 0 : 1;
      stop = __shfl(stop, 0);
    }
    if (threadIdx.x == 0) {
      s_task[0] = ch;
      s_task[1] = tile;
      s_task[2] = stop;
    }
  }
  __syncthreads();
  const int ch = s_task[0], tile = s_task[1];
  if (s_task[2]) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const int e = plan.ent[ch];
  const MatDesc d = desc[e];
  const int code = plan.code[ch];
  const int k0 = (code / LPP) * PB, sp = code % LPP;
  if (sp == LPP - 1) {
    chol_syrk_tile<T, true>(smem, pool, d, k0 * NB, (k0 + PB) * NB, tile);
  } else {
    const int j = sp < 2 ? 0 : (sp - 2) / 3 + 1, r = sp < 2 ? sp + 1 : (sp - 2) % 3;
    const int k = k0 + j;
    T *Di = dinv + dinv_off[e] + (int64_t)k * NB * NB;
    if (r == 0) {
      if (plan.mt_update == 4)
        chol_update_tile<T, 4, true>(smem, pool, d, k, k0, tile);
      else
        chol_update_tile<T, 2, true>(smem, pool, d, k, k0, tile);
    } else if (r == 1) {
      chol_diag_block<T, true>(pool, d, k, status ? status + e : nullptr, Di,
                               reinterpret_cast<T(*)[NB + 1]>(smem),
                               reinterpret_cast<T(*)[NB + 1]>(smem + NB * (NB + 1)));
    } else {
      chol_panel_tile<T, true>(smem, pool, d, k, tile, Di);
    }
  }
  // every store of the task acknowledged before the entry's counter moves
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[e], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void zero_ints_kernel(int *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

}  // namespace bddc

// --------------------------------------------------------------------------
// host wrappers

namespace bddc {

LaunchTiming *&launch_timing() {
  static thread_local LaunchTiming *slot = nullptr;
  return slot;
}

namespace {
inline int grid_round(int n) {
  const int g = NXCD * (kXcdChunk > 1 ? kXcdChunk : 1);
  return ((n + g - 1) / g) * g;
}
// the tile map of a launch, cnt(e) tiles for entry e; map.n = 0 (not used)
// when the batch has more entries than a map holds
template <class F>
TileMap tile_map(int batch, F cnt) {
  TileMap m;
  m.n = 0;
  m.xb[NXCD] = 0;
  if (batch <= 0 || batch > kMaxMapEntries) return m;
  m.off[0] = 0;
  for (int e = 0; e < batch; ++e) m.off[e + 1] = m.off[e] + std::max(0, cnt(e));
  m.n = batch;
  return m;
}
// Consecutive tiles in whole runs per XCD, the runs cut where the summed
// cost (cost(e) per tile of entry e) reaches each eighth of the total: every
// XCD gets an equal share of the work and mostly whole entries (their
// operand panels stay in one L2).  Returns the grid.
template <class F>
int xcd_balance(TileMap &m, F cost) {
  if (m.n <= 0 || m.off[m.n] <= 0) return 0;
  double tot = 0;
  for (int e = 0; e < m.n; ++e) tot += (double)(m.off[e + 1] - m.off[e]) * std::max(1.0, (double)cost(e));
  m.xb[0] = 0;
  int x = 1;
  double acc = 0;
  for (int e = 0; e < m.n && x < NXCD; ++e) {
    const double c = std::max(1.0, (double)cost(e));
    for (int t = m.off[e]; t < m.off[e + 1] && x < NXCD; ++t) {
      acc += c;
      while (x < NXCD && acc >= tot * x / NXCD) m.xb[x++] = t + 1;
    }
  }
  while (x < NXCD) m.xb[x++] = m.off[m.n];
  m.xb[NXCD] = m.off[m.n];
  int share = 0;
  for (int q = 0; q < NXCD; ++q) share = std::max(share, m.xb[q + 1] - m.xb[q]);
  return NXCD * share;
}
inline int blk(int n, int k) { return std::max(0, std::min(NB, n - k * NB)); }
}  // namespace

#define HIP_RETURN_IF(x)            \
  do {                              \
    hipError_t e_ = (x);            \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// --- GEMM tile autotuning ---------------------------------------------------
// A shape signature (element size, transposes, lower, batch, largest M, N, K)
// maps to the tile shape measured fastest on its first call.  Every candidate
// accumulates each entry of C over K in the same order (KS = 1, MFMA K-steps
// ascending), so they give the same bits and the choice changes only time.
struct TuneKey {
  int elem;
  bool ta, tb, lower;
  int batch, maxM, maxN, maxK;
  bool operator<(const TuneKey &o) const {
    return std::tie(elem, ta, tb, lower, batch, maxM, maxN, maxK) <
           std::tie(o.elem, o.ta, o.tb, o.lower, o.batch, o.maxM, o.maxN, o.maxK);
  }
};
constexpr int N_TILE_SHAPES = 4;  // 128 x 128, 64 x 64, 128 x 64, 64 x 128

std::mutex &tune_mutex() {
  static std::mutex m;
  return m;
}
std::map<TuneKey, int> &tune_table() {
  static std::map<TuneKey, int> t;
  return t;
}
int tune_lookup(const TuneKey &k) {
  std::lock_guard<std::mutex> g(tune_mutex());
  auto it = tune_table().find(k);
  return it == tune_table().end() ? -1 : it->second;
}
void tune_store(const TuneKey &k, int shape) {
  std::lock_guard<std::mutex> g(tune_mutex());
  tune_table().emplace(k, shape);
}

// Times every tile shape on the call's own operands: C (the span the batch
// writes, which also covers A or B where they alias it) is saved first and
// restored before each further trial and before the final launch by the
// caller, so the call's result is that of one product.  Returns the fastest
// shape (the default one on ties), or -1 after a HIP error.
template <class T, class Launch>
int tune_gemm(hipStream_t st, T *C, const GemmDesc *h, int batch, int dflt, Launch &launch) {
  int64_t lo = INT64_MAX, hi = 0;
  for (int e = 0; e < batch; ++e) {
    if (h[e].M <= 0 || h[e].N <= 0) continue;
    lo = std::min(lo, h[e].c_off);
    hi = std::max(hi, h[e].c_off + (int64_t)h[e].ldc * (h[e].N - 1) + h[e].M);
  }
  if (hi <= lo) return dflt;
  const size_t bytes = sizeof(T) * (size_t)(hi - lo);
  void *save = nullptr;
  if (hipMallocAsync(&save, bytes, st) != hipSuccess) {
    (void)hipGetLastError();  // no room for the copy: keep the default shape, untuned
    return dflt;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    (void)hipFreeAsync(save, st);
    return -1;
  }
  float best = 0;
  int pick = dflt;
  bool ok = hipMemcpyAsync(save, C + lo, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess;
  for (int q = 0; q < N_TILE_SHAPES && ok; ++q) {
    const int shape = (dflt + q) % N_TILE_SHAPES;  // the default first
    if (q > 0) ok = hipMemcpyAsync(C + lo, save, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess;
    ok = ok && hipEventRecord(ev[0], st) == hipSuccess;
    if (ok) launch(shape);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(ev[1], st) == hipSuccess &&
         hipEventSynchronize(ev[1]) == hipSuccess;
    float ms = 0;
    ok = ok && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess;
    if (ok && (q == 0 || ms < best)) best = ms, pick = shape;
  }
  ok = ok && hipMemcpyAsync(C + lo, save, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess;
  ok = hipFreeAsync(save, st) == hipSuccess && ok;
  ok = hipEventDestroy(ev[0]) == hipSuccess && ok;
  ok = hipEventDestroy(ev[1]) == hipSuccess && ok;
  return ok ? pick : -1;
}

bool &autotune_enabled() {
  static thread_local bool on = false;
  return on;
}

bool &per_entry_launches() {
  static thread_local bool on = false;
  return on;
}

DevAlloc *&fused_workspace() {
  static thread_local DevAlloc *slot = nullptr;
  return slot;
}

int64_t &fused_max_tasks() {
  static thread_local int64_t limit = kFusedAutoTasks;
  return limit;
}

int64_t autotune_entries() {
  std::lock_guard<std::mutex> g(tune_mutex());
  return (int64_t)tune_table().size();
}

template <class T, int MT, int NT>
static void launch_gemm(hipStream_t st, const T *A, const T *B, T *C, const GemmDesc *d_desc,
                        int batch, int maxM, int maxN, bool transA, bool transB, T alpha, T beta,
                        bool lower, const GemmDesc *h_desc) {
  constexpr int TM = 32 * MT, TN = 32 * NT;
  const int tm = (maxM + TM - 1) / TM, tn = (maxN + TN - 1) / TN;
  // with the host descriptors, each entry's own tiles only (lower: square
  // tiles of square products, the lower triangle's tiles)
  TileMap map;
  map.n = 0;
  bool can_map = h_desc != nullptr && (!lower || TM == TN);
  for (int e = 0; can_map && lower && e < batch; ++e) can_map = h_desc[e].M == h_desc[e].N;
  if (can_map)
    map = tile_map(batch, [&](int e) {
      const GemmDesc &q = h_desc[e];
      if (q.M <= 0 || q.N <= 0) return 0;
      const int a = (q.M + TM - 1) / TM, b = (q.N + TN - 1) / TN;
      return lower ? a * (a + 1) / 2 : a * b;
    });
  const int nt = map.n > 0 ? map.off[map.n] : batch * tm * tn;
  if (nt <= 0) return;
  // tiles of different entries differ in cost by their K: XCD shares by cost
  const int gb = map.n > 0 ? xcd_balance(map, [&](int e) { return h_desc[e].K; }) : 0;
  const dim3 g(gb > 0 ? gb : grid_round(nt)), b(256);
  if (!transA && !transB)
    gemm_kernel<T, false, false, MT, NT><<<g, b, 0, st>>>(A, B, C, d_desc, tm, tn, alpha, beta, lower, batch, map);
  else if (transA && !transB)
    gemm_kernel<T, true, false, MT, NT><<<g, b, 0, st>>>(A, B, C, d_desc, tm, tn, alpha, beta, lower, batch, map);
  else if (!transA && transB)
    gemm_kernel<T, false, true, MT, NT><<<g, b, 0, st>>>(A, B, C, d_desc, tm, tn, alpha, beta, lower, batch, map);
  else
    gemm_kernel<T, true, true, MT, NT><<<g, b, 0, st>>>(A, B, C, d_desc, tm, tn, alpha, beta, lower, batch, map);
}

template <class T>
hipError_t DenseOps<T>::gemm(hipStream_t st, const T *A, const T *B, T *C, const GemmDesc *d_desc,
                             int batch, int maxM, int maxN, bool transA, bool transB, T alpha,
                             T beta, bool lower, const GemmDesc *h_desc) {
  if (batch <= 0 || maxM <= 0 || maxN <= 0) return hipSuccess;
  if (per_entry_launches() && batch > 1 && h_desc) {
    for (int e = 0; e < batch; ++e)
      if (h_desc[e].M > 0 && h_desc[e].N > 0)
        HIP_RETURN_IF(gemm(st, A, B, C, d_desc + e, 1, h_desc[e].M, h_desc[e].N, transA, transB, alpha,
                           beta, lower, h_desc + e));
    return hipSuccess;
  }
  // batches larger than a tile map: sub-batches that each launch only
  // their entries' own tiles
  if (batch > kMaxMapEntries && h_desc) {
    for (int e0 = 0; e0 < batch; e0 += kMaxMapEntries)
      HIP_RETURN_IF(gemm(st, A, B, C, d_desc + e0, std::min(kMaxMapEntries, batch - e0), maxM, maxN,
                         transA, transB, alpha, beta, lower, h_desc + e0));
    return hipSuccess;
  }
  double fl = 0, by = 0;
  if (launch_timing() && h_desc)
    for (int e = 0; e < batch; ++e) {
      const GemmDesc &q = h_desc[e];
      const double mn = lower ? 0.5 * (double)q.M * (q.N + 1) : (double)q.M * q.N;
      fl += 2.0 * mn * q.K;
      by += sizeof(T) * ((double)q.M * q.K + (double)q.K * q.N + (beta != T(0) ? 2.0 : 1.0) * mn);
    }
  LaunchScope ls(st, "gemm_kernel", by, fl);
  auto launch = [&](int shape) {
    switch (shape) {
      case 0: launch_gemm<T, 4, 4>(st, A, B, C, d_desc, batch, maxM, maxN, transA, transB, alpha, beta, lower, h_desc); break;
      case 1: launch_gemm<T, 2, 2>(st, A, B, C, d_desc, batch, maxM, maxN, transA, transB, alpha, beta, lower, h_desc); break;
      case 2: launch_gemm<T, 4, 2>(st, A, B, C, d_desc, batch, maxM, maxN, transA, transB, alpha, beta, lower, h_desc); break;
      default: launch_gemm<T, 2, 4>(st, A, B, C, d_desc, batch, maxM, maxN, transA, transB, alpha, beta, lower, h_desc); break;
    }
  };
  // 128 x 128 tiles for large products, 64 x 64 otherwise, unless the tuner
  // has measured this shape
  int shape = (maxM >= 256 && maxN >= 256) ? 0 : 1;
  if (autotune_enabled() && h_desc && !per_entry_launches()) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_RETURN_IF(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      TuneKey key{sizeof(T), transA, transB, lower, batch, maxM, maxN, 0};
      for (int e = 0; e < batch; ++e) key.maxK = std::max(key.maxK, h_desc[e].K);
      int found = tune_lookup(key);
      if (found < 0) {
        found = tune_gemm(st, C, h_desc, batch, shape, launch);
        if (found < 0) return hipGetLastError();
        tune_store(key, found);
      }
      shape = found;
    }
  }
  launch(shape);
  return hipGetLastError();
}

template <class T>
hipError_t DenseOps<T>::gemm_scatter(hipStream_t st, const T *A, const T *B, T *C,
                                     const GemmDesc *d_desc, const int *map, const int64_t *map_off,
                                     bool map_rows, int batch, int maxM, int maxN,
                                     const GemmDesc *h_desc) {
  if (batch <= 0 || maxM <= 0 || maxN <= 0) return hipSuccess;
  if (per_entry_launches() && batch > 1 && h_desc) {
    for (int e = 0; e < batch; ++e)
      if (h_desc[e].M > 0 && h_desc[e].N > 0)
        HIP_RETURN_IF(gemm_scatter(st, A, B, C, d_desc + e, map, map_off + e, map_rows, 1,
                                   h_desc[e].M, h_desc[e].N, h_desc + e));
    return hipSuccess;
  }
  if (batch > kMaxMapEntries && h_desc) {  // sub-batches, as in gemm
    for (int e0 = 0; e0 < batch; e0 += kMaxMapEntries)
      HIP_RETURN_IF(gemm_scatter(st, A, B, C, d_desc + e0, map, map_off + e0, map_rows,
                                 std::min(kMaxMapEntries, batch - e0), maxM, maxN, h_desc + e0));
    return hipSuccess;
  }
  double fl = 0, by = 0;
  if (launch_timing() && h_desc)
    for (int e = 0; e < batch; ++e) {
      const GemmDesc &q = h_desc[e];
      fl += 2.0 * q.M * q.N * q.K;
      by += sizeof(T) * ((double)q.M * q.K + (double)q.K * q.N + 2.0 * q.M * q.N) + 4.0 * (map_rows ? q.M : q.N);
    }
  LaunchScope ls(st, "gemm_scatter_kernel", by, fl);
  const int tm = (maxM + 63) / 64, tn = (maxN + 63) / 64;
  TileMap tmap;
  tmap.n = 0;
  if (h_desc)
    tmap = tile_map(batch, [&](int e) {
      return h_desc[e].M > 0 && h_desc[e].N > 0 ? ((h_desc[e].M + 63) / 64) * ((h_desc[e].N + 63) / 64) : 0;
    });
  const int nt = tmap.n > 0 ? tmap.off[tmap.n] : batch * tm * tn;
  if (nt <= 0) return hipSuccess;
  gemm_scatter_kernel<T, 2, 2><<<grid_round(nt), 256, 0, st>>>(
      A, B, C, d_desc, map, map_off, map_rows ? 1 : 0, tm, tn, batch, tmap);
  return hipGetLastError();
}

// Panels of PB block columns: within a panel each block column is updated
// by the panel's columns to its left (chol_update_kernel, short K), its
// diagonal block factored and inverted (chol_diag_kernel) and the rows below
// solved (chol_panel_kernel); then the whole trailing matrix is updated by
// the panel at once (chol_syrk_kernel, 128 x 128 tiles, K = PB NB), so most
// flops run as large tile products with many work-groups (PB: the panel
// width in blocks, defined with the kernels).

// The fused Cholesky (potrf_fused_kernel): the host lists, per level, the
// tasks of every entry (largest entries first), uploads the tables with the
// workspace's memory, clears the counters, launches once and checks the
// abort flag (one synchronization).
template <class T>
hipError_t potrf_fused(hipStream_t st, T *pool, const MatDesc *d_desc, const MatDesc *h_desc,
                       int batch, int *status, T *dinv, const int64_t *dinv_off, DevAlloc &ws,
                       int64_t max_tasks, bool &used) {
  used = false;
  int maxn = 0;
  for (int e = 0; e < batch; ++e) maxn = std::max(maxn, h_desc[e].n);
  if (maxn == 0) return hipSuccess;
  const int nblk = (maxn + NB - 1) / NB, panels = (nblk + PB - 1) / PB, LPP = 3 * PB;
  // the update step's row tile: 128 rows when the batch fills the device
  // several times over with them (as the launch-per-step path decides per
  // column), else 64
  int64_t t128 = 0;
  for (int e = 0; e < batch; ++e) t128 += (std::max(0, h_desc[e].n - NB) + 127) / 128;
  const int mt = t128 >= 2048 ? 4 : 2, tmu = 32 * mt;
  auto tasks = [&](int n, int code) -> int64_t {
    const int k0 = (code / LPP) * PB, sp = code % LPP, nb = (n + NB - 1) / NB;
    if (sp == LPP - 1) {
      const int64_t p1 = (int64_t)(k0 + PB) * NB;
      if (p1 >= n) return 0;
      const int64_t a = (n - p1 + 127) / 128;
      return a * (a + 1) / 2;
    }
    const int j = sp < 2 ? 0 : (sp - 2) / 3 + 1, r = sp < 2 ? sp + 1 : (sp - 2) % 3, k = k0 + j;
    if (k >= nb) return 0;
    if (r == 0) return (n - k * NB + tmu - 1) / tmu;
    if (r == 1) return 1;
    return nb - k - 1;
  };
  // chunks (entry, level) with tasks, each entry's in level order
  struct Chunk {
    int code, e;
    int64_t cnt, need;
  };
  std::vector<int> order(batch);
  for (int e = 0; e < batch; ++e) order[e] = e;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h_desc[a].n > h_desc[b].n; });
  std::vector<Chunk> chunks;
  std::vector<int64_t> cum(batch, 0);
  for (int c = 0; c < panels * LPP; ++c)
    for (int e : order) {
      const int64_t t = tasks(h_desc[e].n, c);
      if (t == 0) continue;
      chunks.push_back(Chunk{c, e, t, cum[e]});
      cum[e] += t;
    }
  // entries staggered by phase: entry of rank q starts q mod 3 levels late,
  // so the latency-bound diagonal steps of some entries overlap the tile
  // products of others (measured 3-7% faster than all entries in step)
  {
    std::vector<int> len(batch, 0), rank(batch, 0), idx(chunks.size());
    for (int i = 0; i < batch; ++i) rank[order[i]] = i;
    for (size_t i = 0; i < chunks.size(); ++i) idx[i] = len[chunks[i].e]++;
    std::vector<std::tuple<int, int, int>> key(chunks.size());
    for (size_t i = 0; i < chunks.size(); ++i) {
      const int e = chunks[i].e;
      key[i] = std::make_tuple(idx[i] + rank[e] % 3, rank[e], (int)i);
    }
    std::vector<size_t> perm(chunks.size());
    for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
    std::sort(perm.begin(), perm.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
    std::vector<Chunk> sorted(chunks.size());
    for (size_t i = 0; i < perm.size(); ++i) sorted[i] = chunks[perm[i]];
    chunks.swap(sorted);
  }
  const int C = (int)chunks.size();
  int64_t ntask = 0;
  for (const Chunk &q : chunks) ntask += q.cnt;
  if (ntask > max_tasks) return hipSuccess;  // declined: one launch per step
  used = true;
  if (C == 0) return hipSuccess;
  std::vector<int> plan;
  plan.reserve(4 * (size_t)C + 1);
  int64_t total = 0;
  for (const Chunk &q : chunks) {
    plan.push_back((int)total);
    total += q.cnt;
    if (total >= INT_MAX / 2) return hipErrorInvalidValue;
  }
  plan.push_back((int)total);
  const size_t o_base = 0, o_code = C + 1, o_ent = o_code + C, o_need = o_ent + C, o_ctl = o_need + C;
  for (const Chunk &q : chunks) plan.push_back(q.code);
  for (const Chunk &q : chunks) plan.push_back(q.e);
  for (const Chunk &q : chunks) plan.push_back((int)q.need);
  const int nctl = kFusedCtl + batch + 1;  // counters, then the abort report
  const size_t bytes = sizeof(int) * (o_ctl + nctl);
  int *w = static_cast<int *>(ws.get(bytes));
  hipError_t rc = hipMemcpyAsync(w, plan.data(), sizeof(int) * plan.size(), hipMemcpyHostToDevice, st);
  int *ctl = w + o_ctl, *err = ctl + kFusedCtl + batch;
  if (rc == hipSuccess) {
    zero_ints_kernel<<<(nctl + 255) / 256, 256, 0, st>>>(ctl, nctl);
    rc = hipGetLastError();
  }
  if (rc == hipSuccess) {
    FusedPlan fp{w + o_base, w + o_code, w + o_ent, w + o_need, C, (int)total, mt};
    const int grid = (int)total;  // one task per work-group
    double fl = 0, by = 0;
    if (launch_timing())
      for (int e = 0; e < batch; ++e) {
        const double n = h_desc[e].n;
        fl += n * n * n / 3.0;
        by += sizeof(T) * n * n;
      }
    LaunchScope ls(st, "potrf_fused_kernel", by, fl);
    potrf_fused_kernel<T><<<grid, 256, 0, st>>>(pool, d_desc, status, dinv, dinv_off, fp, ctl, err);
    rc = hipGetLastError();
  }
  int herr = 0;
  if (rc == hipSuccess) rc = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st);
  if (rc == hipSuccess) rc = hipStreamSynchronize(st);
  ws.put(w, bytes);
  if (rc != hipSuccess) return rc;
  return herr ? hipErrorLaunchTimeOut : hipSuccess;
}

template <class T>
hipError_t DenseOps<T>::potrf(hipStream_t st, T *pool, const MatDesc *d_desc,
                              const MatDesc *h_desc, int batch, int *status, T *dinv,
                              const int64_t *dinv_off) {
  if (per_entry_launches() && batch > 1) {
    for (int e = 0; e < batch; ++e)
      HIP_RETURN_IF(potrf(st, pool, d_desc + e, h_desc + e, 1, status ? status + e : nullptr, dinv,
                          dinv_off + e));
    return hipSuccess;
  }
  if (!per_entry_launches() && fused_workspace() && fused_max_tasks() > 0) {
    bool used = false;
    HIP_RETURN_IF(potrf_fused<T>(st, pool, d_desc, h_desc, batch, status, dinv, dinv_off,
                                 *fused_workspace(), fused_max_tasks(), used));
    if (used) return hipSuccess;
  }
  if (batch > kMaxMapEntries) {  // sub-batches, as in gemm
    for (int e0 = 0; e0 < batch; e0 += kMaxMapEntries)
      HIP_RETURN_IF(potrf(st, pool, d_desc + e0, h_desc + e0, std::min(kMaxMapEntries, batch - e0),
                          status ? status + e0 : nullptr, dinv, dinv_off + e0));
    return hipSuccess;
  }
  int maxn = 0;
  for (int e = 0; e < batch; ++e) maxn = std::max(maxn, h_desc[e].n);
  if (maxn == 0) return hipSuccess;
  const int nblk = (maxn + NB - 1) / NB;
  const bool timing = launch_timing() != nullptr;
  for (int k0 = 0; k0 < nblk; k0 += PB) {
    const int k1 = std::min(nblk, k0 + PB);
    for (int k = k0; k < k1; ++k) {
      const int tm = nblk - k;  // row blocks of block column k (for the largest entry)
      const int tu = (maxn - k * NB + 127) / 128;  // 128-row update tiles
      // algorithmic work of block column k over the batch: the update of the
      // column below the diagonal by the panel's columns to its left, the
      // factorization of the diagonal block, and the panel solve under it
      double fu = 0, bu = 0, fd = 0, bd = 0, fp = 0, bp = 0;
      if (timing)
        for (int e = 0; e < batch; ++e) {
          const double nb = blk(h_desc[e].n, k);
          if (nb == 0) continue;
          const double m = h_desc[e].n - (double)k * NB, kk = (double)(k - k0) * NB, below = m - nb;
          fu += 2.0 * (m * nb - 0.5 * nb * (nb - 1)) * kk;
          bu += sizeof(T) * (m * kk + nb * kk + 2.0 * m * nb);
          fd += nb * nb * nb / 3.0;
          bd += sizeof(T) * nb * nb;
          fp += below * nb * nb;
          bp += sizeof(T) * (2.0 * below * nb + 0.5 * nb * nb);
        }
      // the tiles of the rows from block k down, per entry (rows of rt each)
      auto rows_map = [&](int rt, int skip) {
        return tile_map(batch, [&](int e) {
          const int m = h_desc[e].n - k * NB;
          return m > 0 ? (m + rt - 1) / rt - skip : 0;
        });
      };
      if (k > k0) {
        LaunchScope ls(st, "chol_update_kernel", bu, fu);
        if (batch * tu >= 2048) {  // 128-row tiles only when they fill the device several times
          const TileMap map = rows_map(128, 0);
          const int nt = map.n > 0 ? map.off[map.n] : batch * tu;
          if (nt > 0)
            chol_update_kernel<T, 4><<<grid_round(nt), 256, 0, st>>>(pool, d_desc, k, k0, tu, batch, map);
        } else {
          const int t64 = (maxn - k * NB + 63) / 64;
          const TileMap map = rows_map(64, 0);
          const int nt = map.n > 0 ? map.off[map.n] : batch * t64;
          if (nt > 0)
            chol_update_kernel<T, 2><<<grid_round(nt), 256, 0, st>>>(pool, d_desc, k, k0, t64, batch, map);
        }
      }
      {
        LaunchScope ls(st, "chol_diag_kernel", bd, fd);
        chol_diag_kernel<T><<<batch, 64, 0, st>>>(pool, d_desc, k, status, batch, dinv, dinv_off);
      }
      if (tm > 1) {
        LaunchScope ls(st, "chol_panel_kernel", bp, fp);
        const TileMap map = rows_map(NB, 1);  // the blocks below the diagonal one
        const int nt = map.n > 0 ? map.off[map.n] : batch * (tm - 1);
        if (nt > 0)
          chol_panel_kernel<T><<<grid_round(nt), 256, 0, st>>>(pool, d_desc, k, tm - 1, batch, dinv,
                                                               dinv_off, map);
      }
    }
    const int p0 = k0 * NB, p1 = k1 * NB;
    if (p1 < maxn) {
      const int tm = (maxn - p1 + 127) / 128;
      double fs = 0, bs = 0;
      if (timing)
        for (int e = 0; e < batch; ++e) {
          const double m = h_desc[e].n - (double)p1;
          if (m <= 0) continue;
          fs += m * (m + 1) * (p1 - p0);
          bs += sizeof(T) * (m * (p1 - p0) + m * (m + 1));
        }
      LaunchScope ls(st, "chol_syrk_kernel", bs, fs);
      TileMap map = tile_map(batch, [&](int e) {
        const int a = (h_desc[e].n - p1 + 127) / 128;
        return h_desc[e].n > p1 ? a * (a + 1) / 2 : 0;
      });
      const int nt = map.n > 0 ? map.off[map.n] : batch * (tm * (tm + 1) / 2);
      // tiles of equal cost (K = the panel width): equal runs of consecutive
      // tiles per XCD
      const int gb = map.n > 0 ? xcd_balance(map, [](int) { return 1; }) : 0;
      if (nt > 0)
        chol_syrk_kernel<T><<<gb > 0 ? gb : grid_round(nt), 256, 0, st>>>(pool, d_desc, p0, p1, tm, batch, map);
    }
  }
  return hipGetLastError();
}

// Panels of PB block rows, as in potrf: inside a panel, block rows are
// updated by the panel's solved rows (trsm_update_kernel, short K) and solved
// with the inverse diagonal blocks (trsm_diag_kernel); then every row outside
// the panel on the unsolved side is updated by the whole panel at once
// (trsm_gemm_kernel, 128-row tiles, K = PB NB).
template <class T>
hipError_t DenseOps<T>::trsm(hipStream_t st, T *pool_a, T *pool_b, const MatDesc *d_desc,
                             const MatDesc *h_desc, int batch, bool transpose, const T *dinv,
                             const int64_t *dinv_off) {
  if (per_entry_launches() && batch > 1) {
    for (int e = 0; e < batch; ++e)
      HIP_RETURN_IF(trsm(st, pool_a, pool_b, d_desc + e, h_desc + e, 1, transpose, dinv, dinv_off + e));
    return hipSuccess;
  }
  if (batch > kMaxMapEntries) {  // sub-batches, as in gemm
    for (int e0 = 0; e0 < batch; e0 += kMaxMapEntries)
      HIP_RETURN_IF(trsm(st, pool_a, pool_b, d_desc + e0, h_desc + e0, std::min(kMaxMapEntries, batch - e0),
                         transpose, dinv, dinv_off + e0));
    return hipSuccess;
  }
  int maxn = 0, maxr = 0;
  for (int e = 0; e < batch; ++e) {
    maxn = std::max(maxn, h_desc[e].n);
    maxr = std::max(maxr, h_desc[e].nrhs);
  }
  if (maxn == 0 || maxr == 0) return hipSuccess;
  const int nblk = (maxn + NB - 1) / NB;
  const int tn = (maxr + NB - 1) / NB;    // 64-wide column tiles (diagonal step)
  const int tu = (maxr + 127) / 128;      // 128-wide column tiles (update)

  // few tiles: 32-wide tiles, two groups of waves per tile splitting K
  const bool narrow = batch * tu < 512;
  // the column tiles (cw columns each) of the entries that have work at
  // block row k: below the panel start (forward) or with solved rows of the
  // panel below block k (backward)
  auto col_map = [&](int cw, int k, int p0, int p1, int mode) {
    return tile_map(batch, [&](int e) {
      const int n = h_desc[e].n, kb = k * NB;
      if (kb >= n) return 0;
      if (mode == 1 && kb <= p0) return 0;
      if (mode == 2 && std::min(p1, n) - kb - std::min(NB, n - kb) <= 0) return 0;
      return (h_desc[e].nrhs + cw - 1) / cw;
    });
  };
  // few tiles: the update and the diagonal product as two launches, the
  // update with 32-column tiles (twice the work-groups of 64-column ones; the
  // same sums, in the same order)
  auto update = [&](bool bwd, int k, int p0, int p1) {
    const int t32 = (maxr + 31) / 32;
    const TileMap map = col_map(32, k, p0, p1, bwd ? 2 : 1);
    const int nt = map.n > 0 ? map.off[map.n] : batch * t32;
    if (nt <= 0) return;
    if (bwd)
      trsm_update_kernel<T, true, 1, 2><<<grid_round(nt), 512, 0, st>>>(pool_a, pool_b, d_desc, k, p0, p1,
                                                                       t32, batch, map);
    else
      trsm_update_kernel<T, false, 1, 2><<<grid_round(nt), 512, 0, st>>>(pool_a, pool_b, d_desc, k, p0, p1,
                                                                        t32, batch, map);
  };
  // update and diagonal product of block row k in one launch (wide case)
  auto step = [&](bool bwd, int k, int p0, int p1) {
    const TileMap map = col_map(128, k, p0, p1, 0);
    const int nt = map.n > 0 ? map.off[map.n] : batch * tu;
    if (nt <= 0) return;
    if (bwd)
      trsm_step_kernel<T, true><<<grid_round(nt), 256, 0, st>>>(pool_a, pool_b, d_desc, k, p0, p1, tu, batch,
                                                                dinv, dinv_off, map);
    else
      trsm_step_kernel<T, false><<<grid_round(nt), 256, 0, st>>>(pool_a, pool_b, d_desc, k, p0, p1, tu, batch,
                                                                 dinv, dinv_off, map);
  };
  auto diag = [&](bool bwd, int k) {
    const TileMap map = col_map(NB, k, 0, 0, 0);
    const int nt = map.n > 0 ? map.off[map.n] : batch * tn;
    if (nt <= 0) return;
    if (bwd)
      trsm_diag_kernel<T, true><<<grid_round(nt), 256, 0, st>>>(pool_a, pool_b, d_desc, k, tn, batch, dinv,
                                                                dinv_off, map);
    else
      trsm_diag_kernel<T, false><<<grid_round(nt), 256, 0, st>>>(pool_a, pool_b, d_desc, k, tn, batch, dinv,
                                                                 dinv_off, map);
  };
  // rows outside the panel [p0, p1): below it (forward) or above it (backward)
  auto panel_gemm = [&](bool bwd, int p0, int p1) {
    const int rows = bwd ? p0 : maxn - p1;
    if (rows <= 0) return;
    const int tm = (rows + 127) / 128;
    double fg = 0, bg = 0;
    if (launch_timing())
      for (int e = 0; e < batch; ++e) {
        const double n = h_desc[e].n, r = h_desc[e].nrhs;
        const double m = bwd ? (n > p0 ? p0 : 0) : std::max(0.0, n - p1);
        const double kk = bwd ? std::max(0.0, std::min((double)p1, n) - p0) : (n > p1 ? p1 - p0 : 0);
        if (m <= 0 || kk <= 0) continue;
        fg += 2.0 * m * r * kk;
        bg += sizeof(T) * (m * kk + kk * r + 2.0 * m * r);
      }
    LaunchScope ls(st, bwd ? "trsm_gemm_kernel<bwd>" : "trsm_gemm_kernel<fwd>", bg, fg);
    const int tw = maxr >= 128 ? 128 : 64;  // right-hand-side columns per tile
    const int tq = (maxr + tw - 1) / tw;
    // each entry's own tiles: its row tiles on the unsolved side times its
    // column tiles
    TileMap map = tile_map(batch, [&](int e) {
      const int n = h_desc[e].n;
      const int r = bwd ? (p0 < std::min(p1, n) ? p0 : 0) : std::max(0, n - p1);
      return ((r + 127) / 128) * ((h_desc[e].nrhs + tw - 1) / tw);
    });
    const int nt = map.n > 0 ? map.off[map.n] : batch * tm * tq;
    if (nt <= 0) return;
    // equal runs of consecutive tiles per XCD (tiles of equal cost)
    const int gb = map.n > 0 ? xcd_balance(map, [](int) { return 1; }) : 0;
    const unsigned g = gb > 0 ? gb : grid_round(nt);
    if (tw == 128) {
      if (bwd)
        trsm_gemm_kernel<T, true, 4><<<g, 256, 0, st>>>(pool_a, pool_b, d_desc, p0, p1, tm, tq, batch, map);
      else
        trsm_gemm_kernel<T, false, 4><<<g, 256, 0, st>>>(pool_a, pool_b, d_desc, p0, p1, tm, tq, batch, map);
    } else {
      if (bwd)
        trsm_gemm_kernel<T, true, 2><<<g, 256, 0, st>>>(pool_a, pool_b, d_desc, p0, p1, tm, tq, batch, map);
      else
        trsm_gemm_kernel<T, false, 2><<<g, 256, 0, st>>>(pool_a, pool_b, d_desc, p0, p1, tm, tq, batch, map);
    }
  };
  const bool timing = launch_timing() != nullptr;
  // algorithmic work at block row k: the update of the k-th block row of B
  // by the panel's solved rows and the triangular solve with the diagonal
  // block
  auto work = [&](int k, int p0, int p1, double &fu, double &bu, double &fd, double &bd) {
    fu = bu = fd = bd = 0;
    if (!timing) return;
    for (int e = 0; e < batch; ++e) {
      const double nb = blk(h_desc[e].n, k), r = h_desc[e].nrhs;
      if (nb == 0) continue;
      const double other = transpose
                               ? std::min((double)p1, (double)h_desc[e].n) - (double)k * NB - nb
                               : (double)k * NB - p0;
      fu += 2.0 * nb * r * other;
      bu += sizeof(T) * (nb * other + other * r + 2.0 * nb * r);
      fd += nb * nb * r;
      bd += sizeof(T) * (0.5 * nb * nb + 2.0 * nb * r);
    }
  };
  double fu, bu, fd, bd;
  if (!transpose) {
    for (int k0 = 0; k0 < nblk; k0 += PB) {
      const int k1 = std::min(nblk, k0 + PB), p0 = k0 * NB, p1 = k1 * NB;
      for (int k = k0; k < k1; ++k) {
        work(k, p0, p1, fu, bu, fd, bd);
        if (!narrow) {
          LaunchScope ls(st, "trsm_step_kernel<fwd>", bu + bd, fu + fd);
          step(false, k, p0, p1);
          continue;
        }
        if (k > k0) {
          LaunchScope ls(st, "trsm_update_kernel<fwd>", bu, fu);
          update(false, k, p0, p1);
        }
        LaunchScope ls(st, "trsm_diag_kernel<fwd>", bd, fd);
        diag(false, k);
      }
      panel_gemm(false, p0, p1);
    }
  } else {
    // entries of different sizes: block k of an entry is its k-th from the
    // top; walking the panels and their blocks downwards from the largest
    // still visits every entry's blocks bottom-up
    for (int k0 = ((nblk - 1) / PB) * PB; k0 >= 0; k0 -= PB) {
      const int k1 = std::min(nblk, k0 + PB), p0 = k0 * NB, p1 = k1 * NB;
      for (int k = k1 - 1; k >= k0; --k) {
        work(k, p0, p1, fu, bu, fd, bd);
        if (!narrow) {
          LaunchScope ls(st, "trsm_step_kernel<bwd>", bu + bd, fu + fd);
          step(true, k, p0, p1);
          continue;
        }
        if (k < k1 - 1) {
          LaunchScope ls(st, "trsm_update_kernel<bwd>", bu, fu);
          update(true, k, p0, p1);
        }
        LaunchScope ls(st, "trsm_diag_kernel<bwd>", bd, fd);
        diag(true, k);
      }
      panel_gemm(true, p0, p1);
    }
  }
  return hipGetLastError();
}

template <class T>
hipError_t symmetrize_lower(hipStream_t st, T *pool, const MatDesc *d_desc, int batch, int maxn,
                            const MatDesc *h_desc) {
  if (batch <= 0 || maxn <= 0) return hipSuccess;
  if (batch > kMaxMapEntries && h_desc) {  // sub-batches, as in gemm
    for (int e0 = 0; e0 < batch; e0 += kMaxMapEntries)
      HIP_RETURN_IF(symmetrize_lower(st, pool, d_desc + e0, std::min(kMaxMapEntries, batch - e0), maxn,
                                     h_desc + e0));
    return hipSuccess;
  }
  const int nt = (maxn + 31) / 32;
  const TileMap map = h_desc ? tile_map(batch, [&](int e) {
    const int t = (h_desc[e].n + 31) / 32;
    return t * (t + 1) / 2;
  }) : TileMap{0, {}};
  if (map.n > 0) {
    if (map.off[map.n] > 0)
      symmetrize_kernel<T><<<grid_round(map.off[map.n]), 256, 0, st>>>(pool, d_desc, nt, map);
  } else {
    symmetrize_kernel<T><<<dim3((unsigned)(nt * nt), batch), 256, 0, st>>>(pool, d_desc, nt, map);
  }
  return hipGetLastError();
}

template <class T>
hipError_t diag_inverse(hipStream_t st, const T *pool, const MatDesc *d_desc, int batch, int maxn,
                        T *inv, const int64_t *inv_off) {
  if (batch <= 0 || maxn <= 0) return hipSuccess;
  LaunchScope ls(st, "diag_inv_kernel", 0, 0);
  diag_inv_kernel<T><<<dim3((maxn + NB - 1) / NB, batch), 64, 0, st>>>(pool, d_desc, inv, inv_off);
  return hipGetLastError();
}

template <class T, bool UPPER, int M>
static void launch_trsv(hipStream_t st, const T *apool, T *xpool, const MatDesc *d_desc,
                        const TrsvPlan &plan, const T *dinv, const int64_t *dinv_off,
                        const int *order, int *work, int *err, int m, int64_t ldx) {
  trsv_kernel<T, UPPER, M><<<plan.total_blocks, 256, 0, st>>>(apool, xpool, d_desc, dinv, dinv_off,
                                                              order, plan.d_flag_off,
                                                              plan.total_blocks, work, err, m, ldx);
}

template <class T, bool UPPER>
static hipError_t launch_trsv_cols(hipStream_t st, const T *apool, T *xpool,
                                   const MatDesc *d_desc, const TrsvPlan &plan, const T *dinv,
                                   const int64_t *dinv_off, const int *order, int *work, int *err,
                                   int m, int64_t ldx) {
  if (m == 1)
    launch_trsv<T, UPPER, 1>(st, apool, xpool, d_desc, plan, dinv, dinv_off, order, work, err, m, ldx);
  else if (m == 2)
    launch_trsv<T, UPPER, 2>(st, apool, xpool, d_desc, plan, dinv, dinv_off, order, work, err, m, ldx);
  else if (m <= 4)
    launch_trsv<T, UPPER, 4>(st, apool, xpool, d_desc, plan, dinv, dinv_off, order, work, err, m, ldx);
  else if (m <= kTrsvMaxCols)
    launch_trsv<T, UPPER, 8>(st, apool, xpool, d_desc, plan, dinv, dinv_off, order, work, err, m, ldx);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T>
hipError_t trsv_blocked(hipStream_t st, const T *apool, T *xpool, const MatDesc *d_desc,
                        const TrsvPlan &plan, bool upper, const T *dinv, const int64_t *dinv_off,
                        int *work, int *err, int m, int64_t ldx) {
  if (plan.total_blocks == 0 || m == 0) return hipSuccess;
  if (m < 0 || m > kTrsvMaxCols) return hipErrorInvalidValue;
  const int nz = 1 + plan.total_blocks;
  zero_ints_kernel<<<(nz + 255) / 256, 256, 0, st>>>(work, nz);
  const int *order = upper ? plan.d_order_bwd : plan.d_order_fwd;
  // one pass over the stored triangle, the right-hand sides read and written
  LaunchScope ls(st, upper ? "trsv_kernel<upper>" : "trsv_kernel<lower>",
                 sizeof(T) * (plan.tri_elems + 2.0 * plan.rows * m), 2.0 * plan.tri_elems * m);
  if (!upper)
    return launch_trsv_cols<T, false>(st, apool, xpool, d_desc, plan, dinv, dinv_off, order, work,
                                      err, m, ldx);
  return launch_trsv_cols<T, true>(st, apool, xpool, d_desc, plan, dinv, dinv_off, order, work, err,
                                   m, ldx);
}

template <class T>
hipError_t transpose_batched(hipStream_t st, const T *apool, T *bpool, const MatDesc *d_desc,
                             int batch, int maxn, const MatDesc *h_desc) {
  if (batch <= 0 || maxn <= 0) return hipSuccess;
  if (batch > kMaxMapEntries && h_desc) {  // sub-batches, as in gemm
    for (int e0 = 0; e0 < batch; e0 += kMaxMapEntries)
      HIP_RETURN_IF(transpose_batched(st, apool, bpool, d_desc + e0, std::min(kMaxMapEntries, batch - e0),
                                      maxn, h_desc + e0));
    return hipSuccess;
  }
  const TileMap map = h_desc ? tile_map(batch, [&](int e) {
    const int t = (h_desc[e].n + 31) / 32;
    return t * t;
  }) : TileMap{0, {}};
  if (map.n > 0) {
    if (map.off[map.n] > 0)
      transpose_kernel<T><<<grid_round(map.off[map.n]), 256, 0, st>>>(apool, bpool, d_desc, map);
  } else {
    const unsigned t = (unsigned)((maxn + 31) / 32);
    transpose_kernel<T><<<dim3(t, t, batch), 256, 0, st>>>(apool, bpool, d_desc, map);
  }
  return hipGetLastError();
}

void make_trsv_orders(const std::vector<int> &n, std::vector<int> &fwd, std::vector<int> &bwd,
                      std::vector<int> &flag_off, int &total) {
  const int batch = (int)n.size();
  std::vector<int> nblk(batch);
  int maxb = 0;
  total = 0;
  flag_off.resize(batch);
  for (int e = 0; e < batch; ++e) {
    nblk[e] = (n[e] + NB - 1) / NB;
    flag_off[e] = total;
    total += nblk[e];
    maxb = std::max(maxb, nblk[e]);
  }
  fwd.clear();
  bwd.clear();
  for (int lvl = 0; lvl < maxb; ++lvl)
    for (int e = 0; e < batch; ++e)
      if (lvl < nblk[e]) {
        fwd.push_back(e), fwd.push_back(lvl);
        bwd.push_back(e), bwd.push_back(nblk[e] - 1 - lvl);
      }
}

template struct DenseOps<double>;
template struct DenseOps<float>;
template hipError_t symmetrize_lower<double>(hipStream_t, double *, const MatDesc *, int, int,
                                            const MatDesc *);
template hipError_t symmetrize_lower<float>(hipStream_t, float *, const MatDesc *, int, int,
                                           const MatDesc *);
template hipError_t trsv_blocked<double>(hipStream_t, const double *, double *, const MatDesc *,
                                         const TrsvPlan &, bool, const double *, const int64_t *,
                                         int *, int *, int, int64_t);
template hipError_t trsv_blocked<float>(hipStream_t, const float *, float *, const MatDesc *,
                                        const TrsvPlan &, bool, const float *, const int64_t *,
                                        int *, int *, int, int64_t);
template hipError_t diag_inverse<double>(hipStream_t, const double *, const MatDesc *, int, int,
                                         double *, const int64_t *);
template hipError_t diag_inverse<float>(hipStream_t, const float *, const MatDesc *, int, int,
                                        float *, const int64_t *);
template hipError_t transpose_batched<double>(hipStream_t, const double *, double *, const MatDesc *,
                                              int, int, const MatDesc *);
template hipError_t transpose_batched<float>(hipStream_t, const float *, float *, const MatDesc *,
                                             int, int, const MatDesc *);

}  // namespace bddc
