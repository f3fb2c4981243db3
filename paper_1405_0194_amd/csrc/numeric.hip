// Numeric phases on gfx950 (MI355X): assembly of the shifted matrices, the
// supernodal LDL^T factorization, selected inversion, pole sums and inertia.
//
// Paper, Sec. II.A-II.B: for A = H - z S (complex symmetric) compute
// A = L D L^T (L unit lower, D diagonal) and then the entries of A^{-1} on
// the pattern of L; the factorization traverses the elimination tree from the
// leaves to the root and selected inversion from the root to the leaves, both
// as dense matrix products on supernodes.  Sec. II.C: for real shifts the
// number of negative d_k is the inertia count.
//
// Execution model: every launch covers all shifts of a batch (grid.y) and all
// tiles of one panel (a <= 64-column slice of a supernode).  The factorization
// issues supernodes leaves first (by height in the supernodal tree, columns in
// order within one), panels left to right; SelInv runs root to leaves.  Within
// a launch, workgroups own disjoint outputs, so there are no atomics on matrix
// data, and every entry receives its updates in one fixed order, so results
// do not depend on scheduling or on the number of subtree streams.
//
// Per panel p of supernode J (row list E_J, own columns first), with
// B = rows of E_J below the panel's diagonal block:
//   factor:  k_diag   dense LDL^T of the wp x wp diagonal block in LDS; stores
//                     D on the diagonal and L_pp^{-1} below it
//            k_trsm   L_Bp = A_Bp L_pp^{-T} D_p^{-1}
//            k_update A_BB -= L_Bp D_p L_Bp^T, scattered through the maps into
//                     the later columns of J and into ancestor supernodes
//   selinv:  k_lhat   W = L_Bp L_pp^{-1}                       (workspace)
//            k_selinv_off   Z_Bp = -Z_BB W   (Z_BB gathered, symmetric)
//            k_selinv_diag_* Z_pp = L_pp^{-T} D_p^{-1} L_pp^{-1} - W^T Z_Bp
// The products run on FP64 MFMA (v_mfma_f64_16x16x4f64): a complex product
// is four real MFMAs on split real/imaginary LDS tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cstdint>
#include <cstdio>
#include <new>
#include <vector>

#include "pxs_internal.h"
#include "numeric.h"

namespace pxs {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;   // threads per workgroup (4 wave64)
constexpr int TM = 64;    // tile rows (m) and columns (n)
constexpr int KC = 16;    // k-chunk staged in LDS
constexpr int LDP = 65;   // padded LDS row (doubles)

struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cinv(cplx a) {
  double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}

template <bool CPLX>
__device__ __forceinline__ cplx ld_elem(const double* base, int64_t e) {
  if (CPLX) {
    const double2 v = *reinterpret_cast<const double2*>(base + 2 * e);
    return {v.x, v.y};
  }
  return {base[e], 0.0};
}
template <bool CPLX>
__device__ __forceinline__ void st_elem(double* base, int64_t e, cplx v) {
  if (CPLX) {
    *reinterpret_cast<double2*>(base + 2 * e) = make_double2(v.re, v.im);
  } else {
    base[e] = v.re;
  }
}

// An operand element, or zero where ok is false: lanes outside the operand
// read a zero block instead of skipping the load, so every lane issues its
// load without a branch.  The compiler can then count the loads in flight
// exactly and the K loop's two-deep prefetch waits only for the older chunk.
__device__ __align__(16) double kZeroElem[2] = {0.0, 0.0};   // never written

template <bool CPLX>
__device__ __forceinline__ cplx ld_or_zero(const double* base, int64_t e, bool ok) {
  const double* q = ok ? base + (CPLX ? 2 : 1) * e : kZeroElem;
  if (CPLX) {
    const double2 v = *reinterpret_cast<const double2*>(q);
    return {v.x, v.y};
  }
  return {*q, 0.0};
}

// --------------------------------------------------------------------------
// MFMA tile engine: a 256-thread workgroup accumulates a 64 x NTILE tile
// P[m][n] = sum_k A[m][k] B[k][n] (NTILE = 64 or 128).  The 4 waves are laid
// out WM x WN over the tile, each owning BM x BN blocks of 16 x 16.
// Operands are staged in LDS as As[k][m], Bs[k][n] (real and imaginary
// parts split, rows padded by one double).
// v_mfma_f64_16x16x4f64 lane layout (lane l, 0..63):
//   A operand: A[l % 16][l / 16];  B operand: B[l / 16][l % 16];
//   result register r: D[l / 16 + 4 r][l % 16].
// A complex block product is four real MFMAs: re += ar br - ai bi,
// im += ar bi + ai br.  The last argument of the f64 MFMA builtin holds the
// operand negation bits (bit 0 negates A), so -ai costs no instruction.
// --------------------------------------------------------------------------
template <int NTILE>
struct Geo {
  static constexpr int WN = NTILE / 32;        // waves along n
  static constexpr int WM = 4 / WN;            // waves along m
  static constexpr int BM = 64 / WM / 16;      // 16-blocks per wave along m
  static constexpr int BN = 2;                 // 16-blocks per wave along n
  static constexpr int XA = 64 * KC / NT;      // A transfers per thread and chunk
  static constexpr int XB = NTILE * KC / NT;   // B transfers per thread and chunk
};

template <bool CPLX, int NTILE>
struct Acc {
  static constexpr int BM = Geo<NTILE>::BM, BN = Geo<NTILE>::BN;
  dbl4 re[BM][BN];
  dbl4 im[CPLX ? BM : 1][CPLX ? BN : 1];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < BM; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b) {
        re[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
        if (CPLX) im[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
  }
};

template <bool CPLX, int NTILE>
struct Stage {
  double a_re[KC][LDP];
  double a_im[CPLX ? KC : 1][LDP];
  double b_re[KC][NTILE + 1];
  double b_im[CPLX ? KC : 1][NTILE + 1];
  double d_re[KC];                 // per-k scale of the A operand (optional)
  double d_im[CPLX ? KC : 1];
};

// No per-k scaling of the A operand.
struct NoScale {};

// SCALE: A[m][k] is multiplied by the chunk's d_k (staged with the chunk)
// as it is read for the matrix cores.
// Row of the 16-row block a (column of the 16-column block b) of wave w:
// blocks in order, or, with bit 0 (bit 1) of SWZ on a 64 x 64 tile, the
// first wave row (column) taking blocks {0, 3} and the second {1, 2}, so that
// both skip equally many blocks of a triangle (products with a triangular
// operand or a symmetric result).
template <int NTILE, int SWZ>
__device__ __forceinline__ int block_row(int w, int a) {
  using G = Geo<NTILE>;
  if constexpr ((SWZ & 1) != 0) {
    static_assert(G::BM == 2 && G::WM == 2, "block swizzle needs 2 x 2 waves of 2 blocks");
    const int wr = w / G::WN;
    return 16 * (a == 0 ? wr : 3 - wr);
  } else {
    return (w / G::WN) * (G::BM * 16) + a * 16;
  }
}
template <int NTILE, int SWZ>
__device__ __forceinline__ int block_col(int w, int b) {
  using G = Geo<NTILE>;
  if constexpr ((SWZ & 2) != 0) {
    static_assert(G::BN == 2 && G::WN == 2, "block swizzle needs 2 x 2 waves of 2 blocks");
    const int wc = w % G::WN;
    return 16 * (b == 0 ? wc : 3 - wc);
  } else {
    return (w % G::WN) * 32 + b * 16;
  }
}

// MASK >= 0: only the block pairs (a, b) with bit 2a + b set are multiplied
// (the others are zero in this chunk, or not needed).
template <bool CPLX, int NTILE, bool SCALE = false, int MASK = -1, int SWZ = 0>
__device__ __forceinline__ void mfma_chunk(Acc<CPLX, NTILE>& acc, const Stage<CPLX, NTILE>& s) {
  using G = Geo<NTILE>;
  // the compiler's single-wave small-GEMM schedule (interleaves the LDS
  // operand reads with the MFMAs): 1-2% over the default schedule
  __builtin_amdgcn_iglp_opt(1);
  static_assert(MASK < 0 || (G::BM == 2 && G::BN == 2), "block masks need 2 x 2 blocks per wave");
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // a row block is read if any of its pairs is live, a column block likewise
  auto row_live = [](int t) { return MASK < 0 || ((MASK >> (2 * t)) & 3) != 0; };
  auto col_live = [](int t) { return MASK < 0 || ((MASK >> t) & 5) != 0; };
  auto live = [](int a, int b) { return MASK < 0 || ((MASK >> (2 * a + b)) & 1) != 0; };
#pragma unroll
  for (int ks = 0; ks < KC / 4; ++ks) {
    const int k = ks * 4 + lk;
    double ar[G::BM], ai[G::BM], br[G::BN], bi[G::BN];
#pragma unroll
    for (int t = 0; t < G::BM; ++t) {
      if (!row_live(t)) continue;
      ar[t] = s.a_re[k][block_row<NTILE, SWZ>(w, t) + li];
      if (CPLX) ai[t] = s.a_im[k][block_row<NTILE, SWZ>(w, t) + li];
    }
    if (SCALE) {
      const double dr = s.d_re[k];
      if (CPLX) {
        const double di = s.d_im[k];
#pragma unroll
        for (int t = 0; t < G::BM; ++t) {
          if (!row_live(t)) continue;
          const cplx v = cmul(cplx{dr, di}, cplx{ar[t], ai[t]});
          ar[t] = v.re;
          ai[t] = v.im;
        }
      } else {
#pragma unroll
        for (int t = 0; t < G::BM; ++t)
          if (row_live(t)) ar[t] *= dr;
      }
    }
#pragma unroll
    for (int t = 0; t < G::BN; ++t) {
      if (!col_live(t)) continue;
      br[t] = s.b_re[k][block_col<NTILE, SWZ>(w, t) + li];
      if (CPLX) bi[t] = s.b_im[k][block_col<NTILE, SWZ>(w, t) + li];
    }
#pragma unroll
    for (int a = 0; a < G::BM; ++a)
#pragma unroll
      for (int b = 0; b < G::BN; ++b) {
        if (!live(a, b)) continue;
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], acc.re[a][b], 0, 0, 0);
        if (CPLX) {
          acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], acc.re[a][b], 0, 0, 1);   // -ai bi
          acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], acc.im[a][b], 0, 0, 0);
          acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], acc.im[a][b], 0, 0, 0);
        }
      }
  }
}

// Visits every accumulator element as (m, n, value).
template <bool CPLX, int NTILE, int SWZ = 0, class F>
__device__ __forceinline__ void acc_foreach(const Acc<CPLX, NTILE>& acc, F f) {
  using G = Geo<NTILE>;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < G::BM; ++a)
#pragma unroll
    for (int b = 0; b < G::BN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = block_row<NTILE, SWZ>(w, a) + (lane >> 4) + 4 * r;
        const int n = block_col<NTILE, SWZ>(w, b) + (lane & 15);
        cplx v{acc.re[a][b][r], CPLX ? acc.im[a][b][r] : 0.0};
        f(m, n, v);
      }
}

// The idx-th accumulator element of the calling thread (the order in which
// acc_foreach visits them) and its tile coordinates.
template <int NTILE>
constexpr int acc_elems() { return Geo<NTILE>::BM * Geo<NTILE>::BN * 4; }

template <bool CPLX, int NTILE>
__device__ __forceinline__ void acc_at(const Acc<CPLX, NTILE>& acc, int idx, int& m, int& n, cplx& v) {
  using G = Geo<NTILE>;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int wm = (w / G::WN) * (G::BM * 16), wn = (w % G::WN) * 32;
  const int r = idx & 3, b = (idx >> 2) % G::BN, a = (idx >> 2) / G::BN;
  m = wm + a * 16 + (lane >> 4) + 4 * r;
  n = wn + b * 16 + (lane & 15);
  v = cplx{acc.re[a][b][r], CPLX ? acc.im[a][b][r] : 0.0};
}

// target[e] -= P for every accumulator element, in three passes so that a
// thread's memory operations overlap instead of running one element at a
// time: all target positions (addr(m, n, e) may read index maps; false
// skips the element, whose e must still be an in-bounds position of
// target), then all old values, then all stores.  Every target
// belongs to one element of one workgroup, so reordering the stores changes
// no result.
template <bool CPLX, int NTILE, class AF>
__device__ __forceinline__ void acc_sub_into(const Acc<CPLX, NTILE>& acc, double* target, AF addr) {
  constexpr int NE = acc_elems<NTILE>();
  int64_t e[NE];
  bool ok[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    int m, n;
    cplx v;
    acc_at<CPLX, NTILE>(acc, i, m, n, v);
    ok[i] = addr(m, n, e[i]);
  }
  // addr returns an in-bounds position also for skipped elements, so the
  // old values load without branches
  cplx o[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) o[i] = ld_elem<CPLX>(target, e[i]);
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    int m, n;
    cplx v;
    acc_at<CPLX, NTILE>(acc, i, m, n, v);
    if (ok[i]) st_elem<CPLX>(target, e[i], cplx{o[i].re - v.re, o[i].im - v.im});
  }
}

// Staging of one k-chunk of an operand with ROWS rows (64 or NTILE).
// slot(j) gives the (row, k) pair thread t moves in its j-th transfer:
// FAST_K = false puts consecutive threads on consecutive rows (memory
// contiguous along the rows), FAST_K = true on consecutive k.  fetch() reads
// global memory into registers and commit() writes them to LDS, so the next
// chunk's loads are in flight while the current chunk runs on the matrix
// cores.
template <int ROWS, bool FAST_K>
__device__ __forceinline__ void slot(int j, int& ii, int& kk) {
  const int t = threadIdx.x;
  if (!FAST_K) {
    ii = t % ROWS;
    kk = t / ROWS + (NT / ROWS) * j;
  } else {
    kk = t % KC;
    ii = t / KC + (NT / KC) * j;
  }
}

template <int ROWS, int X, bool FAST_K, class Gt>
__device__ __forceinline__ void fetch(cplx (&v)[X], int k0, Gt get) {
#pragma unroll
  for (int j = 0; j < X; ++j) {
    int ii, kk;
    slot<ROWS, FAST_K>(j, ii, kk);
    v[j] = get(ii, k0 + kk);
  }
}

template <bool CPLX, int ROWS, int X, bool FAST_K>
__device__ __forceinline__ void commit(double* re, double* im, const cplx (&v)[X]) {
#pragma unroll
  for (int j = 0; j < X; ++j) {
    int ii, kk;
    slot<ROWS, FAST_K>(j, ii, kk);
    re[kk * (ROWS + 1) + ii] = v[j].re;
    if (CPLX) im[kk * (ROWS + 1) + ii] = v[j].im;
  }
}

// Runtime choice of the staging order for operands whose memory order
// changes from chunk to chunk (a symmetric operand read through one
// triangle).  The flag is uniform across the workgroup; the two slot maps
// are blended with selects, so fetch and commit stay branch-free and the
// pipeline below remains one basic block per chunk.
template <int ROWS>
__device__ __forceinline__ void slot_sel(int j, bool fast, int& ii, int& kk) {
  const int t = threadIdx.x;
  const int ir = t % ROWS, kr = t / ROWS + (NT / ROWS) * j;
  const int kf = t % KC, jf = t / KC + (NT / KC) * j;
  ii = fast ? jf : ir;
  kk = fast ? kf : kr;
}

template <int ROWS, int X, class Gt>
__device__ __forceinline__ void fetch_rt(cplx (&v)[X], int k0, Gt get, bool fast) {
#pragma unroll
  for (int j = 0; j < X; ++j) {
    int ii, kk;
    slot_sel<ROWS>(j, fast, ii, kk);
    v[j] = get(ii, k0 + kk);
  }
}
template <bool CPLX, int ROWS, int X>
__device__ __forceinline__ void commit_rt(double* re, double* im, const cplx (&v)[X], bool fast) {
#pragma unroll
  for (int j = 0; j < X; ++j) {
    int ii, kk;
    slot_sel<ROWS>(j, fast, ii, kk);
    re[kk * (ROWS + 1) + ii] = v[j].re;
    if (CPLX) im[kk * (ROWS + 1) + ii] = v[j].im;
  }
}

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8
// XCDs in linear-id order; this bijection gives each XCD a contiguous range
// of logical ids, so the tiles of one shift (which share the A operand) run
// on the same XCD and share its L2.  Returns the logical (x, y) of the
// caller in a grid of nx x ny.
constexpr int NXCD = 8;
__device__ __forceinline__ void xcd_remap(int& x, int& y) {
  const int nx = gridDim.x, ny = gridDim.y;
  const int total = nx * ny;
  const int b = blockIdx.x + nx * blockIdx.y;
  const int xcd = b % NXCD, idx = b / NXCD;
  const int q = total / NXCD, r = total % NXCD;
  const int logical = (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
  x = logical % nx;
  y = logical / nx;
}

// Double-buffered LDS (two stages) with a two-chunk-deep register
// prefetch: two register sets alternate, so a chunk's global loads have two
// chunks of matrix-core time to land, and one barrier per chunk orders both
// "commit before use" and "use before overwrite" (each stage is rewritten
// one chunk after its use).
//   prologue: R0 <- c0, R1 <- c1, commit R0 -> buf0, R0 <- c2
//   even c:   mfma(buf0); commit R1 (c+1) -> buf1; R1 <- c+3
//   odd  c:   mfma(buf1); commit R0 (c+1) -> buf0; R0 <- c+3
// Chunks past the end are fetched as the last chunk again (clamped index,
// same memory, never used) and committed to the idle stage, so the loop body
// has no data-dependent branches and the wait counts stay exact.
template <bool CPLX, int NTILE>
struct Stage2 {
  Stage<CPLX, NTILE> buf[2];
};

// K loop over [kb, ke): P += A[:, k] B[k, :].  ga(m, k) and gb(n, k) return
// the operands (zero outside the matrices); bfast(k0) picks the B staging
// order per chunk.  gd(k), unless NoScale, returns a factor d_k applied to
// column k of A on its way to the matrix cores (one load per k and chunk
// instead of one per element); it must accept any k of the last chunk.
// Which block pairs (a, b) of the wave take part in a chunk, as a mask of
// bits 2a + b (evaluated per chunk, uniform over the wave): all (AllLive);
// for a triangular A operand on a 64-row tile (TriLive, swizzled block rows),
// both pairs of each row block whose rows meet the chunk's k range in the
// nonzero triangle; for a symmetric 64 x 64 result of which one triangle is
// used (UpperLive), the pairs on or above the block diagonal.
struct AllLive {
  static constexpr bool kAll = true;
  static constexpr int kSwz = 0;
  __device__ int operator()(int) const { return 15; }
};
template <bool LOWER>   // LOWER: A[m][k] = 0 for k > m; else A[m][k] = 0 for k < m
struct TriLive {
  static constexpr bool kAll = false;
  static constexpr int kSwz = 1;
  __device__ int operator()(int k0) const {
    static_assert(KC == 16, "a chunk spans one 16-row block");
    const int wr = (threadIdx.x >> 6) / Geo<64>::WN;
    const int c = k0 / KC;
    const int mb0 = wr, mb1 = 3 - wr;
    const bool l0 = LOWER ? c <= mb0 : c >= mb0;
    const bool l1 = LOWER ? c <= mb1 : c >= mb1;
    return __builtin_amdgcn_readfirstlane((l0 ? 3 : 0) | (l1 ? 12 : 0));   // both column blocks of a live row block
  }
};
// A symmetric 64 x 64 result of which only the entries n >= m are needed:
// the block pairs with column block >= row block (rows and columns swizzled,
// so no wave has more than 3 of its 4 pairs).
struct UpperLive {
  static constexpr bool kAll = false;
  static constexpr int kSwz = 3;
  __device__ int operator()(int) const {
    const int w = threadIdx.x >> 6;
    const int wr = w / Geo<64>::WN, wc = w % Geo<64>::WN;
    int mask = 0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        if ((b == 0 ? wc : 3 - wc) >= (a == 0 ? wr : 3 - wr)) mask |= 1 << (2 * a + b);
    return __builtin_amdgcn_readfirstlane(mask);
  }
};

// The masks these functors return (15, 12, 3, 11, 10; 0 when no pair is
// live) each have an instance below; a functor returning another mask would
// skip its chunk, so a new one adds its masks here.
template <bool CPLX, int NTILE, bool SC, class LV>
__device__ __forceinline__ void run_chunk(Acc<CPLX, NTILE>& acc, const Stage<CPLX, NTILE>& st, LV lv, int k0) {
  if constexpr (LV::kAll) {
    mfma_chunk<CPLX, NTILE, SC>(acc, st);
  } else {
    const int m = lv(k0);
    if (m == 15) mfma_chunk<CPLX, NTILE, SC, 15, LV::kSwz>(acc, st);
    else if (m == 12) mfma_chunk<CPLX, NTILE, SC, 12, LV::kSwz>(acc, st);
    else if (m == 3) mfma_chunk<CPLX, NTILE, SC, 3, LV::kSwz>(acc, st);
    else if (m == 11) mfma_chunk<CPLX, NTILE, SC, 11, LV::kSwz>(acc, st);
    else if (m == 10) mfma_chunk<CPLX, NTILE, SC, 10, LV::kSwz>(acc, st);
  }
}

template <bool CPLX, int NTILE, bool AFAST, class GA, class GB, class BF, class GD = NoScale, class LV = AllLive>
__device__ __forceinline__ void gemm_pipe(Acc<CPLX, NTILE>& acc, Stage2<CPLX, NTILE>& s, int kb, int ke,
                                          GA ga, GB gb, BF bfast, GD gd = GD(), LV lv = LV()) {
  using G = Geo<NTILE>;
  constexpr bool SC = !std::is_same<GD, NoScale>::value;
  if (kb >= ke) return;
  const int nc = (ke - kb + KC - 1) / KC;
  auto kat = [&](int c) { return kb + min(c, nc - 1) * KC; };
  const int t = threadIdx.x;
  auto dfetch = [&](cplx& r, int k0) {
    // every thread loads (the lanes of a wave share KC addresses), so the
    // load is not under a branch; threads t < KC commit it
    if constexpr (SC) r = gd(k0 + (t & (KC - 1)));
  };
  auto dcommit = [&](Stage<CPLX, NTILE>& st, const cplx& r) {
    if constexpr (SC) {
      if (t < KC) {
        st.d_re[t] = r.re;
        if (CPLX) st.d_im[t] = r.im;
      }
    }
  };
  cplx ra0[G::XA], rb0[G::XB], ra1[G::XA], rb1[G::XB];
  cplx rd0{1.0, 0.0}, rd1{1.0, 0.0};
  bool fb0 = bfast(kat(0)), fb1 = bfast(kat(1));
  fetch<64, G::XA, AFAST>(ra0, kat(0), ga);
  fetch_rt<NTILE, G::XB>(rb0, kat(0), gb, fb0);
  dfetch(rd0, kat(0));
  fetch<64, G::XA, AFAST>(ra1, kat(1), ga);
  fetch_rt<NTILE, G::XB>(rb1, kat(1), gb, fb1);
  dfetch(rd1, kat(1));
  commit<CPLX, 64, G::XA, AFAST>(&s.buf[0].a_re[0][0], &s.buf[0].a_im[0][0], ra0);
  commit_rt<CPLX, NTILE, G::XB>(&s.buf[0].b_re[0][0], &s.buf[0].b_im[0][0], rb0, fb0);
  dcommit(s.buf[0], rd0);
  fb0 = bfast(kat(2));
  fetch<64, G::XA, AFAST>(ra0, kat(2), ga);
  fetch_rt<NTILE, G::XB>(rb0, kat(2), gb, fb0);
  dfetch(rd0, kat(2));
  __syncthreads();
  for (int c = 0; c < nc; c += 2) {
    run_chunk<CPLX, NTILE, SC>(acc, s.buf[0], lv, kb + c * KC);
    commit<CPLX, 64, G::XA, AFAST>(&s.buf[1].a_re[0][0], &s.buf[1].a_im[0][0], ra1);
    commit_rt<CPLX, NTILE, G::XB>(&s.buf[1].b_re[0][0], &s.buf[1].b_im[0][0], rb1, fb1);
    dcommit(s.buf[1], rd1);
    fb1 = bfast(kat(c + 3));
    fetch<64, G::XA, AFAST>(ra1, kat(c + 3), ga);
    fetch_rt<NTILE, G::XB>(rb1, kat(c + 3), gb, fb1);
    dfetch(rd1, kat(c + 3));
    __syncthreads();
    if (c + 1 >= nc) break;
    run_chunk<CPLX, NTILE, SC>(acc, s.buf[1], lv, kb + (c + 1) * KC);
    commit<CPLX, 64, G::XA, AFAST>(&s.buf[0].a_re[0][0], &s.buf[0].a_im[0][0], ra0);
    commit_rt<CPLX, NTILE, G::XB>(&s.buf[0].b_re[0][0], &s.buf[0].b_im[0][0], rb0, fb0);
    dcommit(s.buf[0], rd0);
    fb0 = bfast(kat(c + 4));
    fetch<64, G::XA, AFAST>(ra0, kat(c + 4), ga);
    fetch_rt<NTILE, G::XB>(rb0, kat(c + 4), gb, fb0);
    dfetch(rd0, kat(c + 4));
    __syncthreads();
  }
}

struct RowsFast {
  __device__ bool operator()(int) const { return false; }
};
struct KFast {
  __device__ bool operator()(int) const { return true; }
};

// --------------------------------------------------------------------------
// small kernels
// --------------------------------------------------------------------------
__global__ void k_fill_zero(double2* p, int64_t n2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n2; i += stride) p[i] = make_double2(0.0, 0.0);
}

// Real shifts eps_q as the complex shifts (eps_q, 0) of an inertia batch.
__global__ void k_real_shifts(const double* __restrict__ eps, double* __restrict__ shifts, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) {
    shifts[2 * q] = eps[q];
    shifts[2 * q + 1] = 0.0;
  }
}

__global__ void k_zero_i64(int64_t* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// max |H| and max |S| (two-stage, deterministic)
__global__ void k_absmax_partial(const double* __restrict__ H, const double* __restrict__ S,
                                 int64_t nnz, double* partial) {
  __shared__ double sh[2][NT];
  double mh = 0.0, ms = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * NT) {
    mh = fmax(mh, fabs(H[i]));
    ms = fmax(ms, fabs(S[i]));
  }
  sh[0][threadIdx.x] = mh;
  sh[1][threadIdx.x] = ms;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + s]);
      sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sh[0][0];
    partial[2 * blockIdx.x + 1] = sh[1][0];
  }
}
__global__ void k_absmax_final(const double* partial, int nb, double* out) {
  if (threadIdx.x == 0) {
    double mh = 0.0, ms = 0.0;
    for (int b = 0; b < nb; ++b) {
      mh = fmax(mh, partial[2 * b]);
      ms = fmax(ms, partial[2 * b + 1]);
    }
    out[0] = mh;
    out[1] = ms;
  }
}

// A_l = H - w_l S on the input pattern (the rest of the storage is zero).
template <bool CPLX>
__global__ void k_assemble(double* __restrict__ L, int64_t stride, const double* __restrict__ H,
                           const double* __restrict__ S, const int64_t* __restrict__ eoff,
                           int64_t nnz, const double* __restrict__ shifts) {
  const int sh = blockIdx.y;
  const double wr = shifts[2 * sh], wi = shifts[2 * sh + 1];
  double* Ls = L + (CPLX ? 2 : 1) * stride * sh;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * NT) {
    const double h = H[k], s = S[k];
    st_elem<CPLX>(Ls, eoff[k], cplx{h - wr * s, -wi * s});
  }
}

// --------------------------------------------------------------------------
// factor kernels
// --------------------------------------------------------------------------
struct PanelK {
  int64_t off;     // storage offset of the supernode
  int64_t cm;      // index of the supernode's row list in colmap/colseg
  int32_t ld;      // leading dimension of the supernode
  int32_t p0;      // panel's first column (position in the row list)
  int32_t wp;      // panel width
  int32_t nb;      // rows below the panel's diagonal block
  int32_t col0;    // new index of the panel's first column
  int32_t split;   // split-K pieces (SelInv diagonal update)
  int32_t w;       // width of the supernode
  int32_t c;       // rows below the supernode (ld - w)
  int32_t sh0;     // first shift of this launch (grid.y counts from it)
};

struct Common {
  double* L;               // factor storage of shift 0
  int64_t stride;          // elements per shift
  const int64_t* colmap;
  const int64_t* colseg;
  const int32_t* relpos;
  double* work;            // workspace base
  int64_t wps;             // workspace bytes per shift
  int64_t wfix;            // fixed workspace bytes
  const double* shifts;    // device, 2 doubles per shift
  const double* absmax;    // device, max|H|, max|S|
  int64_t* info;           // device, per shift
  int64_t* negc;           // device, per shift
  double pivtol;
  double* G;               // dense Z_CC of the current supernode, per shift of a chunk
  int64_t gstride;         // doubles per shift in G
  int64_t ut;              // Hermitian factorizations: elements from a shift's L region to its U^T region
};

template <bool CPLX>
__device__ __forceinline__ double* shift_base(const Common& c, int sh) {
  return c.L + (CPLX ? 2 : 1) * c.stride * sh;
}

// Where a workgroup finds its panel.  OnePanel: one panel of one system per
// launch (kernel argument), grid = (tiles, shifts).  PanelGroup: a table of
// panels of several systems launched as one grid of sum(tiles x shifts)
// workgroups (the fused execution of a batch of systems); each item's
// workgroups are a contiguous range of logical ids, so after the XCD-aware
// remap the tiles of one item share an XCD as in a single launch.
struct OnePanel {
  Common c;
  PanelK p;
};

struct GroupItem {
  Common c;
  PanelK p;
  int64_t start;   // first logical workgroup of the item
  int32_t tiles;   // workgroups per shift
  int32_t nsh;     // shifts
};

struct PanelGroup {
  const GroupItem* items;
  int32_t n;
};

// LaneGroup: the same as PanelGroup for at most MAX_LANES panels whose items
// travel in the kernel arguments (no device table, so a stream capture
// records them like any other launch): the fused selected inversion of the
// subtree lanes of one system.
constexpr int MAX_LANES = 8;
struct LaneGroup {
  GroupItem it[MAX_LANES];
  int32_t n;
};

// remap: XCD-aware order (else the plain one); bx = tile, by = shift
__device__ __forceinline__ void locate(const OnePanel& src, Common& c, PanelK& p, int& bx, int& by, bool remap) {
  c = src.c;
  p = src.p;
  if (remap) {
    xcd_remap(bx, by);
  } else {
    bx = blockIdx.x;
    by = blockIdx.y;
  }
}

__device__ __forceinline__ void locate(const PanelGroup& src, Common& c, PanelK& p, int& bx, int& by, bool remap) {
  int lx = (int)blockIdx.x, ly = 0;
  if (remap) xcd_remap(lx, ly);   // grid (total, 1): ly stays 0
  const int64_t lid = lx;
  int lo = 0, hi = src.n - 1;     // the last item starting at or before lid
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (src.items[mid].start <= lid) lo = mid;
    else hi = mid - 1;
  }
  const GroupItem& it = src.items[lo];
  c = it.c;
  p = it.p;
  const int64_t local = lid - it.start;
  bx = (int)(local % it.tiles);
  by = (int)(local / it.tiles);
}

__device__ __forceinline__ void locate(const LaneGroup& src, Common& c, PanelK& p, int& bx, int& by, bool remap) {
  int lx = (int)blockIdx.x, ly = 0;
  if (remap) xcd_remap(lx, ly);   // grid (total, 1)
  int i = 0;                      // the last item starting at or before lx
  for (int q = 1; q < src.n; ++q)
    if (src.it[q].start <= lx) i = q;
  const GroupItem& it = src.it[i];
  c = it.c;
  p = it.p;
  const int local = lx - (int)it.start;
  bx = local % it.tiles;
  by = local / it.tiles;
}

// Dense LDL^T of the panel's wp x wp diagonal block in LDS, with L_pp^{-1}
// accumulated along the way.  Step k (one barrier per step, 512 threads, row
// r = t % 64 and every eighth column per thread):
//   trailing update  A[r][j] -= d_k L[r][k] L[j][k]            k+1 < j < r
//   next column      L[r][k+1] = (A[r][k+1] - d_k L[r][k] L[k+1][k]) / d_{k+1}
//   pivots           D[j] -= d_k L[j][k]^2                     j > k (two buffers)
//   inverse          X[r][t] -= L[r][k] X[k][t]  (t < k),  X[r][k] = -L[r][k]
// X = L^{-1} is built from the elementary eliminations in the columns of A
// that step k no longer needs; d_{k+1} is recomputed by every thread that
// needs it from the previous step's values, so the next column's multipliers
// are formed in the same step (look-ahead) and no second barrier is needed.
constexpr int NTD = 512;

template <bool CPLX, class Src>
__global__ void __launch_bounds__(NTD) k_diag(Src src) {
  // a[col][row], row > col: the working matrix, then L^{-1}; L is kept in
  // the other strict triangle, a[row][col] = L[row][col] (one array, 68 KB
  // of LDS, so a workgroup fits on a CU beside one of the matrix kernels)
  __shared__ double a_re[64][LDP];
  __shared__ double a_im[CPLX ? 64 : 1][LDP];
  __shared__ double dd_re[2][64];    // running diagonal, double-buffered by step parity
  __shared__ double dd_im[2][CPLX ? 64 : 1];
  __shared__ double pv_re[64];       // pivots d_k
  __shared__ double pv_im[CPLX ? 64 : 1];
  Common c;
  PanelK p;
  int bx, sh;
  locate(src, c, p, bx, sh, false);
  double* Ls = shift_base<CPLX>(c, sh);
  const int wp = p.wp;
  const int t = threadIdx.x;
  const int64_t dbase = p.off + (int64_t)p.p0 * p.ld + p.p0;
  for (int idx = t; idx < wp * wp; idx += NTD) {
    const int cc = idx / wp, r = idx % wp;
    cplx v{0.0, 0.0};
    if (r >= cc) v = ld_elem<CPLX>(Ls, dbase + (int64_t)cc * p.ld + r);
    a_re[cc][r] = v.re;
    if (CPLX) a_im[cc][r] = v.im;
    if (r == cc) {
      dd_re[0][r] = v.re;
      if (CPLX) dd_im[0][r] = v.im;
    }
  }
  __syncthreads();
  auto inv = [](cplx d) -> cplx { return CPLX ? cinv(d) : cplx{1.0 / d.re, 0.0}; };
  // column 0 of L
  if (t > 0 && t < wp) {
    const cplx d0{dd_re[0][0], CPLX ? dd_im[0][0] : 0.0};
    const cplx v = cmul(cplx{a_re[0][t], CPLX ? a_im[0][t] : 0.0}, inv(d0));
    a_re[t][0] = v.re;
    if (CPLX) a_im[t][0] = v.im;
  }
  __syncthreads();
  const double wabs = sqrt(c.shifts[2 * sh] * c.shifts[2 * sh] + c.shifts[2 * sh + 1] * c.shifts[2 * sh + 1]);
  const double thr = c.pivtol * (c.absmax[0] + (CPLX ? wabs : fabs(c.shifts[2 * sh])) * c.absmax[1]);
  int bad = 0;
  int neg = 0;
  const int r = t & 63, cg = t >> 6;   // eight threads per row
  for (int k = 0; k < wp; ++k) {
    const int cur = k & 1, nxt = cur ^ 1;
    const cplx dk{dd_re[cur][k], CPLX ? dd_im[cur][k] : 0.0};
    if (t == 0) {
      const double ad = CPLX ? sqrt(dk.re * dk.re + dk.im * dk.im) : fabs(dk.re);
      if (!(ad >= thr) && bad == 0) bad = p.col0 + k + 1;
      if (!CPLX && dk.re < 0.0) ++neg;
      pv_re[k] = dk.re;
      if (CPLX) pv_im[k] = dk.im;
    }
    if (r > k && r < wp) {
      const cplx lrk{a_re[r][k], CPLX ? a_im[r][k] : 0.0};
      const cplx dl = cmul(dk, lrk);                 // d_k L[r][k]
      // trailing columns j in (k+1, r): off-diagonal entries of A
      for (int j = k + 2 + cg; j < r; j += NTD / 64) {
        const cplx f = cmul(dl, cplx{a_re[j][k], CPLX ? a_im[j][k] : 0.0});
        a_re[j][r] -= f.re;
        if (CPLX) a_im[j][r] -= f.im;
      }
      if (cg == 0) {
        // running diagonal of row r
        const cplx f = cmul(dl, lrk);
        dd_re[nxt][r] = dd_re[cur][r] - f.re;
        if (CPLX) dd_im[nxt][r] = dd_im[cur][r] - f.im;
      }
      if (cg == 1 && r > k + 1) {
        // look-ahead: L[r][k+1] with d_{k+1} formed from the previous values
        const cplx lk1{a_re[k + 1][k], CPLX ? a_im[k + 1][k] : 0.0};
        const cplx dk1n = cmul(cmul(dk, lk1), lk1);
        const cplx dk1{dd_re[cur][k + 1] - dk1n.re, CPLX ? dd_im[cur][k + 1] - dk1n.im : 0.0};
        const cplx f = cmul(dl, lk1);
        const cplx arn{a_re[k + 1][r] - f.re, CPLX ? a_im[k + 1][r] - f.im : 0.0};
        const cplx v = cmul(arn, inv(dk1));
        a_re[r][k + 1] = v.re;
        if (CPLX) a_im[r][k + 1] = v.im;
      }
      // inverse: columns t < k of X get the elimination of column k
      for (int tc = cg; tc < k; tc += NTD / 64) {
        const cplx f = cmul(lrk, cplx{a_re[tc][k], CPLX ? a_im[tc][k] : 0.0});
        a_re[tc][r] -= f.re;
        if (CPLX) a_im[tc][r] -= f.im;
      }
      if (cg == 2) {
        a_re[k][r] = -lrk.re;
        if (CPLX) a_im[k][r] = -lrk.im;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    // the smallest flagged column wins (0 = none yet), whatever the order in
    // which independent subtrees run
    if (bad) {
      unsigned long long* q = (unsigned long long*)&c.info[sh];
      unsigned long long old = atomicCAS(q, 0ull, (unsigned long long)bad);
      while (old != 0ull && old > (unsigned long long)bad) {
        const unsigned long long seen = atomicCAS(q, old, (unsigned long long)bad);
        if (seen == old) break;
        old = seen;
      }
    }
    if (!CPLX && neg) atomicAdd((unsigned long long*)&c.negc[sh], (unsigned long long)neg);
  }
  for (int idx = t; idx < wp * wp; idx += NTD) {
    const int cc = idx / wp, rr = idx % wp;
    if (rr > cc) st_elem<CPLX>(Ls, dbase + (int64_t)cc * p.ld + rr, cplx{a_re[cc][rr], CPLX ? a_im[cc][rr] : 0.0});
    if (rr == cc) st_elem<CPLX>(Ls, dbase + (int64_t)cc * p.ld + rr, cplx{pv_re[cc], CPLX ? pv_im[cc] : 0.0});
  }
}

// L_Bp = A_Bp L_pp^{-T} D^{-1}: P[c][i] = sum_k Linv[c][k] A[i][k], then / d_c.
// Panel products run on tiles of 64 x TNv (TNv = 64 or 128 rows, a runtime
// option); with double-buffered LDS a 128-row tile uses 100 KB (one
// workgroup per CU), a 64-row tile 67 KB (two per CU).
#define PXS_LB(TNv) __launch_bounds__(NT, (TNv) == 64 ? 2 : 1)

template <bool CPLX, int TN, class Src>
__global__ void PXS_LB(TN) k_trsm(Src src) {
  __shared__ Stage2<CPLX, TN> s;
  __shared__ cplx dinv[64];
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, true);
  const int sh = by;
  double* Ls = shift_base<CPLX>(c, sh);
  const int i0 = bx * TN;
  const int64_t dbase = p.off + (int64_t)p.p0 * p.ld + p.p0;   // (p0, p0)
  const int64_t rbase = dbase + p.wp;                          // first row below
  if (threadIdx.x < p.wp) {
    const cplx d = ld_elem<CPLX>(Ls, dbase + (int64_t)threadIdx.x * p.ld + threadIdx.x);
    dinv[threadIdx.x] = CPLX ? cinv(d) : cplx{1.0 / d.re, 0.0};
  }
  Acc<CPLX, TN> acc;
  acc.zero();
  // L^{-1} is lower triangular: on 64-row tiles the all-zero blocks of a
  // chunk are not multiplied
  using LV = std::conditional_t<TN == 64, TriLive<true>, AllLive>;
  gemm_pipe<CPLX, TN, false>(
      acc, s, 0, p.wp,
      [&](int m, int kg) -> cplx {   // Linv[c][k]: column k of the diagonal block
        const cplx v = ld_or_zero<CPLX>(Ls, dbase + (int64_t)kg * p.ld + m, m < p.wp && kg < p.wp && m > kg);
        return (m == kg && m < p.wp) ? cplx{1.0, 0.0} : v;
      },
      [&](int n, int kg) -> cplx {   // A[i][k]
        const int ig = i0 + n;
        return ld_or_zero<CPLX>(Ls, rbase + (int64_t)kg * p.ld + ig, kg < p.wp && ig < p.nb);
      },
      RowsFast(), NoScale(), LV());
  acc_foreach<CPLX, TN, LV::kSwz>(acc, [&](int m, int n, cplx v) {
    const int ig = i0 + n;
    if (m < p.wp && ig < p.nb) st_elem<CPLX>(Ls, rbase + (int64_t)m * p.ld + ig, cmul(v, dinv[m]));
  });
}

// Left-looking update of panel p from the earlier columns of its own
// supernode: A[r][c] -= sum_{k < p0} L[r][k] d_k L[c][k] for rows r >= p0 of
// the row list and the panel's columns c.  P[c][r] = sum_k (d_k L[c][k]) L[r][k].
template <bool CPLX, int TN, class Src>
__global__ void PXS_LB(TN) k_int_update(Src src) {
  __shared__ Stage2<CPLX, TN> s;
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, true);
  const int sh = by;
  double* Ls = shift_base<CPLX>(c, sh);
  const int r0 = bx * TN;            // rows p0 + r0 .. of the row list
  const int nrows = p.ld - p.p0;
  const int64_t cbase = p.off + p.p0;        // element (row p0, column 0)
  Acc<CPLX, TN> acc;
  acc.zero();
  gemm_pipe<CPLX, TN, false>(
      acc, s, 0, p.p0,
      [&](int m, int kg) -> cplx {   // L[p0 + c][k] (times d_k on the way to the MFMAs)
        return ld_or_zero<CPLX>(Ls, cbase + (int64_t)kg * p.ld + m, m < p.wp && kg < p.p0);
      },
      [&](int n, int kg) -> cplx {   // L[p0 + r][k]
        const int rg = r0 + n;
        return ld_or_zero<CPLX>(Ls, cbase + (int64_t)kg * p.ld + rg, kg < p.p0 && rg < nrows);
      },
      RowsFast(),
      [&](int kg) -> cplx {          // d_k
        return ld_or_zero<CPLX>(Ls, p.off + (int64_t)kg * p.ld + kg, kg < p.p0);
      });
  acc_sub_into<CPLX, TN>(acc, Ls, [&](int m, int n, int64_t& e) {
    const int rg = r0 + n;
    // clamped into the panel (in bounds for skipped elements)
    e = cbase + (int64_t)(p.p0 + min(m, p.wp - 1)) * p.ld + min(rg, nrows - 1);
    return m < p.wp && rg < nrows && rg >= m;
  });
}

__device__ __forceinline__ void tri_index(int b, int& ti, int& tj) {
  // b enumerates the pairs (ti >= tj) row by row: b = ti (ti + 1) / 2 + tj
  int x = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((x + 1) * (x + 2) / 2 <= b) ++x;
  while (x * (x + 1) / 2 > b) --x;
  ti = x;
  tj = b - x * (x + 1) / 2;
}

// Update of the rows/columns below columns [p0, p0 + wp) of a supernode:
// A_BB -= L_B,K D_K L_B,K^T on lower tiles (ti >= tj), scattered through the
// maps (B = row-list positions from p0 + wp on).  Used once per supernode
// with K = all of its columns (p0 = 0, wp = w_J, B = the rows below it).
// P[j][i] = sum_k (d_k L[j][k]) L[i][k].
template <bool CPLX, int TN, class Src>
__global__ void PXS_LB(TN) k_update(Src src) {
  __shared__ Stage2<CPLX, TN> s;
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, true);
  const int sh = by;
  double* Ls = shift_base<CPLX>(c, sh);
  // tiles: 64 columns j (m) by 128 rows i (n); only tiles that reach the
  // lower triangle (some i >= some j) do work
  const int nti = (p.nb + TN - 1) / TN;
  const int tj = bx / nti, ti = bx % nti;
  const int i0 = ti * TN, j0 = tj * TM;
  if (i0 + TN - 1 < j0) return;
  const int base = p.p0 + p.wp;   // row-list position of the first row below
  const int64_t rbase = p.off + base;   // element (row base, column 0)
  const int kb = p.p0, ke = p.p0 + p.wp;
  Acc<CPLX, TN> acc;
  acc.zero();
  gemm_pipe<CPLX, TN, false>(
      acc, s, kb, ke,
      [&](int m, int kg) -> cplx {   // L[j][k] (times d_k on the way to the MFMAs)
        const int jg = j0 + m;
        return ld_or_zero<CPLX>(Ls, rbase + (int64_t)kg * p.ld + jg, kg < ke && jg < p.nb);
      },
      [&](int n, int kg) -> cplx {
        const int ig = i0 + n;
        return ld_or_zero<CPLX>(Ls, rbase + (int64_t)kg * p.ld + ig, kg < ke && ig < p.nb);
      },
      RowsFast(),
      [&](int kg) -> cplx {          // d_k
        return ld_or_zero<CPLX>(Ls, p.off + (int64_t)kg * p.ld + kg, kg < ke);
      });
  const int64_t* cmap = c.colmap + p.cm;
  const int64_t* cseg = c.colseg + p.cm;
  acc_sub_into<CPLX, TN>(acc, Ls, [&](int m, int n, int64_t& e) {
    const int jg = j0 + m, ig = i0 + n;
    // branch-free, so the map loads of all elements are in flight together:
    // indices clamped into the supernode's row list with row >= column
    // (where relpos is defined); a skipped element reads a valid position
    // and is not stored
    const int jc = min(jg, p.nb - 1), ic = min(max(ig, jc), p.nb - 1);
    e = cmap[base + jc] + c.relpos[cseg[base + jc] + base + ic];
    return jg < p.nb && ig < p.nb && ig >= jg;
  });
}

// --------------------------------------------------------------------------
// selected inversion kernels (complex only)
// --------------------------------------------------------------------------
__device__ __forceinline__ double* wbase(const Common& c, int sh) {
  return (double*)((char*)c.work + c.wfix + c.wps * sh);
}

// W = L_Bp Linv: P[c][i] = sum_k Linv[k][c] L[i][k]; W stored W[c * nb + i].
template <int TN, class Src>
__global__ void PXS_LB(TN) k_lhat(Src src) {
  __shared__ Stage2<true, TN> s;
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, true);
  const int sh = p.sh0 + by;
  double* Ls = shift_base<true>(c, sh);
  double* W = wbase(c, sh);
  const int i0 = bx * TN;
  const int64_t dbase = p.off + (int64_t)p.p0 * p.ld + p.p0;
  const int64_t rbase = dbase + p.wp;
  Acc<true, TN> acc;
  acc.zero();
  // A[m][k] = L^{-1}[k][m] vanishes for k < m (see k_trsm)
  using LV = std::conditional_t<TN == 64, TriLive<false>, AllLive>;
  gemm_pipe<true, TN, true>(
      acc, s, 0, p.wp,
      [&](int m, int kg) -> cplx {   // Linv[k][c]: column c of the diagonal block, rows k
        const cplx v = ld_or_zero<true>(Ls, dbase + (int64_t)m * p.ld + kg, m < p.wp && kg < p.wp && kg > m);
        return (kg == m && m < p.wp) ? cplx{1.0, 0.0} : v;
      },
      [&](int n, int kg) -> cplx {
        const int ig = i0 + n;
        return ld_or_zero<true>(Ls, rbase + (int64_t)kg * p.ld + ig, kg < p.wp && ig < p.nb);
      },
      RowsFast(), NoScale(), LV());
  acc_foreach<true, TN, LV::kSwz>(acc, [&](int m, int n, cplx v) {
    const int ig = i0 + n;
    if (m < p.wp && ig < p.nb) st_elem<true>(W, (int64_t)m * p.nb + ig, v);
  });
}

// Z_Bp = -Z_BB W: P[c][i] = sum_k W[k][c] Z(k, i).  Z_BB is symmetric; its
// part inside the supernode's own columns is read from the supernode's
// storage (column min(i, k), row max(i, k)), the part in the rows below it
// from the dense copy G of Z_CC made by k_gather_cc.
template <int TN, class Src>
__global__ void PXS_LB(TN) k_selinv_off(Src src) {
  __shared__ Stage2<true, TN> s;
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, true);
  const int sh = p.sh0 + by;
  double* Ls = shift_base<true>(c, sh);
  const double* W = wbase(c, sh);
  const double* G = c.G + c.gstride * by;
  const int i0 = bx * TN;
  const int base = p.p0 + p.wp;
  Acc<true, TN> acc;
  acc.zero();
  gemm_pipe<true, TN, true>(
      acc, s, 0, p.nb,
      [&](int m, int kg) -> cplx {
        return ld_or_zero<true>(W, (int64_t)m * p.nb + kg, m < p.wp && kg < p.nb);
      },
      [&](int n, int kg) -> cplx {
        const int ig = i0 + n;
        const int qk = base + kg, qi = base + ig;
        const int lo = min(qi, qk), hi = max(qi, qk);
        const bool in_g = lo >= p.w;
        const double* src = in_g ? G : Ls;
        const int64_t e = in_g ? (int64_t)(lo - p.w) * p.c + (hi - p.w) : p.off + (int64_t)lo * p.ld + hi;
        return ld_or_zero<true>(src, e, kg < p.nb && ig < p.nb);
      },
      // both sources are lower triangles stored by column: rows are
      // contiguous for each k when the whole chunk lies on or below the
      // diagonal of the tile; otherwise k is contiguous
      [&](int k0) -> bool { return !(i0 >= k0 + KC - 1); });
  const int64_t rbase = p.off + (int64_t)p.p0 * p.ld + base;
  acc_foreach<true, TN>(acc, [&](int m, int n, cplx v) {
    const int ig = i0 + n;
    if (m < p.wp && ig < p.nb) st_elem<true>(Ls, rbase + (int64_t)m * p.ld + ig, cplx{-v.re, -v.im});
  });
}

// G = Z_CC, lower triangle: G[a + b c] = Z(w + a, w + b) for b <= a < c,
// gathered from the ancestors' storage through the maps.  Each thread moves
// 16 elements of a 64 x 64 tile: first all relative row positions, then all
// values, then the stores, so the loads of a thread are in flight together.
template <class Src>
__global__ void __launch_bounds__(NT) k_gather_cc(Src src) {
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, false);
  const int sh = p.sh0 + by;
  const double* Ls = shift_base<true>(c, sh);
  double* G = c.G + c.gstride * by;
  int ta, tb;
  tri_index(bx, ta, tb);
  const int a0 = ta * TM, b0 = tb * TM;
  const int cc = p.c, w = p.w;
  const int64_t* cmap = c.colmap + p.cm;
  const int64_t* cseg = c.colseg + p.cm;
  const int t = threadIdx.x;
  const int a = a0 + (t & 63);
  int64_t e[16];
  bool ok[16];
  // branch-free, so all map and value loads of a thread are in flight
  // together: indices clamped into Z_CC with row >= column (where relpos is
  // defined); skipped elements read a valid position and are not stored
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int b = b0 + (t >> 6) + 4 * j;
    ok[j] = (a < cc && b < cc && a >= b);
    const int bc = min(b, cc - 1), ac = min(max(a, bc), cc - 1);
    e[j] = cmap[w + bc] + c.relpos[cseg[w + bc] + w + ac];
  }
  cplx v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = ld_elem<true>(Ls, e[j]);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int b = b0 + (t >> 6) + 4 * j;
    if (ok[j]) st_elem<true>(G, (int64_t)b * cc + a, v[j]);
  }
}

// Partial W^T Z_Bp over k in [split * SPLIT_ROWS, ...): P[c][r] = sum_k Z[k][c] W[k][r].
template <class Src>
__global__ void PXS_LB(64) k_selinv_diag_partial(Src src) {
  __shared__ Stage2<true, TM> s;
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, true);
  const int sh = p.sh0 + by;
  const int sp = bx;
  double* Ls = shift_base<true>(c, sh);
  double* W = wbase(c, sh);
  double* part = W + 2 * (int64_t)p.nb * p.wp;   // after W: split x 64 x 64 complex
  const int base = p.p0 + p.wp;
  const int64_t rbase = p.off + (int64_t)p.p0 * p.ld + base;
  const int kb = sp * (int)SPLIT_ROWS, ke = min(p.nb, kb + (int)SPLIT_ROWS);
  Acc<true, TM> acc;
  acc.zero();
  // Z_pp is symmetric and stored by its lower triangle: only P[c][r], r >= c,
  // is summed by k_selinv_diag_final, so the blocks below that are skipped
  gemm_pipe<true, TM, true>(
      acc, s, kb, ke,
      [&](int m, int kg) -> cplx {
        return ld_or_zero<true>(Ls, rbase + (int64_t)m * p.ld + kg, m < p.wp && kg < ke);
      },
      [&](int n, int kg) -> cplx {
        return ld_or_zero<true>(W, (int64_t)n * p.nb + kg, n < p.wp && kg < ke);
      },
      KFast(), NoScale(), UpperLive());
  double* out = part + 2 * (int64_t)sp * 64 * 64;
  acc_foreach<true, TM, UpperLive::kSwz>(acc, [&](int m, int n, cplx v) { st_elem<true>(out, (int64_t)m * 64 + n, v); });
}

// Z_pp = Linv^T D^{-1} Linv - sum of the partials, written over the diagonal block.
// One workgroup per shift (the block is overwritten in place, so it is read
// by the same workgroup that writes it) with 1024 threads: a wave holds one
// column cc and its 64 rows, so the work per wave follows the triangle.
constexpr int NTF = 1024;
template <class Src>
__global__ void __launch_bounds__(NTF) k_selinv_diag_final(Src src) {
  __shared__ double l_re[64][LDP];   // l[col][row] = Linv[row][col]
  __shared__ double l_im[64][LDP];
  __shared__ cplx dinv[64];
  constexpr int NE = 64 * 64 / NTF;
  Common c;
  PanelK p;
  int bx, by;
  locate(src, c, p, bx, by, false);
  const int sh = p.sh0 + by;
  double* Ls = shift_base<true>(c, sh);
  const double* W = wbase(c, sh);
  const double* part = W + 2 * (int64_t)p.nb * p.wp;
  const int wp = p.wp;
  const int t = threadIdx.x;
  const int64_t dbase = p.off + (int64_t)p.p0 * p.ld + p.p0;
  // element (r, cc) of the block at slot u: cc = t / 64 + 16 u, r = t % 64;
  // every load is issued before the first LDS store
  const int r = t & 63, c0 = t >> 6;
  cplx v[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int cc = c0 + u * (NTF / 64);
    v[u] = cplx{0.0, 0.0};
    if (cc < wp && r < wp && r >= cc) v[u] = ld_elem<true>(Ls, dbase + (int64_t)cc * p.ld + r);
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int cc = c0 + u * (NTF / 64);
    cplx x = (r > cc) ? v[u] : cplx{0.0, 0.0};
    if (r == cc && r < wp) {
      x = cplx{1.0, 0.0};
      dinv[r] = cinv(v[u]);
    }
    l_re[cc][r] = x.re;
    l_im[cc][r] = x.im;
  }
  __syncthreads();
  const int nsplit = (p.nb > 0) ? p.split : 0;
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int cc = c0 + u * (NTF / 64);
    if (cc >= wp || r >= wp || r < cc) continue;   // the stored (lower) triangle
    // sum_{k >= r} Linv[k][r] dinv[k] Linv[k][cc]
    cplx s{0.0, 0.0};
    for (int k = r; k < wp; ++k) {
      const cplx a{l_re[r][k], l_im[r][k]};
      const cplx b{l_re[cc][k], l_im[cc][k]};
      const cplx q = cmul(cmul(a, dinv[k]), b);
      s.re += q.re;
      s.im += q.im;
    }
    // partial[m = cc][n = r] holds (W^T Z_Bp)[r][cc]
    for (int sp = 0; sp < nsplit; ++sp) {
      const cplx q = ld_elem<true>(part + 2 * (int64_t)sp * 64 * 64, (int64_t)cc * 64 + r);
      s.re -= q.re;
      s.im -= q.im;
    }
    // each (r, cc) is computed by exactly one thread, and the diagonal block
    // in global memory is no longer read (Linv and D sit in LDS)
    st_elem<true>(Ls, dbase + (int64_t)cc * p.ld + r, s);
  }
}

// --------------------------------------------------------------------------
// pole sums, extraction
// --------------------------------------------------------------------------
// out[g][k] = sum_l Im(omega_{g,l} Z_l[k]); per-block partial traces.
__global__ void __launch_bounds__(NT) k_pole_sum(const double* __restrict__ L, int64_t stride,
                                                 int nshift, const double* __restrict__ wts,
                                                 int nsets, const int64_t* __restrict__ eoff,
                                                 const int32_t* __restrict__ ediag, int64_t nnz,
                                                 const double* __restrict__ H,
                                                 const double* __restrict__ S, double* out,
                                                 double* partial, int accumulate) {
  __shared__ double red[8][NT];
  double tr[8];
  for (int q = 0; q < 8; ++q) tr[q] = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * NT) {
    const int64_t e = eoff[k];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l = 0; l < nshift; ++l) {
      const double2 z = *reinterpret_cast<const double2*>(L + 2 * (stride * l + e));
      for (int g = 0; g < nsets; ++g) {
        const double wr = wts[2 * (g * nshift + l)], wi = wts[2 * (g * nshift + l) + 1];
        acc[g] += wr * z.y + wi * z.x;
      }
    }
    const double mult = ediag[k] == 1 ? 1.0 : 2.0;
    for (int g = 0; g < nsets; ++g) {
      // accumulate: add to the sums of earlier pole chunks (traces stay per chunk)
      out[(int64_t)g * nnz + k] = accumulate ? out[(int64_t)g * nnz + k] + acc[g] : acc[g];
      tr[2 * g] += mult * acc[g] * S[k];
      tr[2 * g + 1] += mult * acc[g] * H[k];
    }
  }
  for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = tr[q];
  __syncthreads();
  for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2)
      for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x < 8) partial[8 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_sum_partials(const double* partial, int nb, double* out) {
  const int q = threadIdx.x;
  if (q < 8) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[8 * b + q];
    out[q] = s;
  }
}

__global__ void k_gather(const double* __restrict__ L, const int64_t* __restrict__ eoff,
                         int64_t nnz, double2* out) {
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * NT)
    out[k] = *reinterpret_cast<const double2*>(L + 2 * eoff[k]);
}

__global__ void k_get_diag(const double* __restrict__ L, const int64_t* __restrict__ diagoff, int n,
                           int cplx_elems, double2* out) {
  // diagoff[j] = element offset of the diagonal entry of new column j
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j < n) {
    const int64_t e = diagoff[j];
    out[j] = cplx_elems ? *reinterpret_cast<const double2*>(L + 2 * e) : make_double2(L[e], 0.0);
  }
}

// --------------------------------------------------------------------------
// host orchestration
// --------------------------------------------------------------------------
namespace {

// Event pairs around the launches of one kernel class (benchmarks only).
struct Profiler {
  int kernel = KC_NONE;
  std::vector<hipEvent_t> ev;   // pool, reused across profiles
  size_t used = 0;
  int64_t launches = 0;
  double work = 0.0;    // algorithmic flops on the exact structure of L (bytes for the memory-bound classes)
  double bytes = 0.0;   // algorithmic HBM bytes: operands read once, results written once
  double stored = 0.0;  // flops on the stored (relaxed supernodal) structure
  int failed = 0;       // HIP error of an event create/record inside the profile, 0 if none
};
Profiler g_prof;

struct ProfScope {
  hipStream_t st;
  bool on;
  double w_, b_, s_;
  // work: exact algorithmic flops (bytes for the memory-bound classes);
  // stored: flops on the stored structure
  ProfScope(int kernel, hipStream_t s, double work, double bytes, double stored)
      : st(s), on(g_prof.kernel == kernel && kernel != KC_NONE), w_(work), b_(bytes), s_(stored) {
    if (!on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
      on = false;   // no event nodes inside captured graphs
      return;
    }
    while (g_prof.ev.size() < g_prof.used + 2) {
      hipEvent_t e;
      const hipError_t ce = hipEventCreate(&e);
      if (ce != hipSuccess) { on = false; g_prof.failed = (int)ce; return; }
      g_prof.ev.push_back(e);
    }
    const hipError_t re = hipEventRecord(g_prof.ev[g_prof.used], st);
    if (re != hipSuccess) { on = false; g_prof.failed = (int)re; }
  }
  ~ProfScope() {
    if (!on) return;
    // a launch counts only with both of its events recorded
    const hipError_t re = hipEventRecord(g_prof.ev[g_prof.used + 1], st);
    if (re != hipSuccess) {
      g_prof.failed = (int)re;
      return;
    }
    g_prof.used += 2;
    g_prof.launches += 1;
    g_prof.work += w_;
    g_prof.bytes += b_;
    g_prof.stored += s_;
  }
};

inline int blocks_for(int64_t n, int cap) {
  int64_t b = (n + NT - 1) / NT;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

PanelK panel_args(const Symbolic& S, const Panel& P) {
  PanelK k;
  k.off = S.off[P.J];
  k.cm = S.rowptr[P.J];
  k.ld = S.ld[P.J];
  k.p0 = P.p0;
  k.wp = P.wp;
  k.nb = P.nb_rows;
  k.col0 = S.sfirst[P.J] + P.p0;
  k.split = split_count(P.nb_rows);
  k.w = S.sfirst[P.J + 1] - S.sfirst[P.J];
  k.c = S.ld[P.J] - k.w;
  k.sh0 = 0;
  return k;
}

}  // namespace

Common make_common(const Symbolic& S, void* L, void* work) {
  Common c;
  c.L = (double*)L;
  c.stride = S.nnzL_store;
  const char* m = (const char*)S.dmaps;
  c.colmap = (const int64_t*)(m + S.o_colmap);
  c.colseg = (const int64_t*)(m + S.o_colseg);
  c.relpos = (const int32_t*)(m + S.o_relpos);
  c.work = (double*)work;
  c.wps = S.work_per_shift;
  c.wfix = S.work_fixed;
  char* w = (char*)work;
  c.absmax = (const double*)(w + WK_ABSMAX);
  c.shifts = (const double*)(w + WK_SHIFTS);
  c.info = (int64_t*)(w + WK_INFO);
  c.negc = (int64_t*)(w + WK_NEGC);
  c.pivtol = S.pivot_tol;
  c.G = nullptr;
  c.gstride = S.gather_per_shift / 8;
  c.ut = 0;
  return c;
}

#define PXS_CHECK_LAUNCH()                         \
  do {                                             \
    hipError_t e_ = hipGetLastError();             \
    if (e_ != hipSuccess) return (int)e_;          \
  } while (0)

int profile_begin(int kernel) {
  g_prof.kernel = kernel;
  g_prof.used = 0;
  g_prof.launches = 0;
  g_prof.work = 0.0;
  g_prof.bytes = 0.0;
  g_prof.stored = 0.0;
  g_prof.failed = 0;
  return 0;
}

int profile_end(double* ms, int64_t* launches, double* work, double* bytes, double* stored) {
  if (g_prof.kernel == KC_NONE) return -1;   // no profile open
  if (g_prof.failed) {                        // totals would be partial
    const int f = g_prof.failed;
    g_prof.kernel = KC_NONE;
    g_prof.used = 0;
    return f;
  }
  double tot = 0.0;
  for (size_t i = 0; i + 1 < g_prof.used; i += 2) {
    hipError_t e = hipEventSynchronize(g_prof.ev[i + 1]);
    if (e != hipSuccess) return (int)e;
    float t = 0.0f;
    e = hipEventElapsedTime(&t, g_prof.ev[i], g_prof.ev[i + 1]);
    if (e != hipSuccess) return (int)e;
    tot += t;
  }
  *ms = tot;
  *launches = g_prof.launches;
  *work = g_prof.work;
  *bytes = g_prof.bytes;
  *stored = g_prof.stored;
  g_prof.kernel = KC_NONE;
  g_prof.used = 0;
  return 0;
}

int upload_shifts(int nshift, const double* shifts_host, void* work, hipStream_t st) {
  hipError_t e = hipMemcpyAsync((char*)work + WK_SHIFTS, shifts_host, sizeof(double) * 2 * nshift,
                                hipMemcpyHostToDevice, st);
  return (int)e;
}

int upload_shifts_device(int nshift, const double* shifts_dev, void* work, hipStream_t st) {
  return (int)hipMemcpyAsync((char*)work + WK_SHIFTS, shifts_dev, sizeof(double) * 2 * nshift,
                             hipMemcpyDeviceToDevice, st);
}

int upload_weights_device(int nshift, int nsets, const double* weights_dev, void* work, hipStream_t st) {
  return (int)hipMemcpyAsync((char*)work + WK_WEIGHTS, weights_dev, sizeof(double) * 2 * nsets * nshift,
                             hipMemcpyDeviceToDevice, st);
}

int upload_weights(int nshift, int nsets, const double* weights_host, void* work, hipStream_t st) {
  hipError_t e = hipMemcpyAsync((char*)work + WK_WEIGHTS, weights_host,
                                sizeof(double) * 2 * nsets * nshift, hipMemcpyHostToDevice, st);
  return (int)e;
}

template <bool CPLX>
int run_factor(const Symbolic& S, const double* H, const double* Sv, int nshift,
               const double* shifts_host, void* L, void* work, hipStream_t st, bool inorder) {
  int e = upload_shifts(nshift, shifts_host, work, st);
  if (e != 0) return e;
  return run_factor_kernels<CPLX>(S, H, Sv, nshift, L, work, st, inorder);
}

// Streams and events owned by the library for the subtree-parallel
// factorization and SelInv (created on first use on the current device,
// kept for the process).
struct StreamPool {
  int device = -1;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
};
StreamPool g_pool;

int ensure_pool(int nstreams, int nevents) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (g_pool.device != dev) {
    g_pool.streams.clear();   // streams of another device are left alone
    g_pool.events.clear();
    g_pool.device = dev;
  }
  while ((int)g_pool.streams.size() < nstreams) {
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return (int)e;
    g_pool.streams.push_back(s);
  }
  while ((int)g_pool.events.size() < nevents) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return (int)e;
    g_pool.events.push_back(ev);
  }
  return 0;
}

// Before the factorization: pivot flags and counts cleared, max|H|, max|S|
// for the pivot threshold, the factor storage zeroed and every shift's
// H - w_l S assembled into it.
template <bool CPLX>
int factor_prologue(const Symbolic& S, const double* H, const double* Sv, int nshift, void* L, void* work,
                    hipStream_t st) {
  char* w = (char*)work;
  hipLaunchKernelGGL(k_zero_i64, dim3((2 * MAX_SHIFTS + NT - 1) / NT), dim3(NT), 0, st,
                     (int64_t*)(w + WK_INFO), 2 * MAX_SHIFTS);
  PXS_CHECK_LAUNCH();
  const char* m = (const char*)S.dmaps;
  const int64_t* eoff = (const int64_t*)(m + S.o_entry_off);
  const int nbm = blocks_for(S.nnz_lower, ABSMAX_BLOCKS);
  hipLaunchKernelGGL(k_absmax_partial, dim3(nbm), dim3(NT), 0, st, H, Sv, S.nnz_lower,
                     (double*)(w + WK_ABSMAX_PART));
  hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(64), 0, st, (const double*)(w + WK_ABSMAX_PART),
                     nbm, (double*)(w + WK_ABSMAX));
  PXS_CHECK_LAUNCH();
  const int64_t total_d = (CPLX ? 2 : 1) * S.nnzL_store * (int64_t)nshift;   // doubles
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(total_d / 2 + 1, 8192)), dim3(NT), 0, st,
                     (double2*)L, total_d / 2);
  if (total_d & 1)
    hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(64), 0, st, (double2*)((double*)L + total_d - 2), (int64_t)1);
  PXS_CHECK_LAUNCH();
  {
    // bytes: H, S, offsets read once per shift block; one element written per entry and shift
    const double ab = (double)S.nnz_lower * (24.0 + (CPLX ? 16.0 : 8.0) * nshift);
    ProfScope ps(KC_ASSEMBLE, st, ab, ab, ab);
    hipLaunchKernelGGL(k_assemble<CPLX>, dim3(blocks_for(S.nnz_lower, 2048), nshift), dim3(NT), 0, st,
                       (double*)L, S.nnzL_store, H, Sv, eoff, S.nnz_lower, (const double*)(w + WK_SHIFTS));
  }
  PXS_CHECK_LAUNCH();
  return 0;
}

template <bool CPLX>
int run_factor_kernels(const Symbolic& S, const double* H, const double* Sv, int nshift, void* L,
                       void* work, hipStream_t st, bool inorder) {
  {
    const int e = factor_prologue<CPLX>(S, H, Sv, nshift, L, work, st);
    if (e) return e;
  }
  Common c = make_common(S, L, work);
  const int TR = S.tile_rows;
  const double fm = CPLX ? 8.0 : 2.0;   // flops per multiply-add
  const double eb = CPLX ? 16.0 : 8.0;  // bytes per element
  // the panel work of one panel: left-looking update from the earlier
  // columns of its supernode, LDL^T of the diagonal block, the rows below
  auto panel_work = [&](const Panel& P, hipStream_t s) -> int {
    PanelK k = panel_args(S, P);
    const PanelMacs& xm = S.xm_panel[&P - S.panels.data()];
    if (k.p0 > 0) {
      const int nrows = k.ld - k.p0;
      ProfScope ps(KC_UPDATE, s, fm * nshift * xm.intu, eb * nshift * ((double)nrows * k.p0 + 2.0 * nrows * k.wp),
                   fm * nshift * ((double)nrows * k.wp - 0.5 * k.wp * (k.wp - 1)) * k.p0);
      if (TR == 64)
        hipLaunchKernelGGL((k_int_update<CPLX, 64, OnePanel>), dim3((nrows + 63) / 64, nshift), dim3(NT), 0, s, OnePanel{c, k});
      else
        hipLaunchKernelGGL((k_int_update<CPLX, 128, OnePanel>), dim3((nrows + 127) / 128, nshift), dim3(NT), 0, s, OnePanel{c, k});
    }
    {
      ProfScope ps(KC_DIAG, s, fm * nshift * xm.diag, eb * nshift * (double)k.wp * (k.wp + 1),
                   fm * nshift * (double)k.wp * k.wp * k.wp / 3.0);
      hipLaunchKernelGGL((k_diag<CPLX, OnePanel>), dim3(1, nshift), dim3(NTD), 0, s, OnePanel{c, k});
    }
    if (k.nb > 0) {
      const int nt = (k.nb + TR - 1) / TR;
      ProfScope ps(KC_TRSM, s, fm * nshift * xm.trsm, eb * nshift * (2.0 * k.nb * k.wp + 0.5 * k.wp * (k.wp + 1)),
                   fm * nshift * (double)k.nb * k.wp * (k.wp + 1) / 2.0);
      if (TR == 64)
        hipLaunchKernelGGL((k_trsm<CPLX, 64, OnePanel>), dim3(nt, nshift), dim3(NT), 0, s, OnePanel{c, k});
      else
        hipLaunchKernelGGL((k_trsm<CPLX, 128, OnePanel>), dim3(nt, nshift), dim3(NT), 0, s, OnePanel{c, k});
    }
    PXS_CHECK_LAUNCH();
    return 0;
  };
  // right-looking: the whole supernode J updates its ancestors once (K = w),
  // scattered into their panels; J's last panel describes its row list
  auto scatter = [&](const Panel& P, hipStream_t s) -> int {
    const int32_t w = S.sfirst[P.J + 1] - S.sfirst[P.J];
    const int32_t below = S.ld[P.J] - w;
    if (below <= 0) return 0;
    PanelK u = panel_args(S, P);
    u.p0 = 0;
    u.wp = w;
    u.nb = below;
    const int ntj = (below + TM - 1) / TM, nti = (below + TR - 1) / TR;
    ProfScope ps(KC_UPDATE, s, fm * nshift * S.xm_update[P.J],
                 eb * nshift * ((double)below * w + (double)below * (below + 1)),
                 fm * nshift * (double)below * (below + 1) / 2.0 * w);
    if (TR == 64)
      hipLaunchKernelGGL((k_update<CPLX, 64, OnePanel>), dim3(ntj * nti, nshift), dim3(NT), 0, s, OnePanel{c, u});
    else
      hipLaunchKernelGGL((k_update<CPLX, 128, OnePanel>), dim3(ntj * nti, nshift), dim3(NT), 0, s, OnePanel{c, u});
    PXS_CHECK_LAUNCH();
    return 0;
  };
  const size_t np = S.panels.size();
  const int ns = S.nsuper;
  const int NS = S.sel_nstreams;
  if ((int)S.fac_order.size() != ns || (int)S.fac_child.size() != ns) return (int)hipErrorInvalidValue;
  std::vector<int> pfirst(ns, -1), plast(ns, -1);
  for (size_t ip = 0; ip < np; ++ip) {
    const int J = S.panels[ip].J;
    if (pfirst[J] < 0) pfirst[J] = (int)ip;
    plast[J] = (int)ip;
  }
  // Supernodes are issued in fac_order on every path, so each entry receives
  // its scatters in the same order and the factors are bit-identical whether
  // the subtree streams are used or not.  Inside a stream capture, or with
  // one subtree stream, everything runs on the caller's stream.
  int err = 0;
  if (S.fused_lanes && NS > 1) {
    // fused lanes (see run_selinv_lanes; no library streams or events, so
    // also on the in-order paths): the panel operations of each lane
    // (the sel_stream subtrees, supernodes in fac_order) and one more lane of
    // the ancestor scatters in fac_order, all on the caller's stream; a
    // launch takes the next operation of every ready lane of one kind.  The
    // first panel operation of J waits for the scatter of fac_child[J] (and
    // so for every scatter before it), a scatter for the last panel
    // operation of its supernode; scatters are never fused with each other.
    enum : int32_t { FK_INT, FK_DIAG, FK_TRSM, FK_UPD };
    struct FOp {
      int32_t kind, J;
      bool first, last;
      GroupItem it;
      double work, bytes, stored;
    };
    if (NS > MAX_LANES) return (int)hipErrorInvalidValue;
    std::vector<std::vector<FOp>> lane(NS + 1);   // lane NS: the scatters
    for (int J : S.fac_order) {
      if (pfirst[J] < 0) continue;
      std::vector<FOp>& ops = lane[S.sel_stream[J]];
      const size_t n0 = ops.size();
      auto add = [&](std::vector<FOp>& v, int32_t kind, const PanelK& k, int64_t tiles, double w, double b,
                     double s) {
        FOp o;
        o.kind = kind;
        o.J = J;
        o.first = &v == &ops && v.size() == n0;
        o.last = false;
        o.it.c = c;
        o.it.p = k;
        o.it.start = 0;
        o.it.tiles = (int32_t)tiles;
        o.it.nsh = nshift;
        o.work = w;
        o.bytes = b;
        o.stored = s;
        v.push_back(o);
      };
      for (int ip = pfirst[J]; ip <= plast[J]; ++ip) {
        const PanelK k = panel_args(S, S.panels[ip]);
        const PanelMacs& xm = S.xm_panel[ip];
        if (k.p0 > 0) {
          const int nrows = k.ld - k.p0;
          add(ops, FK_INT, k, (nrows + TR - 1) / TR, fm * nshift * xm.intu,
              eb * nshift * ((double)nrows * k.p0 + 2.0 * nrows * k.wp),
              fm * nshift * ((double)nrows * k.wp - 0.5 * k.wp * (k.wp - 1)) * k.p0);
        }
        add(ops, FK_DIAG, k, 1, fm * nshift * xm.diag, eb * nshift * (double)k.wp * (k.wp + 1),
            fm * nshift * (double)k.wp * k.wp * k.wp / 3.0);
        if (k.nb > 0)
          add(ops, FK_TRSM, k, (k.nb + TR - 1) / TR, fm * nshift * xm.trsm,
              eb * nshift * (2.0 * k.nb * k.wp + 0.5 * k.wp * (k.wp + 1)),
              fm * nshift * (double)k.nb * k.wp * (k.wp + 1) / 2.0);
      }
      ops.back().last = true;
      if (S.sparent[J] >= 0) add(lane[NS], FK_UPD, panel_args(S, S.panels[plast[J]]), 0, 0.0, 0.0, 0.0);
    }
    std::vector<int64_t> pdone(ns, -1), sdone(ns, -1);   // launch of J's last panel op / scatter
    std::vector<size_t> pos(NS + 1, 0);
    int64_t nl = 0;
    auto ready = [&](int q) {
      if (pos[q] >= lane[q].size()) return false;
      const FOp& o = lane[q][pos[q]];
      if (q == NS) return pdone[o.J] >= 0 && pdone[o.J] < nl;
      if (!o.first) return true;
      const int ch = S.fac_child[o.J];
      return ch < 0 || (sdone[ch] >= 0 && sdone[ch] < nl);
    };
    for (;;) {
      int lead = -1;
      size_t most = 0;
      for (int q = 0; q <= NS; ++q) {
        if (!ready(q)) continue;
        const size_t left = lane[q].size() - pos[q];
        if (left > most) {
          most = left;
          lead = q;
        }
      }
      if (lead < 0) break;
      const int32_t kind = lane[lead][pos[lead]].kind;
      if (kind == FK_UPD) {
        const FOp& o = lane[NS][pos[NS]];
        if ((err = scatter(S.panels[plast[o.J]], st))) return err;
        sdone[o.J] = nl++;
        ++pos[NS];
        continue;
      }
      LaneGroup grp;
      grp.n = 0;
      int64_t start = 0;
      double w = 0.0, b = 0.0, s = 0.0;
      for (int q = 0; q < NS; ++q) {
        if (!ready(q) || lane[q][pos[q]].kind != kind) continue;
        const FOp& o = lane[q][pos[q]];
        GroupItem it = o.it;
        it.start = start;
        start += (int64_t)it.tiles * it.nsh;
        grp.it[grp.n++] = it;
        w += o.work;
        b += o.bytes;
        s += o.stored;
        if (o.last) pdone[o.J] = nl;
        ++pos[q];
      }
      if (start > (int64_t)INT32_MAX) return (int)hipErrorInvalidConfiguration;
      const dim3 grid((unsigned)start);
      if (kind == FK_INT) {
        ProfScope ps(KC_UPDATE, st, w, b, s);
        if (TR == 64) hipLaunchKernelGGL((k_int_update<CPLX, 64, LaneGroup>), grid, dim3(NT), 0, st, grp);
        else hipLaunchKernelGGL((k_int_update<CPLX, 128, LaneGroup>), grid, dim3(NT), 0, st, grp);
      } else if (kind == FK_DIAG) {
        ProfScope ps(KC_DIAG, st, w, b, s);
        hipLaunchKernelGGL((k_diag<CPLX, LaneGroup>), grid, dim3(NTD), 0, st, grp);
      } else {
        ProfScope ps(KC_TRSM, st, w, b, s);
        if (TR == 64) hipLaunchKernelGGL((k_trsm<CPLX, 64, LaneGroup>), grid, dim3(NT), 0, st, grp);
        else hipLaunchKernelGGL((k_trsm<CPLX, 128, LaneGroup>), grid, dim3(NT), 0, st, grp);
      }
      PXS_CHECK_LAUNCH();
      ++nl;
    }
    for (int q = 0; q <= NS; ++q)
      if (pos[q] != lane[q].size()) return (int)hipErrorUnknown;   // unreachable: some lane is always ready
    return 0;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t he = hipStreamIsCapturing(st, &cap);
  if (he != hipSuccess) return (int)he;
  if (cap != hipStreamCaptureStatusNone || NS <= 1 || inorder) {
    for (int J : S.fac_order) {
      if (pfirst[J] < 0) continue;
      for (int ip = pfirst[J]; ip <= plast[J]; ++ip)
        if ((err = panel_work(S.panels[ip], st))) return err;
      if ((err = scatter(S.panels[plast[J]], st))) return err;
    }
    return 0;
  }
  // subtree streams: the panel work of J on pool stream sel_stream[J] once
  // the scatters into J are done (the scatter of fac_child[J] and, the
  // caller's stream being in order, every scatter issued before it); the
  // scatter of J on the caller's stream after J's panel work.  Scatters of
  // different supernodes write the same ancestor entries, so they stay on
  // the one stream, in fac_order.
  if ((err = ensure_pool(NS, 2 * ns + 1))) return err;
  hipEvent_t* evp = g_pool.events.data();   // evp[J]: panel work of J done
  hipEvent_t* evs = evp + ns;               // evs[J]: scatter of J done
  hipEvent_t evf = evp[2 * ns];             // assembly done
  if ((he = hipEventRecord(evf, st)) != hipSuccess) return (int)he;
  for (int J : S.fac_order) {
    if (pfirst[J] < 0) continue;
    hipStream_t sj = g_pool.streams[S.sel_stream[J]];
    const int ch = S.fac_child[J];
    if ((he = hipStreamWaitEvent(sj, ch >= 0 ? evs[ch] : evf, 0)) != hipSuccess) return (int)he;
    for (int ip = pfirst[J]; ip <= plast[J]; ++ip)
      if ((err = panel_work(S.panels[ip], sj))) return err;
    if ((he = hipEventRecord(evp[J], sj)) != hipSuccess) return (int)he;
    if (S.sparent[J] < 0) continue;   // a root: joined below
    if ((he = hipStreamWaitEvent(st, evp[J], 0)) != hipSuccess) return (int)he;
    if ((err = scatter(S.panels[plast[J]], st))) return err;
    if ((he = hipEventRecord(evs[J], st)) != hipSuccess) return (int)he;
  }
  for (int J = 0; J < ns; ++J)
    if (S.sparent[J] < 0 && pfirst[J] >= 0)
      if ((he = hipStreamWaitEvent(st, evp[J], 0)) != hipSuccess) return (int)he;
  return 0;
}

template int run_factor<true>(const Symbolic&, const double*, const double*, int, const double*, void*, void*,
                              hipStream_t, bool);
template int run_factor<false>(const Symbolic&, const double*, const double*, int, const double*, void*, void*,
                               hipStream_t, bool);
template int run_factor_kernels<true>(const Symbolic&, const double*, const double*, int, void*, void*, hipStream_t,
                                      bool);
template int run_factor_kernels<false>(const Symbolic&, const double*, const double*, int, void*, void*,
                                       hipStream_t, bool);

int64_t selinv_work_bytes(const Symbolic& S, int nshift) {
  const int chunk = (S.selinv_chunk > 0 && S.selinv_chunk < nshift) ? S.selinv_chunk : nshift;
  int64_t g = 0;
  for (int64_t b : S.gather_bytes) g += b;
  return S.work_fixed + (int64_t)nshift * S.sel_nstreams * S.work_per_shift + (int64_t)chunk * g;
}

int64_t selinv_work_bytes_inorder(const Symbolic& S, int nshift) {
  const int chunk = (S.selinv_chunk > 0 && S.selinv_chunk < nshift) ? S.selinv_chunk : nshift;
  return S.work_fixed + (int64_t)nshift * S.work_per_shift + (int64_t)chunk * S.gather_per_shift;
}

// Workspace of the allocation-free entry point (pxs_density_matrix_noalloc).
// Host code never passes this name to a kernel or a copy: it stands for a
// host-side shadow there; the device address comes from noalloc_scratch.
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

int noalloc_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return 0;
}

#define PXS_HIP(call)                      \
  do {                                     \
    hipError_t e_ = (call);                \
    if (e_ != hipSuccess) return (int)e_;  \
  } while (0)

int selinv_streams_ready(const Symbolic& S) {
  // streams are created here, never inside a stream capture
  return ensure_pool(S.sel_nstreams - 1, 0);
}

int selinv_event_count(const Symbolic& S) { return S.nsuper + S.sel_nstreams + 1; }

namespace {

// Selected inversion with the subtree lanes fused (fused_lanes).  The
// supernodes keep the lanes of the stream assignment (sel_stream) and each
// lane its own workspace regions, as on separate streams; the operations of
// a lane (per supernode from the root down: the Z_CC gather, then per panel
// from the last: L-hat, off-diagonal product, diagonal partials, diagonal
// final) run in their order.  Every launch on the caller's stream takes the
// next operation of each lane whose next operation is of one kind and ready
// -- the first operation of a supernode whose parent is on another lane
// waits until the parent's last operation was in an earlier launch -- and
// runs them as one grid (LaneGroup); the kind is that of the ready lane with
// the most operations left.  Some lane is always ready: the one whose next
// supernode is the highest-numbered, since its parent (a higher number) is
// already done.  Each panel operation computes what it computes on a stream
// of its own, so the results are the bits of the other paths.
enum LaneKind : int32_t { LK_GATHER, LK_LHAT, LK_OFF, LK_DPART, LK_DFIN };

struct LaneOp {
  int32_t kind;
  int32_t J;
  bool first;   // first operation of supernode J
  bool last;    // last operation of J
  GroupItem it;
  double work, bytes, stored;   // profile figures (ProfScope)
};

int lane_launch(int32_t kind, int TR, const LaneGroup& g, int64_t blocks, hipStream_t st) {
  const dim3 grid((unsigned)blocks);
  switch (kind) {
    case LK_GATHER: hipLaunchKernelGGL(k_gather_cc<LaneGroup>, grid, dim3(NT), 0, st, g); break;
    case LK_LHAT:
      if (TR == 64) hipLaunchKernelGGL((k_lhat<64, LaneGroup>), grid, dim3(NT), 0, st, g);
      else hipLaunchKernelGGL((k_lhat<128, LaneGroup>), grid, dim3(NT), 0, st, g);
      break;
    case LK_OFF:
      if (TR == 64) hipLaunchKernelGGL((k_selinv_off<64, LaneGroup>), grid, dim3(NT), 0, st, g);
      else hipLaunchKernelGGL((k_selinv_off<128, LaneGroup>), grid, dim3(NT), 0, st, g);
      break;
    case LK_DPART: hipLaunchKernelGGL(k_selinv_diag_partial<LaneGroup>, grid, dim3(NT), 0, st, g); break;
    case LK_DFIN: hipLaunchKernelGGL(k_selinv_diag_final<LaneGroup>, grid, dim3(NTF), 0, st, g); break;
    default: return (int)hipErrorInvalidValue;
  }
  PXS_CHECK_LAUNCH();
  return 0;
}

const int kLaneClass[5] = {KC_GATHER, KC_LHAT, KC_SELINV_OFF, KC_SELINV_DIAG, KC_NONE};

int run_selinv_lanes(const Symbolic& S, int nshift, void* L, void* work, hipStream_t st) {
  const int NL = S.sel_nstreams;
  if (NL < 1 || NL > MAX_LANES) return (int)hipErrorInvalidValue;
  const int ns = S.nsuper;
  const int TR = S.tile_rows;
  const int chunk = (S.selinv_chunk > 0 && S.selinv_chunk < nshift) ? S.selinv_chunk : nshift;
  // workspace views as on NL streams (selinv_work_bytes)
  std::vector<Common> cs(NL, make_common(S, L, work));
  int64_t gofs = S.work_fixed + (int64_t)nshift * NL * S.work_per_shift;
  for (int q = 0; q < NL; ++q) {
    cs[q].wfix = S.work_fixed + (int64_t)q * nshift * S.work_per_shift;
    cs[q].G = (double*)((char*)work + gofs);
    cs[q].gstride = S.gather_bytes[q] / 8;
    gofs += (int64_t)chunk * S.gather_bytes[q];
  }
  std::vector<int> pfirst(ns, 0);
  for (int ip = (int)S.panels.size() - 1; ip >= 0; --ip) pfirst[S.panels[ip].J] = ip;
  std::vector<std::vector<LaneOp>> lane(NL);
  std::vector<int64_t> done(ns);   // launch of J's last operation, -1 before it
  for (int sh0 = 0; sh0 < nshift; sh0 += chunk) {
    const int nsh = std::min(chunk, nshift - sh0);
    for (auto& v : lane) v.clear();
    for (int J = ns - 1; J >= 0; --J) {
      const int q = S.sel_stream[J];
      std::vector<LaneOp>& ops = lane[q];
      const size_t n0 = ops.size();
      auto add = [&](int32_t kind, const PanelK& k, int64_t tiles, double w, double b, double s) {
        LaneOp o;
        o.kind = kind;
        o.J = J;
        o.first = ops.size() == n0;
        o.last = false;
        o.it.c = cs[q];
        o.it.p = k;
        o.it.start = 0;
        o.it.tiles = (int32_t)tiles;
        o.it.nsh = nsh;
        o.work = w;
        o.bytes = b;
        o.stored = s;
        ops.push_back(o);
      };
      const int first = pfirst[J];
      int last = first;
      while (last + 1 < (int)S.panels.size() && S.panels[last + 1].J == J) ++last;
      PanelK g = panel_args(S, S.panels[last]);
      g.sh0 = sh0;
      if (g.c > 0) {
        const int64_t nt = (g.c + TM - 1) / TM;
        const double gb = (32.0 * nsh + 4.0) * 0.5 * g.c * (g.c + 1);
        add(LK_GATHER, g, nt * (nt + 1) / 2, gb, gb, gb);
      }
      for (int ip = last; ip >= first; --ip) {
        PanelK k = panel_args(S, S.panels[ip]);
        k.sh0 = sh0;
        const PanelMacs& xm = S.xm_panel[ip];
        if (k.nb > 0) {
          const int64_t nt = (k.nb + TR - 1) / TR;
          add(LK_LHAT, k, nt, 0.0, 16.0 * nsh * (2.0 * k.nb * k.wp + 0.5 * k.wp * (k.wp + 1)),
              8.0 * nsh * (double)k.nb * k.wp * (k.wp + 1) / 2.0);
          add(LK_OFF, k, nt, 8.0 * nsh * xm.off, 16.0 * nsh * (0.5 * k.nb * (k.nb + 1) + 2.0 * k.nb * k.wp),
              8.0 * nsh * (double)k.nb * k.nb * k.wp);
          add(LK_DPART, k, k.split, 8.0 * nsh * xm.sdiag, 16.0 * nsh * (2.0 * k.nb * k.wp + (double)k.wp * k.wp),
              8.0 * nsh * (double)k.nb * k.wp * k.wp);
        }
        add(LK_DFIN, k, 1, 0.0, 0.0, 0.0);
      }
      ops.back().last = true;
    }
    std::fill(done.begin(), done.end(), (int64_t)-1);
    std::vector<size_t> pos(NL, 0);
    int64_t nl = 0;   // launches of this chunk so far
    auto ready = [&](int q) {
      if (pos[q] >= lane[q].size()) return false;
      const LaneOp& o = lane[q][pos[q]];
      if (!o.first) return true;
      const int P = S.sparent[o.J];
      return P < 0 || S.sel_stream[P] == q || (done[P] >= 0 && done[P] < nl);
    };
    for (;;) {
      int lead = -1;
      size_t most = 0;
      for (int q = 0; q < NL; ++q) {
        if (!ready(q)) continue;
        const size_t left = lane[q].size() - pos[q];
        if (left > most) {
          most = left;
          lead = q;
        }
      }
      if (lead < 0) break;
      const int32_t kind = lane[lead][pos[lead]].kind;
      LaneGroup grp;
      grp.n = 0;
      int64_t start = 0;
      double w = 0.0, b = 0.0, s = 0.0;
      for (int q = 0; q < NL; ++q) {
        if (!ready(q) || lane[q][pos[q]].kind != kind) continue;
        const LaneOp& o = lane[q][pos[q]];
        GroupItem it = o.it;
        it.start = start;
        start += (int64_t)it.tiles * it.nsh;
        grp.it[grp.n++] = it;
        w += o.work;
        b += o.bytes;
        s += o.stored;
        if (o.last) done[o.J] = nl;
        ++pos[q];
      }
      if (start > (int64_t)INT32_MAX) return (int)hipErrorInvalidConfiguration;
      {
        ProfScope ps(kLaneClass[kind], st, w, b, s);
        const int e = lane_launch(kind, TR, grp, start, st);
        if (e) return e;
      }
      ++nl;
    }
    for (int q = 0; q < NL; ++q)
      if (pos[q] != lane[q].size()) return (int)hipErrorUnknown;   // unreachable: some lane is always ready
  }
  return 0;
}

}  // namespace

int run_selinv(const Symbolic& S, int nshift, void* L, void* work, hipStream_t st,
               hipEvent_t* events, bool inorder) {
  if (S.fused_lanes && !inorder && S.sel_nstreams > 1) return run_selinv_lanes(S, nshift, L, work, st);
  // inside a stream capture everything runs on the capturing stream: the
  // subtree streams are used by eager runs only
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  PXS_HIP(hipStreamIsCapturing(st, &cap));
  const bool single = inorder || (cap != hipStreamCaptureStatusNone) || S.sel_nstreams == 1;
  const int NS = single ? 1 : S.sel_nstreams;
  const int ns = S.nsuper;
  const int TR = S.tile_rows;
  // one stream needs no pool: the in-order path creates no streams or events
  int err = single ? 0 : ensure_pool(NS - 1, events ? 0 : selinv_event_count(S));
  if (err) return err;
  std::vector<hipStream_t> strm(NS);
  strm[0] = st;
  for (int q = 1; q < NS; ++q) strm[q] = g_pool.streams[q - 1];
  // events: the caller's (a graph plan keeps its own, since an event last
  // recorded inside a capture must not be waited on outside it) or the
  // pool's; none on one stream
  hipEvent_t* ev = single ? nullptr : (events ? events : g_pool.events.data());   // ev[J]: SelInv of J done
  hipEvent_t* ev_join = single ? nullptr : ev + ns;   // ev_join[q], q >= 1
  hipEvent_t ev_fork = single ? nullptr : ev[ns + NS];
  const int chunk = (S.selinv_chunk > 0 && S.selinv_chunk < nshift) ? S.selinv_chunk : nshift;
  // per-stream workspace views
  std::vector<Common> cs(NS, make_common(S, L, work));
  // workspace views (selinv_work_bytes): per-shift regions of all streams,
  // then the dense Z_CC regions of all streams; one stream alone uses one
  // per-shift region and a Z_CC area with the largest stride right after it
  // (selinv_work_bytes_inorder <= selinv_work_bytes)
  int64_t gofs = S.work_fixed + (int64_t)nshift * (single ? 1 : S.sel_nstreams) * S.work_per_shift;
  for (int q = 0; q < NS; ++q) {
    cs[q].wfix = S.work_fixed + (int64_t)q * nshift * S.work_per_shift;
    cs[q].G = (double*)((char*)work + gofs);
    cs[q].gstride = (single ? S.gather_per_shift : S.gather_bytes[q]) / 8;
    gofs += (int64_t)chunk * S.gather_bytes[q];
  }
  auto stream_of = [&](int J) { return single ? 0 : S.sel_stream[J]; };
  // first panel of every supernode (panels are grouped by supernode, in order)
  std::vector<int> pfirst(ns, 0);
  for (int ip = (int)S.panels.size() - 1; ip >= 0; --ip) pfirst[S.panels[ip].J] = ip;

  for (int sh0 = 0; sh0 < nshift; sh0 += chunk) {
    const int nsh = std::min(chunk, nshift - sh0);
    if (NS > 1) {
      PXS_HIP(hipEventRecord(ev_fork, st));
      for (int q = 1; q < NS; ++q) PXS_HIP(hipStreamWaitEvent(strm[q], ev_fork, 0));
    }
    // supernodes from the roots down; a child on another stream waits for
    // its parent's event
    for (int J = ns - 1; J >= 0; --J) {
      const int q = stream_of(J);
      hipStream_t sj = strm[q];
      const Common& c = cs[q];
      const int P = S.sparent[J];
      if (P >= 0 && stream_of(P) != q) PXS_HIP(hipStreamWaitEvent(sj, ev[P], 0));
      const int first = pfirst[J];
      int last = first;
      while (last + 1 < (int)S.panels.size() && S.panels[last + 1].J == J) ++last;
      PanelK g = panel_args(S, S.panels[last]);
      g.sh0 = sh0;
      if (g.c > 0) {
        const int nt = (g.c + TM - 1) / TM;
        // bytes: the lower triangle of Z_CC read from the ancestors and written to G, relative positions
        const double gb = (32.0 * nsh + 4.0) * 0.5 * g.c * (g.c + 1);
        ProfScope ps(KC_GATHER, sj, gb, gb, gb);
        hipLaunchKernelGGL(k_gather_cc<OnePanel>, dim3(nt * (nt + 1) / 2, nsh), dim3(NT), 0, sj, OnePanel{c, g});
      }
      for (int ip = last; ip >= first; --ip) {
        PanelK k = panel_args(S, S.panels[ip]);
        k.sh0 = sh0;
        const PanelMacs& xm = S.xm_panel[ip];
        if (k.nb > 0) {
          const int nt = (k.nb + TR - 1) / TR;
          {
            // L-hat is a by-product of the blocked algorithm: no exact flops
            ProfScope ps(KC_LHAT, sj, 0.0, 16.0 * nsh * (2.0 * k.nb * k.wp + 0.5 * k.wp * (k.wp + 1)),
                         8.0 * nsh * (double)k.nb * k.wp * (k.wp + 1) / 2.0);
            if (TR == 64)
              hipLaunchKernelGGL((k_lhat<64, OnePanel>), dim3(nt, nsh), dim3(NT), 0, sj, OnePanel{c, k});
            else
              hipLaunchKernelGGL((k_lhat<128, OnePanel>), dim3(nt, nsh), dim3(NT), 0, sj, OnePanel{c, k});
          }
          {
            // bytes: Z_BB (one triangle), L-hat read, Z_Bp written
            ProfScope ps(KC_SELINV_OFF, sj, 8.0 * nsh * xm.off,
                         16.0 * nsh * (0.5 * k.nb * (k.nb + 1) + 2.0 * k.nb * k.wp),
                         8.0 * nsh * (double)k.nb * k.nb * k.wp);
            if (TR == 64)
              hipLaunchKernelGGL((k_selinv_off<64, OnePanel>), dim3(nt, nsh), dim3(NT), 0, sj, OnePanel{c, k});
            else
              hipLaunchKernelGGL((k_selinv_off<128, OnePanel>), dim3(nt, nsh), dim3(NT), 0, sj, OnePanel{c, k});
          }
          {
            ProfScope ps(KC_SELINV_DIAG, sj, 8.0 * nsh * xm.sdiag,
                         16.0 * nsh * (2.0 * k.nb * k.wp + (double)k.wp * k.wp),
                         8.0 * nsh * (double)k.nb * k.wp * k.wp);
            hipLaunchKernelGGL(k_selinv_diag_partial<OnePanel>, dim3(k.split, nsh), dim3(NT), 0, sj, OnePanel{c, k});
          }
        }
        hipLaunchKernelGGL(k_selinv_diag_final<OnePanel>, dim3(1, nsh), dim3(NTF), 0, sj, OnePanel{c, k});
        PXS_CHECK_LAUNCH();
      }
      if (!single && S.cross_child[J]) PXS_HIP(hipEventRecord(ev[J], sj));
    }
    if (NS > 1) {
      for (int q = 1; q < NS; ++q) {
        PXS_HIP(hipEventRecord(ev_join[q], strm[q]));
        PXS_HIP(hipStreamWaitEvent(st, ev_join[q], 0));
      }
    }
  }
  return 0;
}

int run_inertia_async(const Symbolic& S, const double* H, const double* Sv, int nshift, const double* eps_dev,
                      void* L, void* work, int64_t* neg_dev, int64_t* info_dev, hipStream_t st) {
  char* w = (char*)work;
  hipLaunchKernelGGL(k_real_shifts, dim3((nshift + NT - 1) / NT), dim3(NT), 0, st, eps_dev,
                     (double*)(w + WK_SHIFTS), nshift);
  PXS_CHECK_LAUNCH();
  const int e = run_factor_kernels<false>(S, H, Sv, nshift, L, work, st, true);
  if (e) return e;
  PXS_HIP(hipMemcpyAsync(neg_dev, w + WK_NEGC, sizeof(int64_t) * nshift, hipMemcpyDeviceToDevice, st));
  PXS_HIP(hipMemcpyAsync(info_dev, w + WK_INFO, sizeof(int64_t) * nshift, hipMemcpyDeviceToDevice, st));
  return 0;
}

int run_pole_sum(const Symbolic& S, int nshift, const void* L, void* work, const double* H,
                 const double* Sv, int nsets, const double* weights_host, double* out,
                 hipStream_t st) {
  int e = upload_weights(nshift, nsets, weights_host, work, st);
  if (e != 0) return e;
  return run_pole_sum_kernels(S, nshift, L, work, H, Sv, nsets, out, 0, st);
}

int run_pole_sum_kernels(const Symbolic& S, int nshift, const void* L, void* work, const double* H,
                         const double* Sv, int nsets, double* out, int accumulate, hipStream_t st) {
  char* w = (char*)work;
  const char* m = (const char*)S.dmaps;
  const int nb = blocks_for(S.nnz_lower, POLESUM_BLOCKS);
  // bytes: one complex per entry and shift, offsets, flags, H, S, nsets outputs
  const double ab = (double)S.nnz_lower * (16.0 * nshift + 28.0 + 8.0 * nsets);
  ProfScope ps(KC_POLESUM, st, ab, ab, ab);
  hipLaunchKernelGGL(k_pole_sum, dim3(nb), dim3(NT), 0, st, (const double*)L, S.nnzL_store, nshift,
                     (const double*)(w + WK_WEIGHTS), nsets, (const int64_t*)(m + S.o_entry_off),
                     (const int32_t*)(m + S.o_entry_diag), S.nnz_lower, H, Sv, out,
                     (double*)(w + WK_POLESUM_PART), accumulate);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, (const double*)(w + WK_POLESUM_PART), nb,
                     (double*)(w + WK_TRACES));
  PXS_CHECK_LAUNCH();
  return 0;
}

int run_gather(const Symbolic& S, int shift, const void* L, void* out, hipStream_t st) {
  const char* m = (const char*)S.dmaps;
  const double* Ls = (const double*)L + 2 * S.nnzL_store * (int64_t)shift;
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(S.nnz_lower, 4096)), dim3(NT), 0, st, Ls,
                     (const int64_t*)(m + S.o_entry_off), S.nnz_lower, (double2*)out);
  PXS_CHECK_LAUNCH();
  return 0;
}

int run_get_diag(const Symbolic& S, int shift, bool cplx, const void* L, void* out, hipStream_t st) {
  const char* m = (const char*)S.dmaps;
  const double* Ls = (const double*)L + (cplx ? 2 : 1) * S.nnzL_store * (int64_t)shift;
  hipLaunchKernelGGL(k_get_diag, dim3((S.n + NT - 1) / NT), dim3(NT), 0, st, Ls,
                     (const int64_t*)(m + S.o_diagoff), S.n, cplx ? 1 : 0, (double2*)out);
  PXS_CHECK_LAUNCH();
  return 0;
}

#include "hermitian.inc"
#include "batch.inc"

}  // namespace pxs
