// Split-precision MFMA GEMM for gfx950: FP64-accurate-enough products from
// 16-bit matrix cores.
//
//   acc(m, n) = sum_k A(m, k) B(k, n), A and B K-contiguous (KC).
//
// The operands are split once, in an HBM pass (split_planes), into planes
// of 16-bit parts; the GEMM then streams the parts straight into LDS:
//
//   BF16X6: x = h + m + l, three bfloat16 parts taken successively from the
//           exact residuals; products h.h | h.m + m.h + h.l + m.m + l.h
//           (the dropped terms are below 2^-24 relative).
//   FP16X3: x s = h + l, two binary16 parts of x scaled by a power of two s
//           (from the operand's largest magnitude, so that no part
//           overflows and few underflow); products h.h | h.l + l.h.
//
// The leading product and the correction products accumulate in separate
// FP32 accumulators (the corrections are 2^-8 or 2^-11 smaller, so their
// rounding stays negligible); the leading accumulator is folded into FP64
// every FLUSH 32-deep slices, so FP32 rounding does not grow with K, and the
// epilogue receives the FP64 sum.
//
// MFMA: v_mfma_f32_16x16x32_bf16 / _f16.  Operand lane layout (checked on
// the hardware): lane l holds row/column l % 16 and k = 8 (l / 16) + e,
// e = 0..7; the result is laid out like the f32 16x16x4 instruction.
#pragma once

#include "gemm.h"

namespace isdf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

enum { SPLIT_BF16X6 = 0, SPLIT_FP16X3 = 1 };

template <int MODE>
struct SplitT;
template <>
struct SplitT<SPLIT_BF16X6> {
  typedef __bf16 P;
  typedef bf16x8 V;
  static constexpr int NP = 3;
  static constexpr int NPROD = 6;
  __device__ __forceinline__ static int pa(int p) { return p == 0 ? 0 : p == 1 ? 0 : p == 2 ? 1 : p == 3 ? 0 : p == 4 ? 1 : 2; }
  __device__ __forceinline__ static int pb(int p) { return p == 0 ? 0 : p == 1 ? 1 : p == 2 ? 0 : p == 3 ? 2 : p == 4 ? 1 : 0; }
  __device__ __forceinline__ static void split(double x, double, P (&o)[NP]) {
    const P h = (P)(float)x;
    const double r1 = x - (double)(float)h;
    const P m = (P)(float)r1;
    const double r2 = r1 - (double)(float)m;
    o[0] = h;
    o[1] = m;
    o[2] = (P)(float)r2;
  }
  __device__ __forceinline__ static void mma(const V& a, const V& b, f4v& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct SplitT<SPLIT_FP16X3> {
  typedef _Float16 P;
  typedef f16x8 V;
  static constexpr int NP = 2;
  static constexpr int NPROD = 3;
  __device__ __forceinline__ static int pa(int p) { return p == 2 ? 1 : 0; }
  __device__ __forceinline__ static int pb(int p) { return p == 1 ? 1 : 0; }
  __device__ __forceinline__ static void split(double x, double s, P (&o)[NP]) {
    const double y = x * s;
    const P h = (P)y;
    o[0] = h;
    o[1] = (P)(y - (double)h);
  }
  __device__ __forceinline__ static void mma(const V& a, const V& b, f4v& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <int BM, int BN, int WM, int WN>
struct SplitCfg {
  static constexpr int THREADS = WM * WN * ISDF_WAVE;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int MI = WTM / 16, NI = WTN / 16;
  static constexpr int BK = 32;
  // LDS row of one part: 32 16-bit elements (64 bytes, unpadded); the four
  // 16-byte chunks of a row are stored at chunk ^ swz(row), see lds_chunk
  static constexpr int LDK = BK;
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile");
  __device__ __forceinline__ static int orow(int lane, int j) { return 4 * (lane >> 4) + j; }
};

// An operand already split into NP planes of 16-bit parts: part q of
// element (x, k) at p[q * pstride + row(x) * ld + k]; ld and the K extent
// are multiples of 32 (zero-padded), so K needs no guard.
template <class P>
struct PlaneOp {
  const P* p;
  int64_t ld;
  int64_t pstride;
  const int* rows;  // optional gather of x, may be null
};

// LDS position of 16-byte chunk c (0..3) of staged row r.  LDS serves 32
// lanes of a 16-byte access per cycle from 128 four-byte banks: a fragment
// read (16 consecutive rows, chunks 2h and 2h + 1 for lane groups h) and a
// staging store (8 consecutive rows from a multiple of 8, all four chunks)
// then hit 32 distinct 16-byte slots when rows 8..15 of every 16 swap chunk
// pairs (0,1) <-> (2,3).
__device__ __forceinline__ int lds_chunk(int r, int c) { return c ^ ((r >> 2) & 2); }

// Stages one stage of SUB 32-deep slices of a plane operand: the
// NP x X x 4 16-byte chunks of a slice are spread over the workgroup (the
// same chunks of every slice for one thread) and copied to LDS
// [SUB][NP][X][LDK].
template <int MODE, int X, int THREADS, int SUB>
struct PlaneStager {
  typedef SplitT<MODE> S;
  typedef typename S::V V;
  static constexpr int CHUNKS = S::NP * X * 4;
  static constexpr int PER = (CHUNKS + THREADS - 1) / THREADS;
  static_assert(X % 16 == 0, "rows of a stage");
  V v[SUB][PER];
  int64_t off[PER];  // element offset of each chunk's row start (without k)
  __device__ __forceinline__ void init(const PlaneOp<typename S::P>& op, int x0, int xlim, int tid) {
#pragma unroll
    for (int c = 0; c < PER; ++c) {
      const int id = tid + c * THREADS;
      const int q = id / (X * 4), rem = id % (X * 4), x = rem / 4;
      int xr = x0 + x;
      xr = xr < xlim ? xr : (xlim > 0 ? xlim - 1 : 0);  // rows past the edge: any valid row
      const int64_t row = op.rows ? (int64_t)op.rows[xr] : (int64_t)xr;
      off[c] = q * op.pstride + row * op.ld + 8 * (rem % 4);
    }
  }
  // slices k0, k0 + 32, ... of the first nsub of the stage
  __device__ __forceinline__ void load(const PlaneOp<typename S::P>& op, int64_t k0, int nsub, int tid) {
#pragma unroll
    for (int u = 0; u < SUB; ++u)
      if (u == 0 || u < nsub)
#pragma unroll
        for (int c = 0; c < PER; ++c)
          if (CHUNKS % THREADS == 0 || tid + c * THREADS < CHUNKS)
            v[u][c] = *reinterpret_cast<const V*>(op.p + off[c] + k0 + 32 * u);
  }
  __device__ __forceinline__ void store(typename S::P* s, int lds_k, int nsub, int tid) const {
#pragma unroll
    for (int u = 0; u < SUB; ++u)
      if (u == 0 || u < nsub)
#pragma unroll
        for (int c = 0; c < PER; ++c) {
          const int id = tid + c * THREADS;
          if (CHUNKS % THREADS == 0 || id < CHUNKS) {
            const int q = id / (X * 4), rem = id % (X * 4);
            const int r = q * X + rem / 4;
            *reinterpret_cast<V*>(s + (u * S::NP * X + r) * lds_k + 8 * lds_chunk(r, rem % 4)) = v[u][c];
          }
        }
  }
};

// Leading-product accumulator folded into FP64 every FLUSH 32-deep slices:
// FP32 then sums at most 32 FLUSH products per output before a rounding that
// grows with K can build up.
template <class Cfg>
__device__ __forceinline__ void flush_acc(f4v (&acc)[Cfg::MI][Cfg::NI], d4v (&accd)[Cfg::MI][Cfg::NI]) {
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) accd[i][j][r] += (double)acc[i][j][r];
      acc[i][j] = f4v{0, 0, 0, 0};
    }
}

// Number of 32-deep slices per LDS stage: two where the registers allow a
// second staged slice (two 16-bit parts), one otherwise.
template <int MODE, int THREADS>
struct SplitSub {
  static constexpr int value = SplitT<MODE>::NP == 2 ? 2 : 1;
};

// LDS buffers of stages: with two, the next stage is stored into the other
// buffer while this one feeds the MFMAs and one barrier per stage suffices.
// The eight-wavefront tiles run one workgroup per CU, so their LDS has room
// for two (FP16x3 128 KB, BF16x6 96 KB); a barrier there stalls every wave
// of the CU, not one workgroup of two.
template <int MODE, int THREADS>
struct SplitBufs {
  static constexpr int value = THREADS >= 512 ? 2 : 1;
};

// K loop of one operand pair into the leading (acc0, folded into accd every
// FLUSH slices) and correction (acc1) accumulators.  LDS stages of SUB
// slices (one or two buffers, SplitBufs), the next stage prefetched in
// registers; the products and the fold points are those of a loop over
// single slices, so neither SUB nor the buffering changes a bit of the
// result.
template <int MODE, class Cfg, int BM, int BN, int FLUSH>
__device__ __forceinline__ void split_loop(const PlaneOp<typename SplitT<MODE>::P>& A,
                                           const PlaneOp<typename SplitT<MODE>::P>& B, int m0, int n0, int M, int N,
                                           int64_t kbeg, int64_t K, typename SplitT<MODE>::P* smem,
                                           f4v (&acc0)[Cfg::MI][Cfg::NI], f4v (&acc1)[Cfg::MI][Cfg::NI],
                                           d4v (&accd)[Cfg::MI][Cfg::NI]) {
  typedef SplitT<MODE> S;
  typedef typename S::P P;
  typedef typename S::V V;
  constexpr int LDK = Cfg::LDK;
  constexpr int SUB = SplitSub<MODE, Cfg::THREADS>::value;
  constexpr int NBUF = SplitBufs<MODE, Cfg::THREADS>::value;
  constexpr int BK = Cfg::BK;
  constexpr int STAGE = SUB * S::NP * (BM + BN) * LDK;
  P* As = smem;
  P* Bs = smem + SUB * S::NP * BM * LDK;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / (BN / Cfg::WTN), wn = wv % (BN / Cfg::WTN);
  PlaneStager<MODE, BM, Cfg::THREADS, SUB> sa;
  PlaneStager<MODE, BN, Cfg::THREADS, SUB> sb;
  sa.init(A, m0, M, tid);
  sb.init(B, n0, N, tid);
  if (K <= kbeg) return;
  // K - kbeg is a multiple of BK: slices in a stage starting at k
  auto nsub_at = [&](int64_t k) { return (int)((K - k) / BK < SUB ? (K - k) / BK : SUB); };
  sa.load(A, kbeg, nsub_at(kbeg), tid);
  sb.load(B, kbeg, nsub_at(kbeg), tid);
  sa.store(As, LDK, nsub_at(kbeg), tid);
  sb.store(Bs, LDK, nsub_at(kbeg), tid);
  __syncthreads();
  // fragment rows are 16-aligned plus lane & 15, so the swizzle depends on the lane only
  const int q8 = 8 * lds_chunk(lane & 15, lane >> 4);
  int step = 0;
  for (int64_t k0 = kbeg; k0 < K; k0 += SUB * BK) {
    const int64_t kn = k0 + SUB * BK;
    const bool more = kn < K;
    const int nn = more ? nsub_at(kn) : 0, nc = nsub_at(k0);
    if (more) {
      sa.load(A, kn, nn, tid);
      sb.load(B, kn, nn, tid);
    }
#pragma unroll
    for (int u = 0; u < SUB; ++u) {
      if (u > 0 && u >= nc) break;
      const P* Au = As + u * S::NP * BM * LDK;
      const P* Bu = Bs + u * S::NP * BN * LDK;
      V a[S::NP][Cfg::MI], b[S::NP][Cfg::NI];
#pragma unroll
      for (int p = 0; p < S::NP; ++p) {
#pragma unroll
        for (int i = 0; i < Cfg::MI; ++i)
          a[p][i] = *reinterpret_cast<const V*>(Au + (p * BM + wm * Cfg::WTM + i * 16 + (lane & 15)) * LDK + q8);
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j)
          b[p][j] = *reinterpret_cast<const V*>(Bu + (p * BN + wn * Cfg::WTN + j * 16 + (lane & 15)) * LDK + q8);
      }
      // leading products first: the fold below reads acc0 while the
      // correction products still run on the matrix cores
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) S::mma(a[0][i], b[0][j], acc0[i][j]);
#pragma unroll
      for (int pp = 1; pp < S::NPROD; ++pp)
#pragma unroll
        for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
          for (int j = 0; j < Cfg::NI; ++j) S::mma(a[S::pa(pp)][i], b[S::pb(pp)][j], acc1[i][j]);
      if (++step == FLUSH) {
        step = 0;
        flush_acc<Cfg>(acc0, accd);
      }
    }
    if constexpr (NBUF == 2) {
      // the other buffer's last reads ended before the previous barrier
      P* An = (As == smem) ? smem + STAGE : smem;
      if (more) {
        sa.store(An, LDK, nn, tid);
        sb.store(An + SUB * S::NP * BM * LDK, LDK, nn, tid);
      }
      __syncthreads();
      As = An;
      Bs = An + SUB * S::NP * BM * LDK;
    } else {
      __syncthreads();
      if (more) {
        sa.store(As, LDK, nn, tid);
        sb.store(Bs, LDK, nn, tid);
        __syncthreads();
      }
    }
  }
  flush_acc<Cfg>(acc0, accd);
}

// Split of rows of an r-major complex matrix (or a real matrix read as
// one) into planes [NP][rows][ldp] of 16-bit parts; columns 2n .. ldp-1 are
// zero.  `gather` (optional) lists the source rows; scale (optional, device)
// multiplies before the split (binary16).
template <int MODE, class TS>
__global__ void split_planes(const TS* __restrict__ x, int64_t ld, int n, const int* __restrict__ gather,
                             int64_t nr_src, int64_t r0, int rows, typename SplitT<MODE>::P* __restrict__ out,
                             int ldp, int64_t pstride, const double* scale) {
  typedef SplitT<MODE> S;
  const double s = scale ? *scale : 1.0;
  const int cpr = ldp / 8;  // 8-element chunks per row
  const int64_t total = (int64_t)rows * cpr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cpr), k0 = 8 * (int)(e % cpr);
    int64_t src = gather ? (int64_t)gather[r] : r0 + r;
    if (src < 0 || src >= nr_src) src = 0;  // invalid gathers are reported elsewhere
    const TS* row = x + 2 * src * ld;
    typename S::V w[S::NP];
#pragma unroll
    for (int e8 = 0; e8 < 8; ++e8) {
      const int k = k0 + e8;
      const double v = k < 2 * n ? (double)row[k] : 0.0;
      typename S::P o[S::NP];
      S::split(v, s, o);
#pragma unroll
      for (int q = 0; q < S::NP; ++q) w[q][e8] = o[q];
    }
#pragma unroll
    for (int q = 0; q < S::NP; ++q)
      *reinterpret_cast<typename S::V*>(out + q * pstride + (int64_t)r * ldp + k0) = w[q];
  }
}

// Transposed split: planes [NP][ncols][ldk] of the 16-bit parts of the
// columns of an r-major block, x(c, k) = X[k ld + c] (times rowscale[k] when
// given), k < rows, and zero for rows <= k < ldk: the grid rows become the
// contiguous K index of a product contracted over them (X^T Y).  One tile
// of 64 rows x 64 columns per workgroup, transposed through LDS; scale as in
// split_planes.  The same pass can write a second set of planes into out2
// (row pitch ld2, plane stride pstride2, binary16 scale scale2):
//   SECOND = T_DUAL: the transposed planes of X without the row scale, for
//     X^T diag(g) X from one read of X;
//   SECOND = T_ROWS: the row planes of X as split_planes writes them (columns
//     ncols .. ld2-1 zero, rows < `rows`), for a product over X's columns
//     (X F) and one over its rows (X^T Y) from one read of X.
enum { T_ONE = 0, T_DUAL = 1, T_ROWS = 2 };
template <int MODE, class TS, int SECOND>
__global__ __launch_bounds__(256) void split_planes_t(const TS* __restrict__ X, int64_t ld, int ncols, int rows,
                                                      const double* __restrict__ rowscale,
                                                      typename SplitT<MODE>::P* __restrict__ out, int ldk,
                                                      int64_t pstride, const double* scale,
                                                      typename SplitT<MODE>::P* __restrict__ out2, int ld2,
                                                      int64_t pstride2, const double* scale2) {
  typedef SplitT<MODE> S;
  constexpr bool DUAL = SECOND == T_DUAL;
  __shared__ double tile[64][65];
  __shared__ double fk[64];  // DUAL: row scales of the tile (0 past the last row)
  const double sc = scale ? *scale : 1.0;
  const double sc2 = (SECOND != T_ONE && scale2) ? *scale2 : 1.0;
  const int k0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  // all 16 loads of a thread (and its row scales) in flight before any LDS
  // write: indices past the last row or column are clamped to it, so every
  // address is inside X, and those elements are zeroed afterwards; an empty
  // X (no rows or columns) only zeroes the tile
  if (rows > 0 && ncols > 0) {
    const int c = c0 + tx, cc = c < ncols ? c : ncols - 1;
    double v[16], f[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int k = k0 + ty + 4 * t, kc = k < rows ? k : rows - 1;
      v[t] = (double)X[(int64_t)kc * ld + cc];
    }
    if (rowscale) {
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int k = k0 + ty + 4 * t;
        f[t] = rowscale[k < rows ? k : rows - 1];
      }
    } else {
#pragma unroll
      for (int t = 0; t < 16; ++t) f[t] = 1.0;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int k = k0 + ty + 4 * t;
      // the product with 1.0 is exact, so rows without a scale keep their
      // value; DUAL keeps X in the tile and applies the row scale when the
      // scaled planes are written (the same product)
      if (DUAL) {
        tile[ty + 4 * t][tx] = (k < rows && c < ncols) ? v[t] : 0.0;
        if (tx == 0) fk[ty + 4 * t] = k < rows ? f[t] : 0.0;
      } else {
        tile[ty + 4 * t][tx] = (k < rows && c < ncols) ? v[t] * f[t] : 0.0;
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      tile[ty + 4 * t][tx] = 0.0;
      if (DUAL && tx == 0) fk[ty + 4 * t] = 0.0;
    }
  }
  __syncthreads();
  // 64 columns x 8 runs of 8 consecutive k, two per thread
  for (int q = threadIdx.x; q < 512; q += 256) {
    const int cc = q >> 3, run = q & 7;
    const int c = c0 + cc, kb = k0 + 8 * run;
    if (c >= ncols || kb >= ldk) continue;
    typename S::V w[S::NP];
#pragma unroll
    for (int e8 = 0; e8 < 8; ++e8) {
      typename S::P o[S::NP];
      const double x = tile[8 * run + e8][cc];
      if (DUAL) {
        // the row-scaled value rounded on its own, as the single-output pass
        // stores it (no contraction of the product into the split's
        // subtractions)
#pragma clang fp contract(off)
        S::split(x * fk[8 * run + e8], sc, o);
      } else {
        S::split(x, sc, o);
      }
#pragma unroll
      for (int p = 0; p < S::NP; ++p) w[p][e8] = o[p];
    }
#pragma unroll
    for (int p = 0; p < S::NP; ++p)
      *reinterpret_cast<typename S::V*>(out + p * pstride + (int64_t)c * ldk + kb) = w[p];
    if (DUAL) {
#pragma unroll
      for (int e8 = 0; e8 < 8; ++e8) {
        typename S::P o[S::NP];
        S::split(tile[8 * run + e8][cc], sc2, o);
#pragma unroll
        for (int p = 0; p < S::NP; ++p) w[p][e8] = o[p];
      }
#pragma unroll
      for (int p = 0; p < S::NP; ++p)
        *reinterpret_cast<typename S::V*>(out2 + p * pstride2 + (int64_t)c * ld2 + kb) = w[p];
    }
  }
  if (SECOND == T_ROWS) {
    // 64 rows x 8 runs of 8 consecutive columns, two per thread; ld2 is a
    // multiple of 8 no larger than the column tiles' extent, so a run that
    // starts inside a row ends inside it, and its columns past ncols are the
    // tile's zeros
    for (int q = threadIdx.x; q < 512; q += 256) {
      const int kk = q >> 3, run = q & 7;
      const int k = k0 + kk, cb = c0 + 8 * run;
      if (k >= rows || cb >= ld2) continue;
      typename S::V w[S::NP];
#pragma unroll
      for (int e8 = 0; e8 < 8; ++e8) {
        typename S::P o[S::NP];
        S::split(tile[kk][8 * run + e8], sc2, o);
#pragma unroll
        for (int p = 0; p < S::NP; ++p) w[p][e8] = o[p];
      }
#pragma unroll
      for (int p = 0; p < S::NP; ++p)
        *reinterpret_cast<typename S::V*>(out2 + p * pstride2 + (int64_t)k * ld2 + cb) = w[p];
    }
  }
}

// Power-of-two operand scales for the FP16 split, from device magnitudes:
// scales[2 i] = 2^e with max |x| 2^e <= 2^14 (1 if the operand is zero).
__device__ __forceinline__ double pow2_scale_for(double amax) {
  if (!(amax > 0.0) || !(amax < INFINITY)) return 1.0;
  int e;
  frexp(amax, &e);  // amax in [2^(e-1), 2^e)
  return ldexp(1.0, 14 - e);
}

// Tiles of a split-engine launch: all of them, or (lower_only, M = N, BM a
// multiple q of BN) those that reach the lower triangle: q (tm + 1) in row
// block tm, capped at tiles_n in the last one.
__host__ __device__ __forceinline__ int64_t split_tiles(int tiles_m, int tiles_n, int q, int lower_only) {
  if (!lower_only) return (int64_t)tiles_m * tiles_n;
  const int64_t last = (int64_t)q * tiles_m < tiles_n ? (int64_t)q * tiles_m : tiles_n;
  return (int64_t)q * (tiles_m - 1) * tiles_m / 2 + last;
}

// NOPS = 1 or 2 operand pairs (two pairs: two accumulator sets, e.g. the
// Gram blocks of Phi and Psi for the same tile).  With sh.splits > 1 (one
// operand pair only) the grid holds sh.splits groups of tiles, group z
// summing K slice [z kchunk, (z + 1) kchunk) and handing z to the epilogue.  scales: null (BF16X6) or
// device [s_A0, s_B0, s_A1, s_B1] the planes were scaled by (FP16X3).
template <int MODE, int BM, int BN, int WM, int WN, int NOPS, int FLUSH, class Epi>
__global__ __launch_bounds__(WM* WN* ISDF_WAVE, WM* WN >= 8 ? 1 : 2) void gemm_split_kernel(
    GemmShape sh, PlaneOp<typename SplitT<MODE>::P> A0, PlaneOp<typename SplitT<MODE>::P> B0,
    PlaneOp<typename SplitT<MODE>::P> A1, PlaneOp<typename SplitT<MODE>::P> B1, int64_t K1, const double* scales,
    Epi epi) {
  typedef SplitCfg<BM, BN, WM, WN> Cfg;
  typedef SplitT<MODE> S;
  if (sh.abort && *sh.abort) return;
  __shared__ __attribute__((aligned(16))) typename S::P smem[SplitBufs<MODE, Cfg::THREADS>::value * SplitSub<MODE, Cfg::THREADS>::value * S::NP * (BM + BN) *
                                                              Cfg::LDK];
  const int tiles_n = (sh.N + BN - 1) / BN, tiles_m = (sh.M + BM - 1) / BM;
  const int ntiles = (int)split_tiles(tiles_m, tiles_n, BM / BN, sh.lower_only);
  // split-K: slice z of the K range per group of ntiles workgroups
  const int z = blockIdx.x / ntiles;
  const int logical = xcd_remap(blockIdx.x % ntiles, ntiles);
  const int64_t kbeg = (int64_t)z * sh.kchunk;
  const int64_t kend = kbeg + sh.kchunk < sh.K ? kbeg + sh.kchunk : sh.K;
  int tm, tn;
  if (sh.lower_only) {
    // row block tm holds the q (tm + 1) column tiles that reach its last row
    // (q = BM / BN): logical = q tm (tm + 1) / 2 + tn
    constexpr int q = BM / BN;
    tm = (int)((sqrt(1.0 + 8.0 * logical / q) - 1.0) * 0.5);
    while (tm > 0 && (int64_t)q * tm * (tm + 1) / 2 > logical) --tm;
    while (tm + 1 < tiles_m && (int64_t)q * (tm + 1) * (tm + 2) / 2 <= logical) ++tm;
    tn = logical - q * tm * (tm + 1) / 2;
  } else {
    // column by column within groups of 4 row blocks: the tiles one XCD
    // holds at a time (about 32, consecutive logical tiles) then span 4 row
    // and 8 column blocks rather than 1 row and 32 column blocks, so fewer
    // operand slices go through its L2 per K step (Z C^H Gram 7 %, Abar^T Phi
    // 5 % faster at 512-water blocks; 8 row blocks no better)
    constexpr int GR = 4;
    const int first = (logical / (GR * tiles_n)) * GR;
    const int rows_in = tiles_m - first < GR ? tiles_m - first : GR;
    const int local = logical % (GR * tiles_n);
    tm = first + local % rows_in;
    tn = local / rows_in;
  }
  const int m0 = tm * BM, n0 = tn * BN;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv / (BN / Cfg::WTN), wn = wv % (BN / Cfg::WTN);
  TileAt at{m0 + wm * Cfg::WTM, n0 + wn * Cfg::WTN, lane, z, 0};
  double u0 = 1.0, u1 = 1.0;
  if (scales) {
    u0 = 1.0 / (scales[0] * scales[1]);
    u1 = 1.0 / (scales[2] * scales[3]);
  }
  f4v c0[Cfg::MI][Cfg::NI], c1[Cfg::MI][Cfg::NI];
  d4v r0[Cfg::MI][Cfg::NI];
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j) {
      c0[i][j] = c1[i][j] = f4v{0, 0, 0, 0};
      r0[i][j] = d4v{0, 0, 0, 0};
    }
  split_loop<MODE, Cfg, BM, BN, FLUSH>(A0, B0, m0, n0, sh.M, sh.N, kbeg, kend, smem, c0, c1, r0);
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) r0[i][j][r] = (r0[i][j][r] + (double)c1[i][j][r]) * u0;
  if constexpr (NOPS == 2) {
    d4v r1[Cfg::MI][Cfg::NI];
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) {
        c0[i][j] = c1[i][j] = f4v{0, 0, 0, 0};
        r1[i][j] = d4v{0, 0, 0, 0};
      }
    __syncthreads();
    split_loop<MODE, Cfg, BM, BN, FLUSH>(A1, B1, m0, n0, sh.M, sh.N, 0, K1, smem, c0, c1, r1);
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) r1[i][j][r] = (r1[i][j][r] + (double)c1[i][j][r]) * u1;
    epi.template apply2<Cfg>(r0, r1, at);
  } else {
    epi.template apply<Cfg>(r0, at);
  }
}

}  // namespace isdf
