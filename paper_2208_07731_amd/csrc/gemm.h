// MFMA GEMM engine for gfx950 (wave64).
//
//   acc(m, n) = sum_k A(m, k) B(k, n)      m < M, n < N, k in [kbeg, kend)
//
// Operand layouts (element type TA / TB, converted to the compute type T on
// load):
//   KC: element (x, k) at p[x * ld + k]   (k contiguous: rows of a row-major matrix)
//   XC: element (x, k) at p[k * ld + x]   (x contiguous: columns of a row-major matrix)
// where x = m for A and x = n for B.  A may gather its rows through an index
// array (KC only).  The accumulator tile is handed to an epilogue functor.
//
// Tiling: a BM x BN block tile per workgroup of WM x WN wavefronts, BK-deep
// K steps staged through LDS (k-major, padded), register prefetch of the
// next K step while the current one feeds the MFMAs.  Each wavefront owns a
// (BM/WM) x (BN/WN) sub-tile made of 16x16 MFMA tiles:
//   T = double: v_mfma_f64_16x16x4f64, T = float: v_mfma_f32_16x16x4f32.
// Operand lane layout of both (16x4 A, 4x16 B): lane l holds row/col l%16,
// k = l/16.  Result: lane l holds column l%16 and four rows, j = 0..3:
// rows 4*(l/16) + j for the f32 instruction, rows l/16 + 4*j for the f64 one
// (checked on the hardware).
//
// Block-to-tile mapping is XCD aware: workgroups are dispatched round-robin
// over the 8 XCDs, so consecutive logical tiles (same A row block) are given
// to workgroups of the same XCD and share its L2.
#pragma once

#include "common.h"

namespace isdf {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <class T>
struct MfmaT;
template <>
struct MfmaT<double> {
  typedef d4v acc_t;
  __device__ __forceinline__ static void mma(double a, double b, acc_t& c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaT<float> {
  typedef f4v acc_t;
  __device__ __forceinline__ static void mma(float a, float b, acc_t& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

enum { KC = 0, XC = 1 };

template <class TS>
struct Operand {
  const TS* p;
  int64_t ld;
  const int* rows;  // optional gather of the x index (KC only), may be null
};

struct GemmShape {
  int M, N;
  int64_t K;
  int64_t kchunk;    // split-K: blockIdx.z covers [z*kchunk, min(K, (z+1)*kchunk))
  int lower_only;    // skip tiles strictly above the diagonal
  const int* abort;  // nonzero *abort turns the launch into a no-op
};

__device__ __forceinline__ int xcd_remap(int bid, int total) {
  const int full = (total / 8) * 8;
  if (bid >= full) return bid;
  return (bid % 8) * (total / 8) + bid / 8;
}

template <class T, int BM, int BN, int BK, int WM, int WN>
struct TileCfg {
  static constexpr int THREADS = WM * WN * ISDF_WAVE;
  static constexpr int WTM = BM / WM, WTN = BN / WN;  // wave tile
  static constexpr int MI = WTM / 16, NI = WTN / 16;  // MFMA tiles per wave
  // LDS row padding: a row stride of (BM + 16) elements puts the four
  // 16-lane groups of an MFMA operand read in alternating bank halves.
  static constexpr int PAD = 16;
  static constexpr int LDA = BM + PAD, LDB = BN + PAD;
  static constexpr int A_ELEMS = BM * BK / THREADS;  // per-thread prefetch
  static constexpr int B_ELEMS = BN * BK / THREADS;
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile");
  static_assert(BK % 4 == 0, "bk");
  static_assert((BM * BK) % THREADS == 0 && (BN * BK) % THREADS == 0, "load split");
  // row (within a 16x16 MFMA tile) of accumulator element j of `lane`
  __device__ __forceinline__ static int orow(int lane, int j) {
    return sizeof(T) == 8 ? (lane >> 4) + 4 * j : 4 * (lane >> 4) + j;
  }
};

// Per-thread prefetch of one BK slice of an operand (X rows x BK), in the
// compute type.  KC: thread -> (x, run of E consecutive k); XC: thread ->
// (k, run of E consecutive x).
template <class T, class TS, int LAYOUT, int X, int BK, int THREADS>
struct Stager {
  static constexpr int E = X * BK / THREADS;
  T v[E];
  __device__ __forceinline__ void load(const Operand<TS>& op, int x0, int xlim, int64_t k0, int64_t klim,
                                       int tid, int64_t rowcache) {
    if (LAYOUT == KC) {
      constexpr int RUNS = BK / E;  // threads per x
      const int x = tid / RUNS;
      const int64_t kb = k0 + (tid % RUNS) * E;
      const bool okx = (x0 + x) < xlim;
      const TS* base = op.p + rowcache * op.ld;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t k = kb + e;
        v[e] = (okx && k < klim) ? (T)base[k] : (T)0;
      }
    } else {
      constexpr int RUNS = X / E;  // threads per k
      const int64_t k = k0 + tid / RUNS;
      const int xb = x0 + (tid % RUNS) * E;
      const bool okk = k < klim;
      const TS* base = op.p + k * op.ld;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = xb + e;
        v[e] = (okk && x < xlim) ? (T)base[x] : (T)0;
      }
    }
  }
  // LDS tile s[BK][X + pad]
  __device__ __forceinline__ void store(T* s, int lds_ld, int tid) const {
    if (LAYOUT == KC) {
      constexpr int RUNS = BK / E;
      const int x = tid / RUNS;
      const int kb = (tid % RUNS) * E;
#pragma unroll
      for (int e = 0; e < E; ++e) s[(kb + e) * lds_ld + x] = v[e];
    } else {
      constexpr int RUNS = X / E;
      const int k = tid / RUNS;
      const int xb = (tid % RUNS) * E;
#pragma unroll
      for (int e = 0; e < E; ++e) s[k * lds_ld + xb + e] = v[e];
    }
  }
  // Global row of this thread's x (KC), resolved once per tile.
  __device__ __forceinline__ static int64_t row_of(const Operand<TS>& op, int x0, int xlim, int tid) {
    if (LAYOUT != KC) return 0;
    constexpr int RUNS = BK / E;
    const int x = x0 + tid / RUNS;
    const int xc = x < xlim ? x : (xlim > 0 ? xlim - 1 : 0);
    return op.rows ? (int64_t)op.rows[xc] : (int64_t)xc;
  }
};

// Runs the K loop of one operand pair into acc.
template <class Cfg, class T, class TA, int LA, class TB, int LB, int BM, int BN, int BK>
__device__ __forceinline__ void mma_loop(const Operand<TA>& A, const Operand<TB>& B, int m0, int n0, int M,
                                         int N, int64_t kbeg, int64_t kend, T* As, T* Bs,
                                         typename MfmaT<T>::acc_t (&acc)[Cfg::MI][Cfg::NI]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wm = wv / (BN / Cfg::WTN);
  const int wn = wv % (BN / Cfg::WTN);
  Stager<T, TA, LA, BM, BK, Cfg::THREADS> sa;
  Stager<T, TB, LB, BN, BK, Cfg::THREADS> sb;
  const int64_t rowa = Stager<T, TA, LA, BM, BK, Cfg::THREADS>::row_of(A, m0, M, tid);
  const int64_t rowb = Stager<T, TB, LB, BN, BK, Cfg::THREADS>::row_of(B, n0, N, tid);
  if (kbeg >= kend) return;
  sa.load(A, m0, M, kbeg, kend, tid, rowa);
  sb.load(B, n0, N, kbeg, kend, tid, rowb);
  sa.store(As, Cfg::LDA, tid);
  sb.store(Bs, Cfg::LDB, tid);
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      sa.load(A, m0, M, k0 + BK, kend, tid, rowa);
      sb.load(B, n0, N, k0 + BK, kend, tid, rowb);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[Cfg::MI], b[Cfg::NI];
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i) a[i] = As[kr * Cfg::LDA + wm * Cfg::WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) b[j] = Bs[kr * Cfg::LDB + wn * Cfg::WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) MfmaT<T>::mma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
    if (more) {
      sa.store(As, Cfg::LDA, tid);
      sb.store(Bs, Cfg::LDB, tid);
      __syncthreads();
    }
  }
}

// Tile coordinates handed to epilogues.
struct TileAt {
  int m_wave, n_wave;  // first row / column of this wavefront's sub-tile
  int lane;
  int z;               // split-K index
};

// Generic kernel: NOPS = 1 (one operand pair) or 2 (two pairs into two
// accumulator sets, same tile, e.g. Phi and Psi Gram blocks).
template <class T, int BM, int BN, int BK, int WM, int WN, class TA, int LA, class TB, int LB, int NOPS,
          class Epi>
__global__ __launch_bounds__(WM* WN* ISDF_WAVE) void gemm_kernel(GemmShape sh, Operand<TA> A0, Operand<TB> B0,
                                                                 Operand<TA> A1, Operand<TB> B1, int64_t K1,
                                                                 Epi epi) {
  typedef TileCfg<T, BM, BN, BK, WM, WN> Cfg;
  if (sh.abort && *sh.abort) return;
  __shared__ T As[BK * Cfg::LDA];
  __shared__ T Bs[BK * Cfg::LDB];
  const int tiles_n = (sh.N + BN - 1) / BN;
  const int tiles_m = (sh.M + BM - 1) / BM;
  const int logical = xcd_remap(blockIdx.x, tiles_m * tiles_n);
  const int tm = logical / tiles_n, tn = logical % tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  if (sh.lower_only && n0 > m0 + BM - 1) return;
  const int z = blockIdx.z;
  const int64_t kbeg = (int64_t)z * sh.kchunk;
  const int64_t kend = kbeg + sh.kchunk < sh.K ? kbeg + sh.kchunk : sh.K;

  typename MfmaT<T>::acc_t acc0[Cfg::MI][Cfg::NI];
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j) acc0[i][j] = typename MfmaT<T>::acc_t{0, 0, 0, 0};
  mma_loop<Cfg, T, TA, LA, TB, LB, BM, BN, BK>(A0, B0, m0, n0, sh.M, sh.N, kbeg, kend, As, Bs, acc0);

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int wm = wv / (BN / Cfg::WTN), wn = wv % (BN / Cfg::WTN);
  TileAt at{m0 + wm * Cfg::WTM, n0 + wn * Cfg::WTN, lane, z};
  if constexpr (NOPS == 2) {
    typename MfmaT<T>::acc_t acc1[Cfg::MI][Cfg::NI];
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) acc1[i][j] = typename MfmaT<T>::acc_t{0, 0, 0, 0};
    __syncthreads();
    mma_loop<Cfg, T, TA, LA, TB, LB, BM, BN, BK>(A1, B1, m0, n0, sh.M, sh.N, 0, K1, As, Bs, acc1);
    epi.template apply2<Cfg>(acc0, acc1, at);
  } else {
    epi.template apply<Cfg>(acc0, at);
  }
}

// ------------------------------------------------------------- epilogues
// C(m, n) = alpha * acc + beta * C(m, n), optionally scaled per row by
// rowscale[m] and written into split-K slice z (C + z * zstride).
template <class TC>
struct EpiStore {
  TC* C;
  int64_t ldc;
  int M, N;
  double alpha, beta;
  const double* rowscale;  // may be null
  int64_t zstride;
  template <class Cfg, class Acc>
  __device__ __forceinline__ void apply(const Acc (&acc)[Cfg::MI][Cfg::NI], const TileAt& at) const {
    TC* Cz = C + at.z * zstride;
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) {
        const int n = at.n_wave + j * 16 + (at.lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = at.m_wave + i * 16 + Cfg::orow(at.lane, r);
          if (m < M && n < N) {
            double v = alpha * (double)acc[i][j][r];
            if (rowscale) v *= rowscale[m];
            TC* c = Cz + (int64_t)m * ldc + n;
            if (beta != 0.0) v += beta * (double)(*c);
            *c = (TC)v;
          }
        }
      }
  }
};

}  // namespace isdf
