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
// K steps staged through LDS (double buffered, padded), register prefetch of
// the K step after next, and a software-pipelined step (fragment reads,
// stores and the barrier placed between pairs of MFMA sub-steps).  Each wavefront owns a
// (BM/WM) x (BN/WN) sub-tile made of 16x16 MFMA tiles:
//   T = double: v_mfma_f64_16x16x4f64, T = float: v_mfma_f32_16x16x4f32.
// Operand lane layout of both (16x4 A, 4x16 B): lane l holds row/col l%16,
// k = l/16.  Result: lane l holds column l%16 and four rows, j = 0..3:
// rows 4*(l/16) + j for the f32 instruction, rows l/16 + 4*j for the f64 one
// (checked on the hardware).
//
// Block-to-tile mapping is XCD aware: workgroups are dispatched round-robin
// over the 8 XCDs, so consecutive logical tiles are given to workgroups of
// the same XCD and share its L2; logical tiles run down groups of 8 row
// blocks, column by column, so the ~64 workgroups resident on one XCD cover
// about 8 row blocks x 8 column blocks of the output rather than 4 x 16.
//
// Each wave raises its issue priority while it issues a pair's MFMAs
// (s_setprio).  With two waves per SIMD from two workgroups, the raised
// priority lets one finish its MFMAs first and staggers the two, so that
// one is less often waiting at its barrier or LDS stores while the other
// does too (about 3 % on the large FP64 products; an epilogue type can opt
// out, see EpiPrio).
#pragma once

#include <type_traits>

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
  const int* rows;       // optional gather of the x index (KC only), may be null
  const double* kscale;  // optional per-k factor: element (x, k) * kscale[k], may be null
};

struct GemmShape {
  int M, N;
  int64_t K;
  int64_t kchunk;    // split-K slice z covers [z*kchunk, min(K, (z+1)*kchunk))
  int splits;        // number of K slices (grid = tiles x splits, one dimension)
  int lower_only;    // only tiles on or below the diagonal (M == N)
  const int* abort;  // nonzero *abort turns the launch into a no-op
  int64_t sa, sb;    // batch strides of A and B (elements); batch index = blockIdx.y
};

// Number of tiles a launch enumerates.
__host__ __device__ __forceinline__ int64_t gemm_tiles(int tiles_m, int tiles_n, int lower_only) {
  return lower_only ? (int64_t)tiles_m * (tiles_m + 1) / 2 : (int64_t)tiles_m * tiles_n;
}

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
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile");
  static_assert(BK % 16 == 0, "bk");
  static_assert((BM * BK) % THREADS == 0 && (BN * BK) % THREADS == 0, "load split");
  // row (within a 16x16 MFMA tile) of accumulator element j of `lane`
  __device__ __forceinline__ static int orow(int lane, int j) {
    return sizeof(T) == 8 ? (lane >> 4) + 4 * j : 4 * (lane >> 4) + j;
  }
};

// LDS image of one BK slice of an operand (X x BK elements of T):
//   KC: [X][BK + PK] -- k contiguous, as loaded from a KC operand
//   XC: [BK][X + PX] -- x contiguous, as loaded from an XC operand
// Both are read with the same k order: in MFMA sub-step s of a 16-deep
// chunk c, lane group q = lane / 16 supplies k = 16 c + 4 q + s for A and B
// alike, so a KC lane reads four consecutive k with one vector load.
template <class T, int LAYOUT, int X, int BK>
struct Lds {
  static constexpr int PK = 16 / (int)sizeof(T);  // 16-byte pad per row
  // XC rows padded by 4 elements: the four lane groups of a read (rows 4
  // apart) then start 32 (FP64) or 16 (FP32) banks apart
  static constexpr int PX = 4;
  static constexpr int SIZE = LAYOUT == KC ? X * (BK + PK) : BK * (X + PX);
  __device__ __forceinline__ static int at(int x, int k) {
    return LAYOUT == KC ? x * (BK + PK) + k : k * (X + PX) + x;
  }
};

template <class TS>
__device__ __forceinline__ void load_pair(const TS* p, double& a, double& b);
template <>
__device__ __forceinline__ void load_pair<double>(const double* p, double& a, double& b) {
  double2 v = *reinterpret_cast<const double2*>(p);
  a = v.x;
  b = v.y;
}
template <>
__device__ __forceinline__ void load_pair<float>(const float* p, double& a, double& b) {
  float2 v = *reinterpret_cast<const float2*>(p);
  a = v.x;
  b = v.y;
}

// Per-thread prefetch of one BK slice of an operand (X rows x BK), in the
// compute type.  KC: thread -> (x, run of E consecutive k); XC: thread ->
// (k, E / 2 pairs of consecutive x), consecutive threads on consecutive
// pairs.  Interior slices of aligned operands use
// unguarded pair loads; edge slices guard every element.
template <class T, class TS, int LAYOUT, int X, int BK, int THREADS>
struct Stager {
  static constexpr int E = X * BK / THREADS;
  static_assert(E % 2 == 0, "pairs");
  T v[E];
  double fk;  // XC: scale of this thread's k row (1 without scales)
  __device__ __forceinline__ void load(const Operand<TS>& op, int x0, int xlim, int64_t k0, int64_t klim, int tid,
                                       int64_t rowcache, bool aligned) {
    const bool interior = aligned && (x0 + X <= xlim) && (k0 + BK <= klim);
    if (LAYOUT == KC) {
      constexpr int RUNS = BK / E;  // threads per x
      const int x = tid / RUNS;
      const int64_t kb = k0 + (tid % RUNS) * E;
      const TS* base = op.p + rowcache * op.ld + kb;
      if (interior) {
#pragma unroll
        for (int e = 0; e < E; e += 2) {
          double a, b;
          load_pair<TS>(base + e, a, b);
          if (op.kscale) {
            a *= op.kscale[kb + e];
            b *= op.kscale[kb + e + 1];
          }
          v[e] = (T)a;
          v[e + 1] = (T)b;
        }
      } else {
        const bool okx = (x0 + x) < xlim;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const bool ok = okx && kb + e < klim;
          const double f = (ok && op.kscale) ? op.kscale[kb + e] : 1.0;
          v[e] = ok ? (T)(base[e] * f) : (T)0;
        }
      }
    } else {
      // RUNS threads per k row; pair c of a thread sits 2 RUNS elements to
      // the right of pair c - 1, so consecutive lanes take consecutive x
      // pairs and a wave instruction reads whole cache lines
      constexpr int RUNS = X / E;
      const int64_t k = k0 + tid / RUNS;
      const int xb = x0 + 2 * (tid % RUNS);
      const TS* base = op.p + k * op.ld + xb;
      // the row scale is applied when the slice is stored, so that nothing
      // waits for these loads before then (elements outside the operand are
      // zero, so a clamped row index is enough for theirs)
      fk = 1.0;
      if (op.kscale) fk = op.kscale[k < klim ? k : klim - 1];
      if (interior) {
#pragma unroll
        for (int c = 0; c < E / 2; ++c) {
          double a, b;
          load_pair<TS>(base + 2 * RUNS * c, a, b);
          v[2 * c] = (T)a;
          v[2 * c + 1] = (T)b;
        }
      } else {
        const bool okk = k < klim;
#pragma unroll
        for (int c = 0; c < E / 2; ++c) {
          const int x = xb + 2 * RUNS * c;
          v[2 * c] = (okk && x < xlim) ? (T)base[2 * RUNS * c] : (T)0;
          v[2 * c + 1] = (okk && x + 1 < xlim) ? (T)base[2 * RUNS * c + 1] : (T)0;
        }
      }
    }
  }
  __device__ __forceinline__ void store(T* s, int tid) const {
    typedef Lds<T, LAYOUT, X, BK> L;
    if (LAYOUT == KC) {
      constexpr int RUNS = BK / E;
      T* d = s + L::at(tid / RUNS, (tid % RUNS) * E);
#pragma unroll
      for (int e = 0; e < E; ++e) d[e] = v[e];
    } else {
      constexpr int RUNS = X / E;
      T* d = s + L::at(2 * (tid % RUNS), tid / RUNS);
#pragma unroll
      for (int c = 0; c < E / 2; ++c) {
        d[2 * RUNS * c] = (T)(v[2 * c] * fk);
        d[2 * RUNS * c + 1] = (T)(v[2 * c + 1] * fk);
      }
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
  __device__ __forceinline__ static bool aligned(const Operand<TS>& op) {
    return (op.ld % 2 == 0) && (((uintptr_t)op.p) % (2 * sizeof(TS)) == 0);
  }
};

// Operand values of lane `lane` for the four sub-steps of chunk c: element
// (x, 16 c + 4 (lane / 16) + s), s = 0..3.
template <class T, int LAYOUT, int X, int BK>
__device__ __forceinline__ void read4(const T* s, int x, int c, int lane, T (&o)[4]) {
  typedef Lds<T, LAYOUT, X, BK> L;
  const int k = 16 * c + 4 * (lane >> 4);
  if (LAYOUT == KC) {
    const T* p = s + L::at(x, k);
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = p[j];
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = s[L::at(x, k + j)];
  }
}

// FP64 accumulator set of a tile (the target of folded FP32 accumulators).
template <class Cfg>
struct FoldAcc {
  d4v v[Cfg::MI][Cfg::NI];
};

template <class Cfg, class A>
__device__ __forceinline__ void fold_into(A (&acc)[Cfg::MI][Cfg::NI], FoldAcc<Cfg>& f) {
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) f.v[i][j][r] += (double)acc[i][j][r];
      acc[i][j] = A{0, 0, 0, 0};
    }
}

// Operand values of lane `lane` for sub-steps s0 and s0 + 1 of chunk c:
// elements (x, 16 c + 4 (lane / 16) + s0 + t), t = 0, 1.
template <class T, int LAYOUT, int X, int BK>
__device__ __forceinline__ void read2(const T* s, int x, int c, int s0, int lane, T (&o)[2]) {
  typedef Lds<T, LAYOUT, X, BK> L;
  const int k = 16 * c + 4 * (lane >> 4) + s0;
  if (LAYOUT == KC) {
    const T* p = s + L::at(x, k);
    o[0] = p[0];
    o[1] = p[1];
  } else {
    o[0] = s[L::at(x, k)];
    o[1] = s[L::at(x, k + 1)];
  }
}

// Runs the K loop of one operand pair into acc, software pipelined so that
// LDS traffic, global loads and the barrier overlap the MFMAs.  Per step i
// (one BK slice, its MFMA sub-steps taken in pairs):
//   * the fragments of the next pair are read while the current pair's
//     MFMAs issue;
//   * after the first pair(s), slice i+1 (loaded into registers during step
//     i-1) is stored into the other LDS buffer and the global loads of slice
//     i+2 are issued, so every load has a whole step to arrive;
//   * the one barrier per step sits before the last pair, whose MFMAs cover
//     the reads of slice i+1's first pair from the other buffer.
// The order of the products into every accumulator is the plain k order,
// as in mma_loop_flat.
template <class Cfg, class T, class TA, int LA, class TB, int LB, int BM, int BN, int BK, int FOLD = 0,
          bool PRIO = true>
__device__ __forceinline__ void mma_loop_pp(const Operand<TA>& A, const Operand<TB>& B, int m0, int n0, int M,
                                            int N, int64_t kbeg, int64_t kend, T* smem,
                                            typename MfmaT<T>::acc_t (&acc)[Cfg::MI][Cfg::NI],
                                            FoldAcc<Cfg>* fold = nullptr) {
  typedef Lds<T, LA, BM, BK> LA_;
  typedef Lds<T, LB, BN, BK> LB_;
  constexpr int STAGE = LA_::SIZE + LB_::SIZE;
  constexpr int NPAIR = BK / 8;  // pairs of MFMA sub-steps per slice
  static_assert(NPAIR % 2 == 0, "pairs");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wm = wv / (BN / Cfg::WTN);
  const int wn = wv % (BN / Cfg::WTN);
  typedef Stager<T, TA, LA, BM, BK, Cfg::THREADS> SA;
  typedef Stager<T, TB, LB, BN, BK, Cfg::THREADS> SB;
  SA sa;
  SB sb;
  const int64_t rowa = SA::row_of(A, m0, M, tid);
  const int64_t rowb = SB::row_of(B, n0, N, tid);
  const bool ala = SA::aligned(A), alb = SB::aligned(B);
  if (kbeg >= kend) return;
  const int xa = wm * Cfg::WTM + (lane & 15), xb = wn * Cfg::WTN + (lane & 15);
  sa.load(A, m0, M, kbeg, kend, tid, rowa, ala);
  sb.load(B, n0, N, kbeg, kend, tid, rowb, alb);
  sa.store(smem, tid);
  sb.store(smem + LA_::SIZE, tid);
  if (kbeg + BK < kend) {
    sa.load(A, m0, M, kbeg + BK, kend, tid, rowa, ala);
    sb.load(B, n0, N, kbeg + BK, kend, tid, rowb, alb);
  }
  __syncthreads();
  T fa[2][Cfg::MI][2], fb[2][Cfg::NI][2];  // fragments of two sub-step pairs
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i) read2<T, LA, BM, BK>(smem, xa + i * 16, 0, 0, lane, fa[0][i]);
#pragma unroll
  for (int j = 0; j < Cfg::NI; ++j) read2<T, LB, BN, BK>(smem + LA_::SIZE, xb + j * 16, 0, 0, lane, fb[0][j]);
  int cur = 0;
  int step = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool next = k0 + BK < kend;
    const T* cbuf = smem + cur * STAGE;
    T* nbuf = smem + (cur ^ 1) * STAGE;
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) {
      const int sl = p & 1, nsl = sl ^ 1;
      if (p + 1 < NPAIR) {
        const int c = (p + 1) >> 1, s0 = 2 * ((p + 1) & 1);
#pragma unroll
        for (int i = 0; i < Cfg::MI; ++i) read2<T, LA, BM, BK>(cbuf, xa + i * 16, c, s0, lane, fa[nsl][i]);
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j)
          read2<T, LB, BN, BK>(cbuf + LA_::SIZE, xb + j * 16, c, s0, lane, fb[nsl][j]);
      } else {
        __syncthreads();  // slice i+1 stored by every wave; reads of this buffer done
        if (next) {
#pragma unroll
          for (int i = 0; i < Cfg::MI; ++i) read2<T, LA, BM, BK>(nbuf, xa + i * 16, 0, 0, lane, fa[nsl][i]);
#pragma unroll
          for (int j = 0; j < Cfg::NI; ++j)
            read2<T, LB, BN, BK>(nbuf + LA_::SIZE, xb + j * 16, 0, 0, lane, fb[nsl][j]);
        }
      }
      if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
          for (int j = 0; j < Cfg::NI; ++j) MfmaT<T>::mma(fa[sl][i][t], fb[sl][j][t], acc[i][j]);
      if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_sched_barrier(0);  // keep each pair's MFMAs in place
      if (p == NPAIR - 2 && next) {
        // slice i+1 (in registers since step i-1) into the other buffer, whose
        // last reads finished before the previous barrier; then the loads of
        // slice i+2, which have a whole step to arrive
        sa.store(nbuf, tid);
        sb.store(nbuf + LA_::SIZE, tid);
        if (k0 + 2 * BK < kend) {
          sa.load(A, m0, M, k0 + 2 * BK, kend, tid, rowa, ala);
          sb.load(B, n0, N, k0 + 2 * BK, kend, tid, rowb, alb);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (FOLD > 0) {
      if (++step == FOLD) {
        step = 0;
        fold_into<Cfg>(acc, *fold);
      }
    }
    cur ^= 1;
  }
  if constexpr (FOLD > 0) fold_into<Cfg>(acc, *fold);
}

// Runs the K loop of one operand pair into acc.  LDS is double buffered:
// the slice for step i+1 is loaded from global memory while step i feeds the
// MFMAs, stored into the other buffer, and one barrier per step separates
// the two.  FOLD > 0 (FP32 only): acc is added into the FP64 set `fold`
// and cleared every FOLD steps and at the end, so FP32 rounding of the
// running sums does not grow with K.
template <class Cfg, class T, class TA, int LA, class TB, int LB, int BM, int BN, int BK, int FOLD = 0>
__device__ __forceinline__ void mma_loop_flat(const Operand<TA>& A, const Operand<TB>& B, int m0, int n0, int M,
                                         int N, int64_t kbeg, int64_t kend, T* smem,
                                         typename MfmaT<T>::acc_t (&acc)[Cfg::MI][Cfg::NI],
                                         FoldAcc<Cfg>* fold = nullptr) {
  typedef Lds<T, LA, BM, BK> LA_;
  typedef Lds<T, LB, BN, BK> LB_;
  constexpr int STAGE = LA_::SIZE + LB_::SIZE;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int wm = wv / (BN / Cfg::WTN);
  const int wn = wv % (BN / Cfg::WTN);
  typedef Stager<T, TA, LA, BM, BK, Cfg::THREADS> SA;
  typedef Stager<T, TB, LB, BN, BK, Cfg::THREADS> SB;
  SA sa;
  SB sb;
  const int64_t rowa = SA::row_of(A, m0, M, tid);
  const int64_t rowb = SB::row_of(B, n0, N, tid);
  const bool ala = SA::aligned(A), alb = SB::aligned(B);
  if (kbeg >= kend) return;
  sa.load(A, m0, M, kbeg, kend, tid, rowa, ala);
  sb.load(B, n0, N, kbeg, kend, tid, rowb, alb);
  sa.store(smem, tid);
  sb.store(smem + LA_::SIZE, tid);
  __syncthreads();
  int cur = 0;
  int step = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      sa.load(A, m0, M, k0 + BK, kend, tid, rowa, ala);
      sb.load(B, n0, N, k0 + BK, kend, tid, rowb, alb);
    }
    const T* As = smem + cur * STAGE;
    const T* Bs = As + LA_::SIZE;
#pragma unroll
    for (int c = 0; c < BK / 16; ++c) {
      T a[Cfg::MI][4], b[Cfg::NI][4];
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i) read4<T, LA, BM, BK>(As, wm * Cfg::WTM + i * 16 + (lane & 15), c, lane, a[i]);
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) read4<T, LB, BN, BK>(Bs, wn * Cfg::WTN + j * 16 + (lane & 15), c, lane, b[j]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
          for (int j = 0; j < Cfg::NI; ++j) MfmaT<T>::mma(a[i][s], b[j][s], acc[i][j]);
    }
    if constexpr (FOLD > 0) {
      if (++step == FOLD) {
        step = 0;
        fold_into<Cfg>(acc, *fold);
      }
    }
    if (more) {
      T* nxt = smem + (cur ^ 1) * STAGE;
      sa.store(nxt, tid);
      sb.store(nxt + LA_::SIZE, tid);
    }
    __syncthreads();
    cur ^= 1;
  }
  if constexpr (FOLD > 0) fold_into<Cfg>(acc, *fold);
}

// Whether a kernel raises the wave priority around its MFMAs: yes, unless
// the epilogue type says kPrio = false (measured per epilogue).
template <class E, class = void>
struct EpiPrio {
  static constexpr bool value = true;
};
template <class E>
struct EpiPrio<E, std::void_t<decltype(E::kPrio)>> {
  static constexpr bool value = E::kPrio;
};

// The K loop of one operand pair: the software-pipelined form, except for
// folded FP32 accumulators, whose extra FP64 set leaves no registers for it.
template <class Cfg, class T, class TA, int LA, class TB, int LB, int BM, int BN, int BK, int FOLD = 0,
          bool PRIO = true>
__device__ __forceinline__ void mma_loop(const Operand<TA>& A, const Operand<TB>& B, int m0, int n0, int M,
                                         int N, int64_t kbeg, int64_t kend, T* smem,
                                         typename MfmaT<T>::acc_t (&acc)[Cfg::MI][Cfg::NI],
                                         FoldAcc<Cfg>* fold = nullptr) {
  if constexpr (FOLD > 0)
    mma_loop_flat<Cfg, T, TA, LA, TB, LB, BM, BN, BK, FOLD>(A, B, m0, n0, M, N, kbeg, kend, smem, acc, fold);
  else
    mma_loop_pp<Cfg, T, TA, LA, TB, LB, BM, BN, BK, 0, PRIO>(A, B, m0, n0, M, N, kbeg, kend, smem, acc, fold);
}

// Tile coordinates handed to epilogues.
struct TileAt {
  int m_wave, n_wave;  // first row / column of this wavefront's sub-tile
  int lane;
  int z;               // split-K index
  int batch;           // batch index
};

// Generic kernel: NOPS = 1 (one operand pair) or 2 (two pairs into two
// accumulator sets, same tile, e.g. Phi and Psi Gram blocks).
template <class T, int BM, int BN, int BK, int WM, int WN, class TA, int LA, class TB, int LB, int NOPS,
          class Epi, int FOLD = 0>
__global__ __launch_bounds__(WM* WN* ISDF_WAVE, 2) void gemm_kernel(GemmShape sh, Operand<TA> A0, Operand<TB> B0,
                                                                 Operand<TA> A1, Operand<TB> B1, int64_t K1,
                                                                 Epi epi) {
  static_assert(FOLD == 0 || sizeof(T) == 4, "folding is for FP32 accumulators");
  typedef TileCfg<T, BM, BN, BK, WM, WN> Cfg;
  if (sh.abort && *sh.abort) return;
  constexpr int STAGE = Lds<T, LA, BM, BK>::SIZE + Lds<T, LB, BN, BK>::SIZE;
  __shared__ __attribute__((aligned(16))) T smem[2 * STAGE];
  const int tiles_n = (sh.N + BN - 1) / BN;
  const int tiles_m = (sh.M + BM - 1) / BM;
  const int ntiles = (int)gemm_tiles(tiles_m, tiles_n, sh.lower_only);
  const int bid = blockIdx.x;
  int z, logical;
  if (sh.splits > 1 && sh.splits % 8 == 0) {
    // split-K: each XCD owns whole K slices (z = xcd, xcd + 8, ...), so the
    // operands of a slice are fetched into one L2 and shared by every tile
    const int xcd = bid % 8, q = bid / 8;
    z = xcd + 8 * (q / ntiles);
    logical = q % ntiles;
  } else {
    z = bid / ntiles;
    logical = xcd_remap(bid % ntiles, ntiles);
  }
  int tm, tn;
  if (sh.lower_only) {  // row-major enumeration of the lower triangle of tiles
    tm = (int)((sqrt(8.0 * logical + 1.0) - 1.0) * 0.5);
    while ((int64_t)(tm + 1) * (tm + 2) / 2 <= logical) ++tm;
    while ((int64_t)tm * (tm + 1) / 2 > logical) --tm;
    tn = logical - tm * (tm + 1) / 2;
  } else {  // groups of GM row blocks, column-major inside a group
    constexpr int GM = 8;
    const int g = logical / (GM * tiles_n), r = logical % (GM * tiles_n);
    const int rows_in = tiles_m - g * GM < GM ? tiles_m - g * GM : GM;  // last group may be short
    tm = g * GM + r % rows_in;
    tn = r / rows_in;
  }
  const int m0 = tm * BM, n0 = tn * BN;
  const int batch = blockIdx.y;
  if (batch) {
    A0.p += batch * sh.sa;
    B0.p += batch * sh.sb;
  }
  const int64_t kbeg = (int64_t)z * sh.kchunk;
  const int64_t kend = kbeg + sh.kchunk < sh.K ? kbeg + sh.kchunk : sh.K;

  typedef typename MfmaT<T>::acc_t acc_t;
  acc_t acc0[Cfg::MI][Cfg::NI];
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j) acc0[i][j] = acc_t{0, 0, 0, 0};
  FoldAcc<Cfg> f0;
  if constexpr (FOLD > 0) {
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) f0.v[i][j] = d4v{0, 0, 0, 0};
  }
  mma_loop<Cfg, T, TA, LA, TB, LB, BM, BN, BK, FOLD, EpiPrio<Epi>::value>(A0, B0, m0, n0, sh.M, sh.N, kbeg, kend, smem,
                                                                         acc0, &f0);

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int wm = wv / (BN / Cfg::WTN), wn = wv % (BN / Cfg::WTN);
  TileAt at{m0 + wm * Cfg::WTM, n0 + wn * Cfg::WTN, lane, z, batch};
  if constexpr (NOPS == 2) {
    acc_t acc1[Cfg::MI][Cfg::NI];
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) acc1[i][j] = acc_t{0, 0, 0, 0};
    FoldAcc<Cfg> f1;
    if constexpr (FOLD > 0) {
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) f1.v[i][j] = d4v{0, 0, 0, 0};
    }
    __syncthreads();
    mma_loop<Cfg, T, TA, LA, TB, LB, BM, BN, BK, FOLD, EpiPrio<Epi>::value>(A1, B1, m0, n0, sh.M, sh.N, 0, K1, smem,
                                                                           acc1, &f1);
    if constexpr (FOLD > 0)
      epi.template apply2<Cfg>(f0.v, f1.v, at);
    else
      epi.template apply2<Cfg>(acc0, acc1, at);
  } else {
    if constexpr (FOLD > 0)
      epi.template apply<Cfg>(f0.v, at);
    else
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
  int64_t bstride;  // batch stride of C
  template <class Cfg, class Acc>
  __device__ __forceinline__ void apply(const Acc (&acc)[Cfg::MI][Cfg::NI], const TileAt& at) const {
    TC* Cz = C + at.z * zstride + at.batch * bstride;
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
