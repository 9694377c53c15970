// Split-precision MFMA GEMM for gfx950: FP64-accurate-enough products from
// 16-bit matrix cores.
//
//   acc(m, n) = sum_k A(m, k) B(k, n),  A and B given K-contiguous (KC) in
//   double or float, split while they are staged into LDS:
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
// rounding stays negligible and the leading sum sees one rounding per
// 32-deep MFMA), and the epilogue receives their sum in FP64.
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
  static constexpr int LDK = BK + 8;  // LDS row of one part, 16-bit elements (80 bytes)
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile");
  __device__ __forceinline__ static int orow(int lane, int j) { return 4 * (lane >> 4) + j; }
};

// Stages one BK slice of a KC operand: thread -> (x, E consecutive k),
// source kept in registers, split into NP part planes [X][LDK] on store.
template <int MODE, class TS, int X, int THREADS>
struct SplitStager {
  typedef SplitT<MODE> S;
  static constexpr int BK = 32;
  static constexpr int E = X * BK / THREADS;
  static constexpr int RUNS = BK / E;
  static_assert(E % 8 == 0, "runs of whole 16-byte parts");
  double v[E];
  __device__ __forceinline__ void load(const Operand<TS>& op, int x0, int xlim, int64_t k0, int64_t klim, int tid,
                                       int64_t row, bool aligned) {
    const int x = tid / RUNS;
    const int64_t kb = k0 + (tid % RUNS) * E;
    const TS* base = op.p + row * op.ld + kb;
    if (aligned && x0 + X <= xlim && k0 + BK <= klim) {
#pragma unroll
      for (int e = 0; e < E; e += 2) load_pair<TS>(base + e, v[e], v[e + 1]);
    } else {
      const bool okx = x0 + x < xlim;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = (okx && kb + e < klim) ? (double)base[e] : 0.0;
    }
  }
  __device__ __forceinline__ void store(typename S::P* s, int lds_k, int tid, double scale) const {
    const int x = tid / RUNS, kb = (tid % RUNS) * E;
    typename S::P parts[S::NP][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      typename S::P o[S::NP];
      S::split(v[e], scale, o);
#pragma unroll
      for (int p = 0; p < S::NP; ++p) parts[p][e] = o[p];
    }
#pragma unroll
    for (int p = 0; p < S::NP; ++p) {
      typename S::V* d = reinterpret_cast<typename S::V*>(s + (p * X + x) * lds_k + kb);
#pragma unroll
      for (int q = 0; q < E / 8; ++q) {
        typename S::V w;
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = parts[p][8 * q + e];
        d[q] = w;
      }
    }
  }
  __device__ __forceinline__ static int64_t row_of(const Operand<TS>& op, int x0, int xlim, int tid) {
    const int x = x0 + tid / RUNS;
    const int xc = x < xlim ? x : (xlim > 0 ? xlim - 1 : 0);
    return op.rows ? (int64_t)op.rows[xc] : (int64_t)xc;
  }
  __device__ __forceinline__ static bool aligned(const Operand<TS>& op) {
    return (op.ld % 2 == 0) && (((uintptr_t)op.p) % (2 * sizeof(TS)) == 0);
  }
};

// K loop of one operand pair into the leading (acc0) and correction (acc1)
// accumulators.  Single LDS buffer, the next slice prefetched in registers.
template <int MODE, class Cfg, class TA, class TB, int BM, int BN>
__device__ __forceinline__ void split_loop(const Operand<TA>& A, const Operand<TB>& B, int m0, int n0, int M, int N,
                                           int64_t K, double sa, double sb, typename SplitT<MODE>::P* smem,
                                           f4v (&acc0)[Cfg::MI][Cfg::NI], f4v (&acc1)[Cfg::MI][Cfg::NI]) {
  typedef SplitT<MODE> S;
  typedef typename S::P P;
  typedef typename S::V V;
  constexpr int LDK = Cfg::LDK;
  P* As = smem;
  P* Bs = smem + S::NP * BM * LDK;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / (BN / Cfg::WTN), wn = wv % (BN / Cfg::WTN);
  typedef SplitStager<MODE, TA, BM, Cfg::THREADS> SA;
  typedef SplitStager<MODE, TB, BN, Cfg::THREADS> SB;
  SA sa_;
  SB sb_;
  const int64_t rowa = SA::row_of(A, m0, M, tid), rowb = SB::row_of(B, n0, N, tid);
  const bool ala = SA::aligned(A), alb = SB::aligned(B);
  if (K <= 0) return;
  sa_.load(A, m0, M, 0, K, tid, rowa, ala);
  sb_.load(B, n0, N, 0, K, tid, rowb, alb);
  sa_.store(As, LDK, tid, sa);
  sb_.store(Bs, LDK, tid, sb);
  __syncthreads();
  const int q8 = 8 * (lane >> 4);
  for (int64_t k0 = 0; k0 < K; k0 += Cfg::BK) {
    const bool more = k0 + Cfg::BK < K;
    if (more) {
      sa_.load(A, m0, M, k0 + Cfg::BK, K, tid, rowa, ala);
      sb_.load(B, n0, N, k0 + Cfg::BK, K, tid, rowb, alb);
    }
    V a[S::NP][Cfg::MI], b[S::NP][Cfg::NI];
#pragma unroll
    for (int p = 0; p < S::NP; ++p) {
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
        a[p][i] = *reinterpret_cast<const V*>(As + (p * BM + wm * Cfg::WTM + i * 16 + (lane & 15)) * LDK + q8);
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j)
        b[p][j] = *reinterpret_cast<const V*>(Bs + (p * BN + wn * Cfg::WTN + j * 16 + (lane & 15)) * LDK + q8);
    }
#pragma unroll
    for (int pp = 1; pp < S::NPROD; ++pp)
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) S::mma(a[S::pa(pp)][i], b[S::pb(pp)][j], acc1[i][j]);
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) S::mma(a[0][i], b[0][j], acc0[i][j]);
    __syncthreads();
    if (more) {
      sa_.store(As, LDK, tid, sa);
      sb_.store(Bs, LDK, tid, sb);
      __syncthreads();
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

// NOPS = 1 or 2 operand pairs (two pairs: two accumulator sets, e.g. the
// Gram blocks of Phi and Psi for the same tile).  scales: null (BF16X6) or
// device [s_A0, s_B0, s_A1, s_B1] (FP16X3).
template <int MODE, int BM, int BN, int WM, int WN, class TA, class TB, int NOPS, class Epi>
__global__ __launch_bounds__(WM* WN* ISDF_WAVE, 2) void gemm_split_kernel(GemmShape sh, Operand<TA> A0, Operand<TB> B0,
                                                                       Operand<TA> A1, Operand<TB> B1, int64_t K1,
                                                                       const double* scales, Epi epi) {
  typedef SplitCfg<BM, BN, WM, WN> Cfg;
  typedef SplitT<MODE> S;
  if (sh.abort && *sh.abort) return;
  __shared__ __attribute__((aligned(16))) typename S::P smem[S::NP * (BM + BN) * Cfg::LDK];
  const int tiles_n = (sh.N + BN - 1) / BN, tiles_m = (sh.M + BM - 1) / BM;
  const int ntiles = tiles_m * tiles_n;
  const int logical = xcd_remap(blockIdx.x, ntiles);
  const int tm = logical / tiles_n, tn = logical % tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv / (BN / Cfg::WTN), wn = wv % (BN / Cfg::WTN);
  TileAt at{m0 + wm * Cfg::WTM, n0 + wn * Cfg::WTN, lane, 0, 0};
  double s0a = 1.0, s0b = 1.0, s1a = 1.0, s1b = 1.0;
  if (scales) {
    s0a = scales[0];
    s0b = scales[1];
    s1a = scales[2];
    s1b = scales[3];
  }
  f4v c0[Cfg::MI][Cfg::NI], c1[Cfg::MI][Cfg::NI];
  d4v r0[Cfg::MI][Cfg::NI];
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j) c0[i][j] = c1[i][j] = f4v{0, 0, 0, 0};
  split_loop<MODE, Cfg, TA, TB, BM, BN>(A0, B0, m0, n0, sh.M, sh.N, sh.K, s0a, s0b, smem, c0, c1);
  const double u0 = 1.0 / (s0a * s0b);
#pragma unroll
  for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
    for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) r0[i][j][r] = ((double)c0[i][j][r] + (double)c1[i][j][r]) * u0;
  if constexpr (NOPS == 2) {
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j) c0[i][j] = c1[i][j] = f4v{0, 0, 0, 0};
    __syncthreads();
    split_loop<MODE, Cfg, TA, TB, BM, BN>(A1, B1, m0, n0, sh.M, sh.N, K1, s1a, s1b, smem, c0, c1);
    d4v r1[Cfg::MI][Cfg::NI];
    const double u1 = 1.0 / (s1a * s1b);
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int j = 0; j < Cfg::NI; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) r1[i][j][r] = ((double)c0[i][j][r] + (double)c1[i][j][r]) * u1;
    epi.template apply2<Cfg>(r0, r1, at);
  } else {
    epi.template apply<Cfg>(r0, at);
  }
}

}  // namespace isdf
