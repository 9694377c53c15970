// Shared pieces of the fit and its adjoint: Gram + Hadamard GEMMs, the
// FP64 Cholesky / inverse of C C^H, device state.  Everything here has
// internal linkage (anonymous namespace) so that each translation unit gets
// its own copy of the kernels.
#pragma once
#include <float.h>
#include <limits.h>

#include "gemm_split.h"

namespace isdf {
namespace {

constexpr int NB = 64;  // Cholesky block

struct FitState {
  int abort;    // nonzero: later launches of this call are no-ops
  int pivot;    // first failing pivot (INT_MAX: none)
  int bad_idx;  // first invalid idx position (INT_MAX: none)
  int pad;
  double pmin, pmax;
  double loss;
};

// ------------------------------------------------------------ idx checks
__global__ void fit_state_init(FitState* st) {
  st->abort = 0;
  st->pivot = INT_MAX;
  st->bad_idx = INT_MAX;
  st->pad = 0;
  st->pmin = INFINITY;
  st->pmax = 0.0;
  st->loss = 0.0;
}

__global__ void check_idx(const int32_t* __restrict__ idx, int n_mu, int64_t nr, int* __restrict__ marker,
                          FitState* st) {
  int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= n_mu) return;
  int v = idx[mu];
  bool bad = v < 0 || v >= nr;
  if (!bad) bad = atomicAdd(&marker[v], 1) != 0;
  if (bad) {
    atomicMin(&st->bad_idx, mu);
    atomicOr(&st->abort, 1);
  }
}

// E[n][k], n = 32 b + 16 c + t -> column nu = 16 b + t, part c (0: Re A, 1: Im A);
// k = 2 i + comp multiplies (re, im) of orbital i of the grid row.
// With Phi_mu[nu][i] = a + i b:  Re A = sum x a + y b,  Im A = sum y a - x b.
template <class TS, class T>
__global__ void pack_gram_rhs(const TS* __restrict__ phi, int64_t ld, int n, const int32_t* __restrict__ idx,
                              int n_mu, int64_t nr, int rows, T* __restrict__ E) {
  const int64_t total = (int64_t)rows * 2 * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / (2 * n));
    const int k = (int)(e % (2 * n));
    const int b = r >> 5, c = (r >> 4) & 1, t = r & 15;
    const int nu = b * 16 + t;
    double v = 0.0;
    if (nu < n_mu) {
      int64_t p = idx[nu];
      if (p < 0 || p >= nr) p = 0;  // invalid entries are reported by check_idx
      const int i = k >> 1, comp = k & 1;
      double2 z = Cplx<TS>::load(phi + 2 * (p * ld + i));
      if (c == 0) v = comp == 0 ? z.x : z.y;
      else v = comp == 0 ? -z.y : z.x;
    }
    E[e] = (T)v;
  }
}

// Gram + Hadamard epilogue.  Accumulator pairs (j, j+1) of a wavefront hold
// Re and Im of the same column nu.
enum { G_REAL = 0, G_CPLX = 1, G_EMB = 2 };
struct EpiGram {
  double* G;  // may be null (only A / B wanted)
  int64_t ldg;  // doubles
  int M;
  int n_mu;
  int mode;
  double* Aout;  // optional: A (and B) as interleaved complex rows, ld ldab doubles
  double* Bout;
  int64_t ldab;
  template <class Cfg, class Acc>
  __device__ __forceinline__ void apply(const Acc (&acc)[Cfg::MI][Cfg::NI], const TileAt& at) const {
    // Psi = Phi: G = |A|^2 (real)
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int jp = 0; jp < Cfg::NI / 2; ++jp) {
        const int nu = ((at.n_wave + 32 * jp) >> 5) * 16 + (at.lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = at.m_wave + i * 16 + Cfg::orow(at.lane, r);
          if (m < M && nu < n_mu) {
            const double re = (double)acc[i][2 * jp][r], im = (double)acc[i][2 * jp + 1][r];
            if (G) G[(int64_t)m * ldg + nu] = re * re + im * im;
            if (Aout) *reinterpret_cast<double2*>(Aout + (int64_t)m * ldab + 2 * nu) = make_double2(re, im);
          }
        }
      }
  }
  template <class Cfg, class Acc>
  __device__ __forceinline__ void apply2(const Acc (&a)[Cfg::MI][Cfg::NI], const Acc (&b)[Cfg::MI][Cfg::NI],
                                         const TileAt& at) const {
    // G = A .* conj(B)
#pragma unroll
    for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
      for (int jp = 0; jp < Cfg::NI / 2; ++jp) {
        const int nu = ((at.n_wave + 32 * jp) >> 5) * 16 + (at.lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = at.m_wave + i * 16 + Cfg::orow(at.lane, r);
          if (m < M && nu < n_mu) {
            const double ar = (double)a[i][2 * jp][r], ai = (double)a[i][2 * jp + 1][r];
            const double br = (double)b[i][2 * jp][r], bi = (double)b[i][2 * jp + 1][r];
            const double x = ar * br + ai * bi, y = ai * br - ar * bi;
            if (Aout) *reinterpret_cast<double2*>(Aout + (int64_t)m * ldab + 2 * nu) = make_double2(ar, ai);
            if (Bout) *reinterpret_cast<double2*>(Bout + (int64_t)m * ldab + 2 * nu) = make_double2(br, bi);
            if (!G) continue;
            if (mode == G_CPLX) {
              *reinterpret_cast<double2*>(G + (int64_t)m * ldg + 2 * nu) = make_double2(x, y);
            } else {
              *reinterpret_cast<double2*>(G + (int64_t)(2 * m) * ldg + 2 * nu) = make_double2(x, y);
              *reinterpret_cast<double2*>(G + (int64_t)(2 * m + 1) * ldg + 2 * nu) = make_double2(-y, x);
            }
          }
        }
      }
  }
};

// ------------------------------------------------------------ Cholesky
// Factors the kb x kb diagonal block at (k0, k0) of X in place (lower) and
// writes its inverse into the same block of Y.  The inverse is reduced
// alongside the elimination (L X = I solved row by row: at step j,
// X_j = R_j / l_jj and R_i -= l_ij X_j for i > j).  Step j updates with the
// unscaled column j and 1 / pivot; column j (and row j of R) are scaled at
// the start of step j + 1, when nothing reads them any more, so each step
// needs a single barrier.  Threads form a 16 x 16 grid over (row, column).
__global__ __launch_bounds__(256) void potrf_diag(double* __restrict__ X, int64_t ldx, int k0, int kb,
                                                  double* __restrict__ Y, int64_t ldy, FitState* st) {
  if (st->abort) return;
  __shared__ double a[NB][NB + 1];
  __shared__ double r[NB][NB + 1];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int i = ty; i < kb; i += 16)
    for (int j = tx; j < kb; j += 16) {
      a[i][j] = j <= i ? X[(int64_t)(k0 + i) * ldx + k0 + j] : 0.0;
      r[i][j] = i == j ? 1.0 : 0.0;
    }
  __syncthreads();
  int failed = -1;
  double il_prev = 0.0;
  for (int j = 0; j < kb; ++j) {
    const double piv = a[j][j];
    if (!(piv > 0.0) || !(piv < INFINITY)) {
      failed = j;
      break;
    }
    if (j > 0) {  // scale column j - 1 of L and row j - 1 of the inverse
      const int p = j - 1;
      if (tid < kb) {
        if (tid > p) a[tid][p] *= il_prev;
        else r[p][tid] *= il_prev;
      }
    }
    const double l = sqrt(piv), ip = 1.0 / piv;
    if (tid == 0) {
      atomic_min_pos(&st->pmin, piv);
      atomic_max_pos(&st->pmax, piv);
    }
    for (int i = j + 1 + ty; i < kb; i += 16) {
      const double aij = a[i][j] * ip;
      for (int c = j + 1 + tx; c <= i; c += 16) a[i][c] -= aij * a[c][j];
      for (int c = tx; c <= j; c += 16) r[i][c] -= aij * r[j][c];
    }
    __syncthreads();
    if (tid == 0) a[j][j] = l;  // read again only by the scaling of step j + 1
    il_prev = 1.0 / l;
  }
  if (failed >= 0) {
    if (tid == 0) {
      atomicMin(&st->pivot, k0 + failed);
      atomicOr(&st->abort, 1);
    }
    return;
  }
  {  // scale the last column / row
    const int p = kb - 1;
    if (tid < kb) {
      if (tid > p) a[tid][p] *= il_prev;
      else r[p][tid] *= il_prev;
    }
  }
  __syncthreads();
  for (int i = ty; i < kb; i += 16)
    for (int j = tx; j < kb; j += 16) {
      if (j <= i) X[(int64_t)(k0 + i) * ldx + k0 + j] = a[i][j];
      Y[(int64_t)(k0 + i) * ldy + k0 + j] = j <= i ? r[i][j] : 0.0;
    }
}

__global__ void fit_finish(const FitState* st, isdf_fit_info* info, double* loss_out, int backward) {
  int status = ISDF_OK;
  if (st->bad_idx != INT_MAX) status = ISDF_E_BAD_IDX;
  else if (st->pivot != INT_MAX) status = ISDF_E_NOT_PD;
  else if (st->abort) status = ISDF_E_NONFINITE;
  info->status = status;
  info->pivot = st->pivot == INT_MAX ? -1 : st->pivot;
  info->bad_idx = st->bad_idx == INT_MAX ? -1 : st->bad_idx;
  info->reserved = 0;
  info->pivot_min = st->pmin == INFINITY ? 0.0 : st->pmin;
  info->pivot_max = st->pmax;
  info->loss = st->loss;
  if (backward && loss_out) *loss_out = st->loss;
}

// ------------------------------------------------------------ launches
template <class T, int BM, int BN, int BK, int WM, int WN, class TA, int LA, class TB, int LB, int NOPS,
          int FOLD = 0, class Epi>
static bool launch_gemm(int M, int N, int64_t K, Operand<TA> A0, Operand<TB> B0, Operand<TA> A1,
                        Operand<TB> B1, int64_t K1, const Epi& epi, int lower_only, const int* abort,
                        hipStream_t st, int splits = 1, int batch = 1, int64_t sa = 0, int64_t sb = 0) {
  if (M <= 0 || N <= 0) return true;
  GemmShape sh;
  sh.M = M;
  sh.N = N;
  sh.K = K;
  sh.kchunk = splits > 1 ? ceil_div(ceil_div(K, splits), BK) * BK : K;
  sh.splits = splits;
  sh.lower_only = lower_only && M == N && BM == BN;
  sh.abort = abort;
  sh.sa = sa;
  sh.sb = sb;
  const int64_t tiles = gemm_tiles((int)ceil_div(M, BM), (int)ceil_div(N, BN), sh.lower_only);
  dim3 grid((unsigned)(tiles * splits), (unsigned)batch, 1);
  hipLaunchKernelGGL((gemm_kernel<T, BM, BN, BK, WM, WN, TA, LA, TB, LB, NOPS, Epi, FOLD>), grid,
                     dim3(WM * WN * ISDF_WAVE), 0, st, sh, A0, B0, A1, B1, K1, epi);
  return launch_ok();
}

// Plain FP64 GEMM C = alpha op(A) op(B) + beta C.
template <int LA, int LB, class TC, class TA = double>
static bool dgemm(int M, int N, int64_t K, const TA* A, int64_t lda, const double* B, int64_t ldb, TC* C,
                  int64_t ldc, double alpha, double beta, int lower_only, const int* abort, hipStream_t st,
                  const double* rowscale = nullptr) {
  EpiStore<TC> epi{C, ldc, M, N, alpha, beta, rowscale, 0, 0};
  Operand<TA> a{A, lda, nullptr};
  Operand<double> b{B, ldb, nullptr};
  return launch_gemm<double, 128, 128, 16, 2, 2, TA, LA, double, LB, 1>(M, N, K, a, b, a, b, 0, epi, lower_only,
                                                                       abort, st);
}

// Batched FP64 GEMM: batch b uses A + b sa, B + b sb, C + b sc.
template <int LA, int LB>
static bool dgemm_batched(int M, int N, int64_t K, const double* A, int64_t lda, int64_t sa, const double* B,
                          int64_t ldb, int64_t sb, double* C, int64_t ldc, int64_t sc, int batch, double alpha,
                          const int* abort, hipStream_t st) {
  EpiStore<double> epi{C, ldc, M, N, alpha, 0.0, nullptr, 0, sc};
  Operand<double> a{A, lda, nullptr, nullptr};
  Operand<double> b{B, ldb, nullptr, nullptr};
  return launch_gemm<double, 128, 128, 16, 2, 2, double, LA, double, LB, 1>(M, N, K, a, b, a, b, 0, epi, 0, abort, st,
                                                                           1, batch, sa, sb);
}

// GEMM in compute type T with split-K slices written to C + z * zstride.
// bscale: optional per-k factor of B; lower_only: skip tiles above the diagonal.
template <class T, int LA, int LB, class TA, class TB, class TC>
static bool tgemm(int M, int N, int64_t K, const TA* A, int64_t lda, const TB* B, int64_t ldb, TC* C, int64_t ldc,
                  double alpha, double beta, const int* abort, hipStream_t st, int splits = 1,
                  int64_t zstride = 0, const double* bscale = nullptr, int lower_only = 0) {
  EpiStore<TC> epi{C, ldc, M, N, alpha, beta, nullptr, zstride, 0};
  Operand<TA> a{A, lda, nullptr, nullptr};
  Operand<TB> b{B, ldb, nullptr, bscale};
  return launch_gemm<T, 128, 128, 16, 2, 2, TA, LA, TB, LB, 1>(M, N, K, a, b, a, b, 0, epi, lower_only, abort, st,
                                                               splits);
}

// Cholesky of X (n x n, lower, in place) and W = X^-1 into X:
//  1. blocked right-looking Cholesky, 64-wide diagonal blocks factored and
//     inverted in LDS, panel L21 = A21 L11^-T and trailing update on MFMA;
//  2. Y = L^-1 by recursive doubling: once every aligned segment of size b
//     has its inverse, a pair [[A, 0], [L21, C]] gets its lower-left block
//     -C^-1 L21 A^-1 (two GEMMs, batched over all pairs of the level);
//  3. W = Y^T Y.
struct InvWork {
  double* Y;  // [n][n]
  double* R;  // [n][n] scratch
};

static int spd_inverse(double* X, int n, InvWork w, FitState* st, hipStream_t s) {
  const int* ab = &st->abort;
  const int nblk = (int)ceil_div(n, NB);
  if (!fill<double>(w.Y, (int64_t)n * n, 0.0, s)) return ISDF_E_HIP;
  for (int b = 0; b < nblk; ++b) {
    const int k0 = b * NB, kb = n - k0 < NB ? n - k0 : NB;
    hipLaunchKernelGGL(potrf_diag, dim3(1), dim3(256), 0, s, X, (int64_t)n, k0, kb, w.Y, (int64_t)n, st);
    if (!launch_ok()) return ISDF_E_HIP;
    const int rest = n - k0 - kb;
    if (rest <= 0) continue;
    double* P = X + (int64_t)(k0 + kb) * n + k0;
    // panel: L21 = A21 L11^-T (in place: each workgroup reads all K of its rows before writing them)
    if (!dgemm<KC, KC>(rest, kb, kb, P, n, w.Y + (int64_t)k0 * n + k0, n, P, n, 1.0, 0.0, 0, ab, s))
      return ISDF_E_HIP;
    // trailing: A22 -= L21 L21^T (lower tiles)
    double* T = X + (int64_t)(k0 + kb) * n + (k0 + kb);
    if (!dgemm<KC, KC>(rest, rest, kb, P, n, P, n, T, n, -1.0, 1.0, 1, ab, s)) return ISDF_E_HIP;
  }
  const int64_t ld = n;
  for (int b = NB; b < n; b *= 2) {
    const int pairs = n / (2 * b);
    const int64_t step = 2 * (int64_t)b * (ld + 1);  // from one pair's origin to the next
    if (pairs > 0) {
      // R_p = L21 A^-1, then C-block rows of Y: -C^-1 R_p
      if (!dgemm_batched<KC, XC>(b, b, b, X + (int64_t)b * ld, ld, step, w.Y, ld, step, w.R, b, (int64_t)b * b,
                                 pairs, 1.0, ab, s))
        return ISDF_E_HIP;
      if (!dgemm_batched<KC, XC>(b, b, b, w.Y + (int64_t)b * ld + b, ld, step, w.R, b, (int64_t)b * b,
                                 w.Y + (int64_t)b * ld, ld, step, pairs, -1.0, ab, s))
        return ISDF_E_HIP;
    }
    const int o = pairs * 2 * b, rem = n - o;
    if (rem > b) {  // ragged last pair: A of size b, C of size rem - b
      const int c = rem - b;
      const int64_t org = (int64_t)o * (ld + 1);
      if (!dgemm_batched<KC, XC>(c, b, b, X + org + (int64_t)b * ld, ld, 0, w.Y + org, ld, 0, w.R, b, 0, 1, 1.0, ab,
                                 s))
        return ISDF_E_HIP;
      if (!dgemm_batched<KC, XC>(c, b, c, w.Y + org + (int64_t)b * ld + b, ld, 0, w.R, b, 0,
                                 w.Y + org + (int64_t)b * ld, ld, 0, 1, -1.0, ab, s))
        return ISDF_E_HIP;
    }
  }
  // W = Y^T Y
  if (!dgemm<XC, XC>(n, n, n, w.Y, n, w.Y, n, X, n, 1.0, 0.0, 0, ab, s)) return ISDF_E_HIP;
  return ISDF_OK;
}

// Precision policy of the orbital contractions (the Gram blocks and the
// adjoint's products with Phi_mu / Phi).  E: storage of packed right-hand
// sides, and compute type of the plain engines; Q: compute type of the
// split-K reductions over grid rows; SPLIT: split engine or -1.
template <int PREC>
struct Prec;
template <>
struct Prec<ISDF_P_FP64> {
  typedef double E;
  typedef double Q;
  static constexpr int SPLIT = -1;
};
template <>
struct Prec<ISDF_P_FP32> {
  typedef float E;
  typedef float Q;
  static constexpr int SPLIT = -1;
};
template <>
struct Prec<ISDF_P_BF16X6> {
  typedef double E;
  typedef float Q;
  static constexpr int SPLIT = SPLIT_BF16X6;
};
template <>
struct Prec<ISDF_P_FP16X3> {
  typedef double E;
  typedef float Q;
  static constexpr int SPLIT = SPLIT_FP16X3;
};

// Slices between FP64 folds of the leading accumulator.
constexpr int SPLIT_FLUSH = 2;

// Output tile of the one-operand-pair split products: 128 x 128 with eight
// wavefronts of 64 x 32 (one workgroup per CU at two wavefronts per SIMD).
// Against 128 x 64 tiles of four wavefronts each operand panel serves twice
// the outputs, and the 512 threads stage a slice with half the registers
// each; bitwise the same products.
template <int MODE>
struct SplitTile {
  static constexpr int BM = 128, BN = 128, WM = 2, WN = 4;
};

// lower_only (M = N): only the tiles that reach the lower triangle, for
// symmetric products whose upper triangle is mirrored afterwards.
template <int MODE, int BM, int BN, int WM, int WN, int NOPS, class Epi>
static bool launch_split(int M, int N, int64_t K, PlaneOp<typename SplitT<MODE>::P> A0,
                         PlaneOp<typename SplitT<MODE>::P> B0, PlaneOp<typename SplitT<MODE>::P> A1,
                         PlaneOp<typename SplitT<MODE>::P> B1, int64_t K1, const double* scales, const Epi& epi,
                         const int* abort, hipStream_t st, int lower_only = 0, int splits = 1) {
  static_assert(BM % BN == 0, "tile");
  if (M <= 0 || N <= 0) return true;
  GemmShape sh{};
  sh.M = M;
  sh.N = N;
  sh.K = K;
  sh.splits = NOPS == 1 && splits > 1 ? splits : 1;
  sh.kchunk = sh.splits > 1 ? ceil_div(ceil_div(K, sh.splits), 32) * 32 : K;  // whole 32-deep slices
  sh.lower_only = lower_only && M == N;
  sh.abort = abort;
  const int64_t tiles = split_tiles((int)ceil_div(M, BM), (int)ceil_div(N, BN), BM / BN, sh.lower_only) * sh.splits;
  hipLaunchKernelGGL((gemm_split_kernel<MODE, BM, BN, WM, WN, NOPS, SPLIT_FLUSH, Epi>), dim3((unsigned)tiles),
                     dim3(WM * WN * ISDF_WAVE), 0, st, sh, A0, B0, A1, B1, K1, scales, epi);
  return launch_ok();
}

// Plane buffers of the split engines (16-bit parts, K padded to 32).
struct SplitWork {
  void* rows_a;      // parts of orbital rows of Phi  [NP][rows_cap][ldp_a]
  void* rows_b;      //                     of Psi    [NP][rows_cap][ldp_b]
  void* e_a;         // parts of the packed Gram right-hand side of Phi [NP][e_rows][ldp_a]
  void* e_b;         //                                          of Psi
  int ldp_a, ldp_b;  // row pitch of the planes
  int k_a, k_b;      // K extent: 2 n rounded up to 32
  int64_t rows_cap;
  int e_rows;        // 2 N_mu rounded up to 32
};

// K extent of the planes of an n-column complex operand (2 n reals rounded
// up to 32) and their row pitch (the same; see ldk_of for a padded pitch).
static inline int kext_of(int n) { return (int)ceil_div(2 * (int64_t)n, 32) * 32; }
static inline int ldp_of(int n) { return kext_of(n); }
static inline size_t plane_bytes(int np, int64_t rows, int ldp) { return (size_t)np * rows * ldp * 2; }

template <int MODE, class TS>
static bool split_rows(const TS* x, int64_t ld, int n, const int* gather, int64_t nr_src, int64_t r0, int rows,
                       void* out, int ldp, int64_t rows_cap, const double* scale, hipStream_t s) {
  if (rows <= 0) return true;
  const int64_t work = (int64_t)rows * (ldp / 8);
  int64_t blocks = ceil_div(work, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((split_planes<MODE, TS>), dim3((unsigned)blocks), dim3(256), 0, s, x, ld, n, gather, nr_src, r0,
                     rows, (typename SplitT<MODE>::P*)out, ldp, rows_cap * ldp, scale);
  return launch_ok();
}

// Largest |real or imaginary part| of an r-major complex matrix, folded into
// *out (positive doubles order like their bit patterns).
template <class TS>
__global__ void absmax_rows(const TS* __restrict__ x, int64_t ld, int n, int64_t nr, double* out) {
  double m = 0.0;
  for (int64_t r = blockIdx.x; r < nr; r += gridDim.x)
    for (int k = threadIdx.x; k < 2 * n; k += blockDim.x) m = fmax(m, fabs((double)x[2 * r * ld + k]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, ISDF_WAVE));
  if ((threadIdx.x & 63) == 0 && m > 0.0) atomic_max_pos(out, m);
}

// scale[i] = 2^e with amax[src[i]] 2^e <= 2^14 (binary16 operands).
__global__ void pow2_scales(const double* amax, double* scale, int a0, int a1, int a2, int a3) {
  scale[0] = pow2_scale_for(amax[a0]);
  scale[1] = pow2_scale_for(amax[a1]);
  scale[2] = pow2_scale_for(amax[a2]);
  scale[3] = pow2_scale_for(amax[a3]);
}

template <class TS>
static bool absmax(const TS* x, int64_t ld, int n, int64_t nr, double* out, hipStream_t s) {
  int64_t blocks = nr < 2048 ? nr : 2048;
  hipLaunchKernelGGL((absmax_rows<TS>), dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, x, ld, n, nr, out);
  return launch_ok();
}

// Operand scales of the Gram blocks: sc[0..3] = (Phi, E_phi, Psi, E_psi);
// amax[0], amax[1] receive max |Phi|, max |Psi|.  Only the FP16 split uses
// them; the other precisions pass null scales.
template <int PREC, class TS>
static bool gram_scales(const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                        bool aliased, int64_t nr, double* amax, double* sc, hipStream_t s) {
  if (Prec<PREC>::SPLIT != SPLIT_FP16X3) return true;
  if (!fill<double>(amax, 2, 0.0, s)) return false;
  if (!absmax<TS>(phi, ld_phi, n_phi, nr, amax, s)) return false;
  if (!aliased && !absmax<TS>(psi, ld_psi, n_psi, nr, amax + 1, s)) return false;
  hipLaunchKernelGGL(pow2_scales, dim3(1), dim3(1), 0, s, (const double*)amax, sc, 0, 0, aliased ? 0 : 1,
                     aliased ? 0 : 1);
  return launch_ok();
}

// Operand scales of a Gram product over the rows [r0, r0 + rows) only
// (FP16 split; a power of two per operand, so any bound of its magnitude
// will do): sc[0], sc[2] for those rows of Phi and Psi, sc[1], sc[3] for the
// packed right-hand sides E_phi, E_psi (the interpolation rows), whose
// maxima land in amax[2], amax[3]; amax[0], amax[1] receive the rows'.
template <int PREC, class TS>
static bool gram_scales_rows(const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                             bool aliased, int64_t r0, int64_t rows, const double* Ephi, const double* Epsi,
                             int nmu16, double* amax, double* sc, hipStream_t s) {
  if (Prec<PREC>::SPLIT != SPLIT_FP16X3) return true;
  if (!fill<double>(amax, 4, 0.0, s)) return false;
  if (rows > 0 && !absmax<TS>(phi + 2 * r0 * ld_phi, ld_phi, n_phi, rows, amax, s)) return false;
  if (!absmax<double>(Ephi, n_phi, n_phi, 2 * (int64_t)nmu16, amax + 2, s)) return false;
  if (!aliased) {
    if (rows > 0 && !absmax<TS>(psi + 2 * r0 * ld_psi, ld_psi, n_psi, rows, amax + 1, s)) return false;
    if (!absmax<double>(Epsi, n_psi, n_psi, 2 * (int64_t)nmu16, amax + 3, s)) return false;
  }
  hipLaunchKernelGGL(pow2_scales, dim3(1), dim3(1), 0, s, (const double*)amax, sc, 0, 2, aliased ? 0 : 1,
                     aliased ? 2 : 3);
  return launch_ok();
}

// Gram + Hadamard of `rows` orbital rows (gathered through `gather` if
// non-null, else starting at row r0) into G (and optionally A, B).
template <int PREC, class TS>
static bool gram(const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi, bool aliased,
                 const typename Prec<PREC>::E* Ephi, const typename Prec<PREC>::E* Epsi, int nmu16, int n_mu,
                 const int* gather, int64_t nr, int64_t r0, int rows, double* G, int64_t ldg, int mode,
                 const int* abort, hipStream_t s, const double* scales, const SplitWork* sw, double* Aout = nullptr,
                 double* Bout = nullptr) {
  typedef typename Prec<PREC>::E T;
  constexpr int SPLIT = Prec<PREC>::SPLIT;
  EpiGram epi{G, ldg, rows, n_mu, mode, Aout, Bout, 2 * (int64_t)n_mu};
  const int N = 2 * nmu16;
  Operand<TS> a0{phi + 2 * r0 * ld_phi, 2 * ld_phi, gather, nullptr};
  Operand<T> b0{Ephi, 2 * (int64_t)n_phi, nullptr, nullptr};
  Operand<TS> a1{psi + 2 * r0 * ld_psi, 2 * ld_psi, gather, nullptr};
  Operand<T> b1{Epsi, 2 * (int64_t)n_psi, nullptr, nullptr};
  if constexpr (SPLIT >= 0) {
    typedef typename SplitT<SPLIT>::P P;
    const double* sc = SPLIT == SPLIT_FP16X3 ? scales : nullptr;
    if (!split_rows<SPLIT, TS>(phi, ld_phi, n_phi, gather, nr, gather ? 0 : r0, rows, sw->rows_a, sw->ldp_a,
                               sw->rows_cap, sc, s))
      return false;
    PlaneOp<P> pa0{(const P*)sw->rows_a, sw->ldp_a, sw->rows_cap * sw->ldp_a, nullptr};
    PlaneOp<P> pb0{(const P*)sw->e_a, sw->ldp_a, (int64_t)sw->e_rows * sw->ldp_a, nullptr};
    if (aliased)
      return launch_split<SPLIT, SplitTile<SPLIT>::BM, SplitTile<SPLIT>::BN, SplitTile<SPLIT>::WM,
                          SplitTile<SPLIT>::WN, 1>(rows, N, sw->k_a, pa0, pb0, pa0, pb0, 0, sc, epi, abort, s);
    if (!split_rows<SPLIT, TS>(psi, ld_psi, n_psi, gather, nr, gather ? 0 : r0, rows, sw->rows_b, sw->ldp_b,
                               sw->rows_cap, sc ? sc + 2 : nullptr, s))
      return false;
    PlaneOp<P> pa1{(const P*)sw->rows_b, sw->ldp_b, sw->rows_cap * sw->ldp_b, nullptr};
    PlaneOp<P> pb1{(const P*)sw->e_b, sw->ldp_b, (int64_t)sw->e_rows * sw->ldp_b, nullptr};
    return launch_split<SPLIT, 64, 64, 2, 2, 2>(rows, N, sw->k_a, pa0, pb0, pa1, pb1, sw->k_b, sc, epi, abort, s);
  } else {
    // FP32: accumulators folded into FP64 every 2 steps (32-deep)
    constexpr int FOLD = sizeof(T) == 4 ? 2 : 0;
    if (aliased)
      return launch_gemm<T, 128, 128, 16, 2, 2, TS, KC, T, KC, 1, FOLD>(rows, N, 2 * (int64_t)n_phi, a0, b0, a0, b0,
                                                                         0, epi, 0, abort, s);
    return launch_gemm<T, 128, 64, 16, 2, 2, TS, KC, T, KC, 2, FOLD>(rows, N, 2 * (int64_t)n_phi, a0, b0, a1, b1,
                                                                      2 * (int64_t)n_psi, epi, 0, abort, s);
  }
}

// F[n][k] (n = 2 i + c', k = 2 nu + c): real form of right-multiplication by
// Phi_mu, (x + iy)(a + ib) = (xa - yb) + i(xb + ya) with Phi_mu[nu][i] = a + ib.
template <class TS, class T>
__global__ void pack_adj_rhs(const TS* __restrict__ phi, int64_t ld, int n, const int32_t* __restrict__ idx,
                             int n_mu, int64_t nr, T* __restrict__ F) {
  const int64_t total = (int64_t)2 * n * 2 * n_mu;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / (2 * n_mu)), k = (int)(e % (2 * n_mu));
    const int i = row >> 1, cp = row & 1, nu = k >> 1, c = k & 1;
    int64_t p = idx[nu];
    if (p < 0 || p >= nr) p = 0;
    const double2 z = Cplx<TS>::load(phi + 2 * (p * ld + i));
    double v;
    if (cp == 0) v = c == 0 ? z.x : -z.y;
    else v = c == 0 ? z.y : z.x;
    F[e] = (T)v;
  }
}

template <class TS, class T>
static bool pack(const TS* phi, int64_t ld, int n, const int* idx, int n_mu, int64_t nr, int nmu16, T* E,
                 hipStream_t s) {
  const int64_t total = (int64_t)2 * nmu16 * 2 * n;
  int64_t blocks = ceil_div(total, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((pack_gram_rhs<TS, T>), dim3((unsigned)blocks), dim3(256), 0, s, phi, ld, n, idx, n_mu, nr,
                     2 * nmu16, E);
  return launch_ok();
}

// Parts of the packed Gram right-hand sides (split precisions only).
template <int PREC>
static bool split_rhs(const double* Ephi, const double* Epsi, int n_phi, int n_psi, bool aliased,
                      const double* scales, const SplitWork* sw, hipStream_t s) {
  constexpr int SPLIT = Prec<PREC>::SPLIT;
  if constexpr (SPLIT >= 0) {
    const double* sc = SPLIT == SPLIT_FP16X3 ? scales : nullptr;
    if (!split_rows<SPLIT, double>(Ephi, n_phi, n_phi, nullptr, sw->e_rows, 0, sw->e_rows, sw->e_a, sw->ldp_a,
                                   sw->e_rows, sc ? sc + 1 : nullptr, s))
      return false;
    if (!aliased && !split_rows<SPLIT, double>(Epsi, n_psi, n_psi, nullptr, sw->e_rows, 0, sw->e_rows, sw->e_b,
                                               sw->ldp_b, sw->e_rows, sc ? sc + 3 : nullptr, s))
      return false;
  }
  return true;
}

// Carves the plane buffers of a split precision (no-op otherwise).
static SplitWork carve_split(Carver& c, isdf_prec prec, int n_phi, int n_psi, bool aliased, int n_mu,
                             int64_t rows_cap) {
  SplitWork w{};
  if (prec != ISDF_P_BF16X6 && prec != ISDF_P_FP16X3) return w;
  const int np = prec == ISDF_P_BF16X6 ? 3 : 2;
  w.ldp_a = ldp_of(n_phi);
  w.ldp_b = ldp_of(n_psi);
  w.k_a = kext_of(n_phi);
  w.k_b = kext_of(n_psi);
  w.rows_cap = rows_cap;
  w.e_rows = (int)ceil_div(2 * (int64_t)ceil_div(n_mu, 16) * 16, 32) * 32;
  w.rows_a = c.take<char>(plane_bytes(np, rows_cap, w.ldp_a));
  w.e_a = c.take<char>(plane_bytes(np, w.e_rows, w.ldp_a));
  if (!aliased) {
    w.rows_b = c.take<char>(plane_bytes(np, rows_cap, w.ldp_b));
    w.e_b = c.take<char>(plane_bytes(np, w.e_rows, w.ldp_b));
  }
  return w;
}

static bool fit_args_ok(const isdf_grid* g, isdf_dtype dt, const void* phi, int64_t ld_phi, int n_phi,
                        const void* psi, int64_t ld_psi, int n_psi, const int32_t* idx, int n_mu, isdf_prec prec,
                        int64_t* nr_out) {
  if (!g) return false;
  for (int a = 0; a < 3; ++a)
    if (g->n[a] <= 0) return false;
  const int64_t nr = (int64_t)g->n[0] * g->n[1] * g->n[2];
  if (nr >= INT32_MAX) return false;
  if (dt != ISDF_C128 && dt != ISDF_C64) return false;
  if (!phi || !psi || !idx || n_phi <= 0 || n_psi <= 0 || ld_phi < n_phi || ld_psi < n_psi) return false;
  if (n_mu <= 0 || n_mu > nr) return false;
  if (prec < ISDF_P_FP64 || prec > ISDF_P_FP16X3) return false;
  *nr_out = nr;
  return true;
}

// Bytes per element of the packed right-hand sides (E, F) and gathered
// rows: the FP32 engine stages them in float, every other precision in
// double (the split engines split them while staging).
static size_t tsize_of(isdf_prec p) { return p == ISDF_P_FP32 ? sizeof(float) : sizeof(double); }

}  // namespace
}  // namespace isdf
