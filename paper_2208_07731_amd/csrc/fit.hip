// Least-squares fit of the interpolation vectors (Sec. 2.1, eqs. decomMatrix,
// theta, muRownuCol, muRownuColden and the solver of Sec. 2.4 of
// arXiv:2208.07731):
//
//   Theta = G M^-1,  G = Z C^H = A .* conj(B),  A = Phi Phi_mu^H,  B = Psi Psi_mu^H,
//   M = C C^H = G[idx, :]  (Hermitian positive definite).
//
// Complex arithmetic is carried as real GEMMs on MFMA:
//  * Gram blocks: the orbital rows, read in place as real rows
//    (re_0, im_0, re_1, im_1, ...), times a packed coefficient matrix E built
//    from Phi_mu whose rows give Re A and Im A of the same column nu in two
//    16-column blocks, so that one lane holds both and the Hadamard product
//    with conj(B) happens in registers (epilogue), never in memory.
//  * M and its inverse: the complex case uses the real 2x2-block form
//    [[re, im], [-im, re]] of every entry, a real symmetric positive definite
//    matrix of order 2 N_mu whose inverse is the block form of M^-1; the
//    aliased case (Psi = Phi) is real from the start.
//  * Cholesky M = L L^T (blocked, 64-wide diagonal blocks factored and
//    inverted in LDS, panel and trailing updates on the FP64 GEMM), then
//    L^-1 by block forward substitution and M^-1 = L^-T L^-1.
//  * Theta rows = G rows times M^-1 (FP64 GEMM), one r-block at a time.
#include "fitlib.h"

namespace isdf {

struct FitPlan {
  FitState* st;
  double* amax;  // [2] max |Phi|, max |Psi|
  double* sc;    // [4] binary16 operand scales of the Gram blocks
  int* marker;
  void* Ephi;
  void* Epsi;
  InvWork inv;
  double* G;
  SplitWork sw;
  double* Th;    // residual mode: Theta of one r-block (FP64)
  double* part;  // residual mode: per-workgroup (||Z||^2 - Re G.Theta, ||Z||^2) pairs
  size_t bytes;
};

constexpr int RESID_BLOCKS = 512;  // workgroups per r-block of the residual reduction

static FitPlan plan_fit(void* ws, size_t cap, int64_t nr, int n_mu, int n_phi, int n_psi, bool aliased,
                        isdf_prec prec, int64_t rblock, bool resid = false) {
  const size_t tsize = tsize_of(prec);
  Carver c(ws, cap);
  FitPlan P{};
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  const int n1 = aliased ? n_mu : 2 * n_mu;
  P.st = c.take<FitState>(1);
  P.amax = c.take<double>(2);
  P.sc = c.take<double>(4);
  P.marker = c.take<int>(nr);
  P.Ephi = c.take<char>((size_t)2 * nmu16 * 2 * n_phi * tsize);
  P.Epsi = aliased ? nullptr : c.take<char>((size_t)2 * nmu16 * 2 * n_psi * tsize);
  P.inv.Y = c.take<double>((size_t)n1 * n1);
  P.inv.R = c.take<double>((size_t)n1 * n1);
  P.G = c.take<double>((size_t)rblock * n1);
  P.sw = carve_split(c, prec, n_phi, n_psi, aliased, n_mu, rblock > n_mu ? rblock : n_mu);
  if (resid) {
    P.Th = c.take<double>((size_t)rblock * n1);
    P.part = c.take<double>((size_t)2 * RESID_BLOCKS * ceil_div(nr, rblock));
  }
  P.bytes = c.used;
  return P;
}

// Residual terms of rows [r0, r0 + rows): per row, with G and Theta read as
// n1 reals (Re G conj(Theta) summed over nu is their dot product),
// ||Z(r)||^2 = rho_phi(r) rho_psi(r); pairs (||Z(r)||^2 - dot, ||Z(r)||^2)
// summed per workgroup into part.
template <class TS>
__global__ __launch_bounds__(PAIR_THREADS) void fit_resid_rows(const double* __restrict__ G,
                                                               const double* __restrict__ Th, int rows, int n1,
                                                               const TS* __restrict__ phi, int64_t ldp, int nphi,
                                                               const TS* __restrict__ psi, int64_t lds, int npsi,
                                                               int aliased, int64_t r0, double* __restrict__ part) {
  const int lane = threadIdx.x & (ISDF_WAVE - 1);
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / ISDF_WAVE;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / ISDF_WAVE;
  double acc = 0.0, zz = 0.0;
  for (int64_t q = wave; q < rows; q += nwaves) {
    double dot = 0.0, rp = 0.0, rs = 0.0;
    for (int k = lane; k < n1; k += ISDF_WAVE) dot += G[q * n1 + k] * Th[q * n1 + k];
    const int64_t r = r0 + q;
    for (int i = lane; i < nphi; i += ISDF_WAVE) {
      const double2 z = Cplx<TS>::load(phi + 2 * (r * ldp + i));
      rp += z.x * z.x + z.y * z.y;
    }
    if (!aliased)
      for (int j = lane; j < npsi; j += ISDF_WAVE) {
        const double2 z = Cplx<TS>::load(psi + 2 * (r * lds + j));
        rs += z.x * z.x + z.y * z.y;
      }
    dot = wave_sum(dot);
    rp = wave_sum(rp);
    rs = aliased ? rp : wave_sum(rs);
    acc += rp * rs - dot;
    zz += rp * rs;
  }
  if (lane != 0) acc = zz = 0.0;
  block_pair_store(acc, zz, part);
}

template <int PREC, class TS, class TT>
static int fit_run(int64_t nr, const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                   bool aliased, const int32_t* idx, int n_mu, double* minv, uint32_t flags, int64_t row0,
                   int64_t nrows, TT* theta, int64_t ld_theta, int64_t rblock, isdf_fit_info* info,
                   const FitPlan& P, hipStream_t s) {
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  const int n1 = aliased ? n_mu : 2 * n_mu;
  const int* ab = &P.st->abort;
  typedef typename Prec<PREC>::E T;
  hipLaunchKernelGGL(fit_state_init, dim3(1), dim3(1), 0, s, P.st);
  if (!launch_ok()) return ISDF_E_HIP;
  T* Ephi = (T*)P.Ephi;
  T* Epsi = aliased ? Ephi : (T*)P.Epsi;
  if (!pack<TS, T>(phi, ld_phi, n_phi, idx, n_mu, nr, nmu16, Ephi, s)) return ISDF_E_HIP;
  if (!aliased && !pack<TS, T>(psi, ld_psi, n_psi, idx, n_mu, nr, nmu16, Epsi, s)) return ISDF_E_HIP;
  if (!gram_scales<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, nr, P.amax, P.sc, s)) return ISDF_E_HIP;
  if (!split_rhs<PREC>((const double*)Ephi, (const double*)Epsi, n_phi, n_psi, aliased, P.sc, &P.sw, s))
    return ISDF_E_HIP;
  if (flags & ISDF_FIT_FACTOR) {
    if (!fill<int>(P.marker, nr, 0, s)) return ISDF_E_HIP;
    hipLaunchKernelGGL(check_idx, dim3((unsigned)ceil_div(n_mu, 256)), dim3(256), 0, s, idx, n_mu, nr, P.marker,
                       P.st);
    if (!launch_ok()) return ISDF_E_HIP;
    // M = C C^H: the Gram + Hadamard of the interpolation rows themselves
    if (!gram<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, Ephi, Epsi, nmu16, n_mu, idx, nr, 0, n_mu,
                        minv, n1, aliased ? G_REAL : G_EMB, ab, s, P.sc, &P.sw))
      return ISDF_E_HIP;
    ISDF_TRY(spd_inverse(minv, n1, P.inv, P.st, s));
  }
  for (int64_t r = 0; r < nrows; r += rblock) {
    const int rows = (int)(nrows - r < rblock ? nrows - r : rblock);
    if (!gram<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, Ephi, Epsi, nmu16, n_mu, nullptr, nr,
                        row0 + r, rows, P.G, n1, aliased ? G_REAL : G_CPLX, ab, s, P.sc, &P.sw))
      return ISDF_E_HIP;
    const int64_t ldt = aliased ? ld_theta : 2 * ld_theta;
    if (!dgemm<KC, KC, TT>(rows, n1, n1, P.G, n1, minv, n1, theta + r * ldt, ldt, 1.0, 0.0, 0, ab, s))
      return ISDF_E_HIP;
  }
  hipLaunchKernelGGL(fit_finish, dim3(1), dim3(1), 0, s, P.st, info, (double*)nullptr, 0);
  if (!launch_ok()) return ISDF_E_HIP;
  return ISDF_OK;
}

// ||Z - Theta C||_F^2 and ||Z||_F^2 for the Theta of (C C^H)^-1 = minv, r-block
// by r-block: Gram + Hadamard, Theta = G minv (FP64), row terms, fixed-order sums.
template <int PREC, class TS>
static int resid_run(int64_t nr, const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                     bool aliased, const int32_t* idx, int n_mu, const double* minv, int64_t rblock, double* out,
                     isdf_fit_info* info, const FitPlan& P, hipStream_t s) {
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  const int n1 = aliased ? n_mu : 2 * n_mu;
  const int* ab = &P.st->abort;
  typedef typename Prec<PREC>::E T;
  hipLaunchKernelGGL(fit_state_init, dim3(1), dim3(1), 0, s, P.st);
  if (!launch_ok()) return ISDF_E_HIP;
  T* Ephi = (T*)P.Ephi;
  T* Epsi = aliased ? Ephi : (T*)P.Epsi;
  if (!pack<TS, T>(phi, ld_phi, n_phi, idx, n_mu, nr, nmu16, Ephi, s)) return ISDF_E_HIP;
  if (!aliased && !pack<TS, T>(psi, ld_psi, n_psi, idx, n_mu, nr, nmu16, Epsi, s)) return ISDF_E_HIP;
  if (!gram_scales<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, nr, P.amax, P.sc, s)) return ISDF_E_HIP;
  if (!split_rhs<PREC>((const double*)Ephi, (const double*)Epsi, n_phi, n_psi, aliased, P.sc, &P.sw, s))
    return ISDF_E_HIP;
  int64_t blk = 0;
  for (int64_t r = 0; r < nr; r += rblock, ++blk) {
    const int rows = (int)(nr - r < rblock ? nr - r : rblock);
    if (!gram<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, Ephi, Epsi, nmu16, n_mu, nullptr, nr, r, rows,
                        P.G, n1, aliased ? G_REAL : G_CPLX, ab, s, P.sc, &P.sw))
      return ISDF_E_HIP;
    if (!dgemm<KC, KC, double>(rows, n1, n1, P.G, n1, minv, n1, P.Th, n1, 1.0, 0.0, 0, ab, s)) return ISDF_E_HIP;
    hipLaunchKernelGGL((fit_resid_rows<TS>), dim3(RESID_BLOCKS), dim3(PAIR_THREADS), 0, s, (const double*)P.G,
                       (const double*)P.Th, rows, n1, phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased ? 1 : 0, r,
                       P.part + 2 * RESID_BLOCKS * blk);
    if (!launch_ok()) return ISDF_E_HIP;
  }
  hipLaunchKernelGGL(sum_pairs, dim3(1), dim3(PAIR_THREADS), 0, s, (const double*)P.part,
                     (int)(RESID_BLOCKS * blk), out);
  hipLaunchKernelGGL(fit_finish, dim3(1), dim3(1), 0, s, P.st, info, (double*)nullptr, 0);
  if (!launch_ok()) return ISDF_E_HIP;
  return ISDF_OK;
}

}  // namespace isdf

using namespace isdf;

extern "C" size_t isdf_fit_residual_workspace(const isdf_grid* grid, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                                              int32_t aliased, int32_t prec_in, int64_t rblock) {
  if (!prec_valid(prec_in)) return 0;
  const isdf_prec prec = (isdf_prec)prec_in;
  if (!grid || n_mu <= 0 || n_phi <= 0 || n_psi <= 0 || rblock <= 0) return 0;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (nr <= 0) return 0;
  if (rblock > nr) rblock = nr;
  return plan_fit(nullptr, 0, nr, n_mu, n_phi, n_psi, aliased != 0, prec, rblock, true).bytes;
}

extern "C" int isdf_fit_residual(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi,
                                 int32_t n_phi, const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx,
                                 int32_t n_mu, int32_t prec_in, const double* minv, int64_t rblock, double* out,
                                 isdf_fit_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  if (!prec_valid(prec_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const isdf_prec prec = (isdf_prec)prec_in;
  int64_t nr = 0;
  if (!fit_args_ok(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, &nr)) return ISDF_E_ARG;
  if (!minv || !out || !info || rblock <= 0) return ISDF_E_ARG;
  if (prec == ISDF_P_FP64 && dt != ISDF_C128) return ISDF_E_ARG;
  if (rblock > nr) rblock = nr;
  if (ceil_div(nr, rblock) * RESID_BLOCKS > INT32_MAX) return ISDF_E_ARG;
  const bool aliased = phi == psi && ld_phi == ld_psi && n_phi == n_psi;
  FitPlan P = plan_fit(ws, ws_bytes, nr, n_mu, n_phi, n_psi, aliased, prec, rblock, true);
  if (!ws || P.bytes > ws_bytes) return ISDF_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
#define ISDF_RES_ARGS(TS) \
  nr, (const TS*)phi, ld_phi, n_phi, (const TS*)psi, ld_psi, n_psi, aliased, idx, n_mu, minv, rblock, out, info, P, s
  if (dt == ISDF_C128) {
    switch (prec) {
      case ISDF_P_FP64: return resid_run<ISDF_P_FP64, double>(ISDF_RES_ARGS(double));
      case ISDF_P_FP32: return resid_run<ISDF_P_FP32, double>(ISDF_RES_ARGS(double));
      case ISDF_P_BF16X6: return resid_run<ISDF_P_BF16X6, double>(ISDF_RES_ARGS(double));
      default: return resid_run<ISDF_P_FP16X3, double>(ISDF_RES_ARGS(double));
    }
  }
  switch (prec) {
    case ISDF_P_FP32: return resid_run<ISDF_P_FP32, float>(ISDF_RES_ARGS(float));
    case ISDF_P_BF16X6: return resid_run<ISDF_P_BF16X6, float>(ISDF_RES_ARGS(float));
    default: return resid_run<ISDF_P_FP16X3, float>(ISDF_RES_ARGS(float));
  }
#undef ISDF_RES_ARGS
}

extern "C" size_t isdf_fit_minv_elems(int32_t n_mu, int32_t aliased) {
  if (n_mu <= 0) return 0;
  const size_t n1 = aliased ? (size_t)n_mu : 2 * (size_t)n_mu;
  return n1 * n1;
}

extern "C" size_t isdf_fit_workspace(const isdf_grid* grid, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                                     int32_t aliased, int32_t prec_in, int64_t rblock) {
  if (!prec_valid(prec_in)) return 0;
  const isdf_prec prec = (isdf_prec)prec_in;
  if (!grid || n_mu <= 0 || n_phi <= 0 || n_psi <= 0 || rblock <= 0) return 0;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (nr <= 0) return 0;
  return plan_fit(nullptr, 0, nr, n_mu, n_phi, n_psi, aliased != 0, prec, rblock).bytes;
}

extern "C" int isdf_fit(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi, int32_t n_phi,
                        const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx, int32_t n_mu,
                        int32_t prec_in, double* minv, uint32_t flags, int64_t row0, int64_t nrows, void* theta,
                        int64_t ld_theta, int64_t rblock, isdf_fit_info* info, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  if (!prec_valid(prec_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const isdf_prec prec = (isdf_prec)prec_in;
  int64_t nr = 0;
  if (!fit_args_ok(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, &nr)) return ISDF_E_ARG;
  if (flags & ~ISDF_FIT_FACTOR) return ISDF_E_ARG;
  if (!minv || !info || (nrows > 0 && !theta) || row0 < 0 || nrows < 0 || row0 + nrows > nr) return ISDF_E_ARG;
  if (ld_theta < n_mu || rblock <= 0) return ISDF_E_ARG;
  if (prec == ISDF_P_FP64 && dt != ISDF_C128) return ISDF_E_ARG;
  const bool aliased = phi == psi && ld_phi == ld_psi && n_phi == n_psi;
  FitPlan P = plan_fit(ws, ws_bytes, nr, n_mu, n_phi, n_psi, aliased, prec, rblock);
  if (!ws || P.bytes > ws_bytes) return ISDF_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
#define ISDF_FIT_ARGS(TS, TT)                                                                                   \
  nr, (const TS*)phi, ld_phi, n_phi, (const TS*)psi, ld_psi, n_psi, aliased, idx, n_mu, minv, flags, row0, nrows, \
      (TT*)theta, ld_theta, rblock, info, P, s
  if (dt == ISDF_C128) {
    switch (prec) {
      case ISDF_P_FP64: return fit_run<ISDF_P_FP64, double, double>(ISDF_FIT_ARGS(double, double));
      case ISDF_P_FP32: return fit_run<ISDF_P_FP32, double, double>(ISDF_FIT_ARGS(double, double));
      case ISDF_P_BF16X6: return fit_run<ISDF_P_BF16X6, double, double>(ISDF_FIT_ARGS(double, double));
      default: return fit_run<ISDF_P_FP16X3, double, double>(ISDF_FIT_ARGS(double, double));
    }
  }
  switch (prec) {
    case ISDF_P_FP32: return fit_run<ISDF_P_FP32, float, float>(ISDF_FIT_ARGS(float, float));
    case ISDF_P_BF16X6: return fit_run<ISDF_P_BF16X6, float, float>(ISDF_FIT_ARGS(float, float));
    default: return fit_run<ISDF_P_FP16X3, float, float>(ISDF_FIT_ARGS(float, float));
  }
#undef ISDF_FIT_ARGS
}

// Workspace layout of isdf_zc (the size query and the call share it).
struct ZcPlan {
  int* ab;
  double* amax;
  double* sc;
  void* Ephi;
  void* Epsi;
  SplitWork sw;
  size_t bytes;
};

static ZcPlan plan_zc(void* ws, size_t cap, int n_mu, int n_phi, int n_psi, bool aliased, isdf_prec prec,
                      int64_t nrows) {
  Carver c(ws, cap);
  ZcPlan P{};
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  P.ab = c.take<int>(64);
  P.amax = c.take<double>(4);
  P.sc = c.take<double>(4);
  P.Ephi = c.take<char>((size_t)2 * nmu16 * 2 * n_phi * tsize_of(prec));
  P.Epsi = aliased ? P.Ephi : c.take<char>((size_t)2 * nmu16 * 2 * n_psi * tsize_of(prec));
  P.sw = carve_split(c, prec, n_phi, n_psi, aliased, n_mu, nrows > 0 ? nrows : 1);
  P.bytes = c.used;
  return P;
}

extern "C" size_t isdf_zc_workspace(int32_t n_mu, int32_t n_phi, int32_t n_psi, int32_t aliased, int32_t prec_in,
                                    int64_t nrows) {
  if (!prec_valid(prec_in)) return 0;
  const isdf_prec prec = (isdf_prec)prec_in;
  if (n_mu <= 0 || n_phi <= 0 || n_psi <= 0 || nrows < 0) return 0;
  return plan_zc(nullptr, 0, n_mu, n_phi, n_psi, aliased != 0, prec, nrows).bytes;
}

template <int PREC, class TS>
static int zc_run(int64_t nr, const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                  bool aliased, const int32_t* idx, int n_mu, int64_t row0, int64_t nrows, double* G, int64_t ldg,
                  double* A, double* B, const ZcPlan& P, hipStream_t s) {
  typedef typename Prec<PREC>::E T;
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  T* Ephi = (T*)P.Ephi;
  T* Epsi = (T*)P.Epsi;
  if (!fill<int>(P.ab, 1, 0, s)) return ISDF_E_HIP;
  if (!pack<TS, T>(phi, ld_phi, n_phi, idx, n_mu, nr, nmu16, Ephi, s)) return ISDF_E_HIP;
  if (!aliased && !pack<TS, T>(psi, ld_psi, n_psi, idx, n_mu, nr, nmu16, Epsi, s)) return ISDF_E_HIP;
  // binary16 scales from this call's rows and the interpolation rows only
  // (a pass over the whole grid per block would cost as much as the block)
  if (!gram_scales_rows<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, row0, nrows, (const double*)Ephi,
                                  (const double*)Epsi, nmu16, P.amax, P.sc, s))
    return ISDF_E_HIP;
  if (!split_rhs<PREC>((const double*)Ephi, (const double*)Epsi, n_phi, n_psi, aliased, P.sc, &P.sw, s))
    return ISDF_E_HIP;
  if (nrows > 0 && !gram<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, Ephi, Epsi, nmu16, n_mu, nullptr,
                                   nr, row0, (int)nrows, G, ldg, aliased ? G_REAL : G_CPLX, P.ab, s, P.sc, &P.sw,
                                   A, aliased ? nullptr : B))
    return ISDF_E_HIP;
  return ISDF_OK;
}

static int zc_dispatch(const isdf_grid* grid, isdf_dtype dt, const void* phi, int64_t ld_phi, int32_t n_phi,
                       const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx, int32_t n_mu,
                       isdf_prec prec, int64_t row0, int64_t nrows, double* G, int64_t ldg, double* A, double* B,
                       bool want_ab, void* ws, size_t ws_bytes, void* stream) {
  int64_t nr = 0;
  if (!fit_args_ok(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, &nr)) return ISDF_E_ARG;
  const bool aliased = phi == psi && ld_phi == ld_psi && n_phi == n_psi;
  if (row0 < 0 || nrows < 0 || row0 + nrows > nr || nrows > INT32_MAX || (nrows > 0 && !G)) return ISDF_E_ARG;
  if (ldg < (aliased ? n_mu : 2 * (int64_t)n_mu)) return ISDF_E_ARG;
  if (want_ab && nrows > 0 && (!A || (!aliased && !B))) return ISDF_E_ARG;
  if (prec == ISDF_P_FP64 && dt != ISDF_C128) return ISDF_E_ARG;
  ZcPlan P = plan_zc(ws, ws_bytes, n_mu, n_phi, n_psi, aliased, prec, nrows);
  if (!ws || P.bytes > ws_bytes) return ISDF_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (!want_ab) A = B = nullptr;
#define ISDF_ZC_ARGS(TS) \
  nr, (const TS*)phi, ld_phi, n_phi, (const TS*)psi, ld_psi, n_psi, aliased, idx, n_mu, row0, nrows, G, ldg, A, B, P, s
  if (dt == ISDF_C128) {
    switch (prec) {
      case ISDF_P_FP64: return zc_run<ISDF_P_FP64, double>(ISDF_ZC_ARGS(double));
      case ISDF_P_FP32: return zc_run<ISDF_P_FP32, double>(ISDF_ZC_ARGS(double));
      case ISDF_P_BF16X6: return zc_run<ISDF_P_BF16X6, double>(ISDF_ZC_ARGS(double));
      default: return zc_run<ISDF_P_FP16X3, double>(ISDF_ZC_ARGS(double));
    }
  }
  switch (prec) {
    case ISDF_P_FP32: return zc_run<ISDF_P_FP32, float>(ISDF_ZC_ARGS(float));
    case ISDF_P_BF16X6: return zc_run<ISDF_P_BF16X6, float>(ISDF_ZC_ARGS(float));
    default: return zc_run<ISDF_P_FP16X3, float>(ISDF_ZC_ARGS(float));
  }
#undef ISDF_ZC_ARGS
}

extern "C" int isdf_zc(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi, int32_t n_phi,
                       const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx, int32_t n_mu,
                       int32_t prec_in, int64_t row0, int64_t nrows, double* G, int64_t ldg, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  if (!prec_valid(prec_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const isdf_prec prec = (isdf_prec)prec_in;
  return zc_dispatch(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, row0, nrows, G, ldg, nullptr,
                     nullptr, false, ws, ws_bytes, stream);
}

extern "C" int isdf_zc_ab(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi, int32_t n_phi,
                          const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx, int32_t n_mu,
                          int32_t prec_in, int64_t row0, int64_t nrows, double* G, int64_t ldg, double* A, double* B,
                          void* ws, size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  if (!prec_valid(prec_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const isdf_prec prec = (isdf_prec)prec_in;
  return zc_dispatch(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, row0, nrows, G, ldg, A, B,
                     true, ws, ws_bytes, stream);
}

extern "C" int isdf_apply_minv(int32_t n_mu, int32_t aliased, const double* minv, const double* G, int64_t ldg,
                               int64_t nrows, int32_t dt_in, void* theta, int64_t ld_theta, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const int64_t n1 = aliased ? n_mu : 2 * (int64_t)n_mu;
  if (n_mu <= 0 || !minv || nrows < 0 || nrows > INT32_MAX || (nrows > 0 && (!G || !theta))) return ISDF_E_ARG;
  if (ldg < n1 || ld_theta < n_mu || (dt != ISDF_C128 && dt != ISDF_C64)) return ISDF_E_ARG;
  if (nrows == 0) return ISDF_OK;
  hipStream_t s = (hipStream_t)stream;
  const int64_t ldt = aliased ? ld_theta : 2 * ld_theta;
  bool ok = dt == ISDF_C128
                ? dgemm<KC, KC, double>((int)nrows, (int)n1, n1, G, ldg, minv, n1, (double*)theta, ldt, 1.0, 0.0, 0,
                                        nullptr, s)
                : dgemm<KC, KC, float>((int)nrows, (int)n1, n1, G, ldg, minv, n1, (float*)theta, ldt, 1.0, 0.0, 0,
                                       nullptr, s);
  return ok ? ISDF_OK : ISDF_E_HIP;
}
