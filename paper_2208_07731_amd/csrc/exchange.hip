// ISDF-compressed exchange operator (eq. v2 of arXiv:2208.07731):
//
//   (V_X psi_j)(r) ~ - sum_mu V'_mu(r) sum_i phi_i(r) phi_i*(r_mu) psi_j(r_mu)
//                  = - [ (V' .* A) Psi_mu ](r, j),   A = Phi Phi_mu^H,
//
// with V'_mu = conj(V_mu) for V_mu the potential of the fit's Theta column
// (eq. v2 expands phi_i* psi_j, the conjugate of the pair density the fit
// interpolates).  Per r-block: A by the Gram engine (rows of A kept, no
// Hadamard with a second block), A .*= conj(V) in place, then one real-form
// GEMM with the packed Psi_mu, scaled by -1, into the caller's output.  FP64
// arithmetic for either storage type.
#include "fitlib.h"

namespace isdf {
namespace {

template <class TS>
__global__ void exch_hadamard(double* __restrict__ A, int rows, int n_mu, const TS* __restrict__ V, int64_t ld_v,
                              int v_complex, int64_t r0, const int* abort) {
  if (*abort) return;
  const int64_t total = (int64_t)rows * n_mu;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n_mu;
    const int mu = (int)(e % n_mu);
    double2 v;
    if (v_complex) v = Cplx<TS>::load(V + 2 * ((r0 + r) * ld_v + mu));
    else v = make_double2((double)V[(r0 + r) * ld_v + mu], 0.0);
    double2* a = reinterpret_cast<double2*>(A) + e;
    const double2 x = *a;
    *a = make_double2(x.x * v.x + x.y * v.y, x.y * v.x - x.x * v.y);  // x conj(v)
  }
}

struct ExchPlan {
  int* ab;
  double* Ephi;
  double* Fpsi;
  double* A;
  size_t bytes;
};

static ExchPlan plan_exch(void* ws, size_t cap, int n_mu, int n_phi, int n_psi, int64_t rblock) {
  Carver c(ws, cap);
  ExchPlan P{};
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  P.ab = c.take<int>(64);
  P.Ephi = c.take<double>((size_t)2 * nmu16 * 2 * n_phi);
  P.Fpsi = c.take<double>((size_t)2 * n_psi * 2 * n_mu);
  P.A = c.take<double>((size_t)rblock * 2 * n_mu);
  P.bytes = c.used;
  return P;
}

static unsigned grid_for(int64_t n) {
  int64_t b = ceil_div(n, 256);
  return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

template <class TS>
static int exch_run(int64_t nr, const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                    const int32_t* idx, int n_mu, const TS* V, int64_t ld_v, int v_complex, TS* W, int64_t ld_w,
                    int64_t rblock, const ExchPlan& P, hipStream_t s) {
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  if (!fill<int>(P.ab, 1, 0, s)) return ISDF_E_HIP;
  if (!pack<TS, double>(phi, ld_phi, n_phi, idx, n_mu, nr, nmu16, P.Ephi, s)) return ISDF_E_HIP;
  hipLaunchKernelGGL((pack_adj_rhs<TS, double>), dim3(grid_for((int64_t)4 * n_psi * n_mu)), dim3(256), 0, s, psi,
                     ld_psi, n_psi, idx, n_mu, nr, P.Fpsi);
  if (!launch_ok()) return ISDF_E_HIP;
  const int64_t two_mu = 2 * (int64_t)n_mu;
  for (int64_t r = 0; r < nr; r += rblock) {
    const int rows = (int)(nr - r < rblock ? nr - r : rblock);
    // A rows = Phi(r) Phi_mu^H (the Gram engine on Phi alone, A written, no G)
    if (!gram<ISDF_P_FP64, TS>(phi, ld_phi, n_phi, phi, ld_phi, n_phi, true, P.Ephi, P.Ephi, nmu16, n_mu, nullptr, nr,
                               r, rows, nullptr, 0, G_REAL, P.ab, s, nullptr, nullptr, P.A, nullptr))
      return ISDF_E_HIP;
    hipLaunchKernelGGL((exch_hadamard<TS>), dim3(grid_for((int64_t)rows * n_mu)), dim3(256), 0, s, P.A, rows, n_mu, V,
                       ld_v, v_complex, r, (const int*)P.ab);
    if (!launch_ok()) return ISDF_E_HIP;
    // W rows = -(conj(V) .* A) Psi_mu
    if (!tgemm<double, KC, KC>(rows, 2 * n_psi, two_mu, (const double*)P.A, two_mu, (const double*)P.Fpsi, two_mu,
                               W + 2 * r * ld_w, 2 * ld_w, -1.0, 0.0, P.ab, s))
      return ISDF_E_HIP;
  }
  return ISDF_OK;
}

}  // namespace
}  // namespace isdf

using namespace isdf;

extern "C" size_t isdf_exchange_workspace(const isdf_grid* grid, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                                          int64_t rblock) {
  if (!grid || n_mu <= 0 || n_phi <= 0 || n_psi <= 0 || rblock <= 0) return 0;
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] <= 0) return 0;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (rblock > nr) rblock = nr;
  return plan_exch(nullptr, 0, n_mu, n_phi, n_psi, rblock).bytes;
}

extern "C" int isdf_exchange(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi, int32_t n_phi,
                             const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx, int32_t n_mu,
                             const void* V, int64_t ld_v, int32_t v_complex, void* W, int64_t ld_w, int64_t rblock,
                             void* ws, size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  int64_t nr = 0;
  if (!fit_args_ok(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, ISDF_P_FP64, &nr)) return ISDF_E_ARG;
  if (!V || !W || ld_v < n_mu || ld_w < n_psi || rblock <= 0) return ISDF_E_ARG;
  if (rblock > nr) rblock = nr;
  ExchPlan P = plan_exch(ws, ws_bytes, n_mu, n_phi, n_psi, rblock);
  if (!ws || P.bytes > ws_bytes) return ISDF_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (dt == ISDF_C128)
    return exch_run<double>(nr, (const double*)phi, ld_phi, n_phi, (const double*)psi, ld_psi, n_psi, idx, n_mu,
                            (const double*)V, ld_v, v_complex, (double*)W, ld_w, rblock, P, s);
  return exch_run<float>(nr, (const float*)phi, ld_phi, n_phi, (const float*)psi, ld_psi, n_psi, idx, n_mu,
                         (const float*)V, ld_v, v_complex, (float*)W, ld_w, rblock, P, s);
}
