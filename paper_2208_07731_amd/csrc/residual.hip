// Cluster residual of Appendix A of arXiv:2208.07731 (eqs. errorISDF, proj,
// Zmu and the first lines of eq. error2), without forming Z:
//
//   R = sum_r [ rho_phi(r) rho_psi(r)
//               - |(Phi(r) . Phi*(p)) conj(Psi(r) . Psi*(p))|^2 / (rho_phi(p) rho_psi(p)) ],
//   p = idx[labels[r]], the interpolation point of r's cluster,
//
// i.e. every row of Z replaced by its projection on its cluster's
// interpolation row.  One wavefront per grid row, lanes over the orbitals;
// per-workgroup sums reduced in a fixed order.
#include "common.h"

namespace isdf {
namespace {

constexpr int RES_BLOCKS = 1024;

template <class TS>
__device__ __forceinline__ void row_pair(const TS* __restrict__ x, int64_t ld, int n, int64_t r, int64_t p, int lane,
                                         double& rr, double& pp, double& dr, double& di) {
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int i = lane; i < n; i += ISDF_WAVE) {
    const double2 z = Cplx<TS>::load(x + 2 * (r * ld + i));
    const double2 q = Cplx<TS>::load(x + 2 * (p * ld + i));
    a += z.x * z.x + z.y * z.y;
    b += q.x * q.x + q.y * q.y;
    c += z.x * q.x + z.y * q.y;  // Re z conj(q)
    d += z.y * q.x - z.x * q.y;  // Im z conj(q)
  }
  rr = wave_sum(a);
  pp = wave_sum(b);
  dr = wave_sum(c);
  di = wave_sum(d);
}

template <class TS>
__global__ __launch_bounds__(PAIR_THREADS) void cluster_resid(const TS* __restrict__ phi, int64_t ldp, int nphi,
                                                              const TS* __restrict__ psi, int64_t lds, int npsi,
                                                              int aliased, const int32_t* __restrict__ labels,
                                                              const int32_t* __restrict__ idx, int n_mu, int64_t nr,
                                                              double* __restrict__ part) {
  const int lane = threadIdx.x & (ISDF_WAVE - 1);
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / ISDF_WAVE;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / ISDF_WAVE;
  double acc = 0.0, bad = 0.0;
  for (int64_t r = wave; r < nr; r += nwaves) {
    const int lab = labels[r];
    int64_t p = -1;
    if (lab >= 0 && lab < n_mu) p = idx[lab];
    if (p < 0 || p >= nr) {
      bad += 1.0;
      continue;
    }
    double rp, pp, ar, ai;
    row_pair<TS>(phi, ldp, nphi, r, p, lane, rp, pp, ar, ai);
    double rs = rp, ps = pp, br = ar, bi = ai;
    if (!aliased) row_pair<TS>(psi, lds, npsi, r, p, lane, rs, ps, br, bi);
    // Z(r) . Z*(p) = a conj(b)
    const double zr = ar * br + ai * bi, zi = ai * br - ar * bi;
    acc += rp * rs - (zr * zr + zi * zi) / (pp * ps);
  }
  // every lane of a wave holds the wave's totals: count them once
  if (lane != 0) acc = bad = 0.0;
  block_pair_store(acc, bad, part);
}

}  // namespace
}  // namespace isdf

using namespace isdf;

extern "C" size_t isdf_cluster_residual_workspace(void) { return (size_t)2 * RES_BLOCKS * sizeof(double); }

extern "C" int isdf_cluster_residual(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi,
                                     int32_t n_phi, const void* psi, int64_t ld_psi, int32_t n_psi,
                                     const int32_t* labels, const int32_t* idx, int32_t n_mu, double* out, void* ws,
                                     size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  if (!grid) return ISDF_E_ARG;
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] <= 0) return ISDF_E_ARG;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (dt != ISDF_C128 && dt != ISDF_C64) return ISDF_E_ARG;
  if (!phi || !psi || !labels || !idx || !out || n_mu <= 0 || n_phi <= 0 || n_psi <= 0) return ISDF_E_ARG;
  if (ld_phi < n_phi || ld_psi < n_psi) return ISDF_E_ARG;
  if (!ws || ws_bytes < isdf_cluster_residual_workspace()) return ISDF_E_WORKSPACE;
  const bool aliased = phi == psi && ld_phi == ld_psi && n_phi == n_psi;
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)ws;
  if (dt == ISDF_C128)
    hipLaunchKernelGGL((cluster_resid<double>), dim3(RES_BLOCKS), dim3(PAIR_THREADS), 0, s, (const double*)phi,
                       ld_phi, n_phi, (const double*)psi, ld_psi, n_psi, aliased ? 1 : 0, labels, idx, n_mu, nr,
                       part);
  else
    hipLaunchKernelGGL((cluster_resid<float>), dim3(RES_BLOCKS), dim3(PAIR_THREADS), 0, s, (const float*)phi, ld_phi,
                       n_phi, (const float*)psi, ld_psi, n_psi, aliased ? 1 : 0, labels, idx, n_mu, nr, part);
  if (!launch_ok()) return ISDF_E_HIP;
  hipLaunchKernelGGL(sum_pairs, dim3(1), dim3(PAIR_THREADS), 0, s, (const double*)part, RES_BLOCKS, out);
  return launch_ok() ? ISDF_OK : ISDF_E_HIP;
}
