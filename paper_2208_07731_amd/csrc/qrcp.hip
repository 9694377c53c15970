// Interpolation points by QR with column pivoting of Z^T (arXiv:2208.07731,
// Sec. 2.1, eq. QRCP; cost in Table 1), without forming Z.
//
// The pivots of Z^T Pi = Q R are those of the pivoted Cholesky factorisation
// of the Gram matrix of Z^T's columns, conj(Z Z^H), and
//   (Z Z^H)(r, r') = (Phi Phi^H)(r, r') conj((Psi Psi^H)(r, r')),
// so one column of it costs two dot products per grid row.  With d_r the
// squared residual norm of column r of Z^T after k pivots (d_r = |R_kk|^2 at
// the pivot), step k is
//   p_k   = argmax_r d_r                       (lowest r on exact ties)
//   c_r   = K(r, p_k) - sum_{j<k} L(r, j) conj(L(p_k, j))
//   L(r,k)= c_r / sqrt(d_{p_k}),   d_r -= |L(r, k)|^2,
// an O(N_r (N_phi + N_psi + k)) pass over the orbitals and the first k
// columns of L: HBM-bound, N_mu dependent passes, O(N_mu^2 N_r) in total.
//
// The randomized variant factors the sketch (Z Omega)^T instead of Z^T, with
// Omega the Khatri-Rao product of random g_phi [N_phi][m], g_psi [N_psi][m]:
// X = Z Omega = (Phi g_phi) .* conj(Psi g_psi) (N_r x m) is one Hadamard Gram
// product of the fit's kind (the random columns in place of the orbital rows
// at the interpolation points), and the same pivoted Cholesky runs on the
// plain Gram matrix X X^H, whose column p is X conj(X(p))^T.
//
// Kernels: qrcp_init (d = the diagonal of the Gram matrix and workgroup top-2
// partials), qrcp_select (one workgroup: global top-2, accept or stop, gather
// the next pivot's row of L) and qrcp_step (one column of L).  Everything a
// step needs lives in device memory, so the host enqueues all 2 N_mu launches
// without synchronising; after a stop every later launch returns at once.
#include <algorithm>

#include "fitlib.h"

namespace isdf {
namespace {

constexpr int QR_TILE = 256;     // grid rows per workgroup (one per thread in phase 2)
constexpr int QR_LPC = 1024;     // pivot-row entries staged in LDS per chunk
constexpr int QR_SEL = 256;      // threads of qrcp_select
constexpr int QR_UNROLL = 4;     // rows per wavefront in flight in phase 1

// Gram matrix K whose pivoted Cholesky is taken:
enum {
  QR_ALIASED = 0,  // K = |Phi Phi^H|^2 (Psi = Phi): real
  QR_HADAMARD = 1, // K = (Phi Phi^H) .* conj(Psi Psi^H): complex Hermitian
  QR_PLAIN = 2     // K = X X^H (X passed as Phi): complex Hermitian
};

struct QrcpState {
  int32_t p;          // current pivot grid index
  int32_t done;       // 1: no further pivots
  int32_t rank;       // pivots accepted so far
  int32_t near_ties;  // accepted steps with gap <= near_tie_rel
  int32_t status;     // ISDF_OK or ISDF_E_NONFINITE
  int32_t pad;
  double dp;          // squared residual of the current pivot, |R_kk|^2
  double d0;          // |R_00|^2
};

// Top-2 of (value, row): best value, lowest row among equal best values,
// and the second largest value (equal to the best on an exact tie).
struct Top2 {
  double d1;
  int64_t r1;
  double d2;
};

__device__ __forceinline__ Top2 top2_merge(Top2 a, Top2 b) {
  const bool a_first = a.d1 > b.d1 || (a.d1 == b.d1 && a.r1 < b.r1);
  Top2 o;
  o.d1 = a_first ? a.d1 : b.d1;
  o.r1 = a_first ? a.r1 : b.r1;
  const double lose = a_first ? b.d1 : a.d1;
  o.d2 = fmax(lose, fmax(a.d2, b.d2));
  return o;
}

__device__ __forceinline__ Top2 top2_wave(Top2 t) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Top2 u;
    u.d1 = __shfl_xor(t.d1, o, ISDF_WAVE);
    u.r1 = __shfl_xor(t.r1, o, ISDF_WAVE);
    u.d2 = __shfl_xor(t.d2, o, ISDF_WAVE);
    t = top2_merge(t, u);
  }
  return t;
}

// Workgroup top-2 of (d, r) over its threads (d < 0: not a candidate) and
// count of non-finite values, stored as part[4 blockIdx.x + {d1, r1, d2, bad}].
__device__ __forceinline__ void block_top2_store(double d, int64_t r, double bad, double* part) {
  __shared__ Top2 red[QR_TILE / ISDF_WAVE];
  __shared__ double rbad[QR_TILE / ISDF_WAVE];
  Top2 t;
  t.d1 = d >= 0.0 ? d : -1.0;
  t.r1 = d >= 0.0 ? r : INT64_MAX;
  t.d2 = -1.0;
  t = top2_wave(t);
  bad = wave_sum(bad);
  const int w = threadIdx.x / ISDF_WAVE;
  if ((threadIdx.x & (ISDF_WAVE - 1)) == 0) {
    red[w] = t;
    rbad[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Top2 a = red[0];
    double b = rbad[0];
    for (int i = 1; i < QR_TILE / ISDF_WAVE; ++i) {
      a = top2_merge(a, red[i]);
      b += rbad[i];
    }
    double* o = part + 4 * blockIdx.x;
    o[0] = a.d1;
    o[1] = a.d1 >= 0.0 ? (double)a.r1 : -1.0;  // exact: grid indices < 2^31
    o[2] = a.d2;
    o[3] = b;
  }
}

template <class TS>
__device__ __forceinline__ double row_norm2(const TS* __restrict__ x, int64_t ld, int n, int64_t r, int lane) {
  double a = 0.0;
  for (int i = lane; i < n; i += ISDF_WAVE) {
    const double2 z = Cplx<TS>::load(x + 2 * (r * ld + i));
    a += z.x * z.x + z.y * z.y;
  }
  return wave_sum(a);
}

// d_r = K(r, r): rho_phi(r) rho_psi(r) = |Z(r)|^2, or |X(r)|^2 (QR_PLAIN).
// One wavefront per row.
template <class TS>
__global__ __launch_bounds__(QR_TILE) void qrcp_init(const TS* __restrict__ phi, int64_t ldp, int nphi,
                                                    const TS* __restrict__ psi, int64_t lds, int npsi,
                                                    int mode, int64_t nr, double* __restrict__ d,
                                                    double* __restrict__ part) {
  const int lane = threadIdx.x & (ISDF_WAVE - 1);
  const int wv = threadIdx.x / ISDF_WAVE;
  const int64_t base = (int64_t)blockIdx.x * QR_TILE + wv * ISDF_WAVE;
  double mine = -1.0;
  for (int rr = 0; rr < ISDF_WAVE; ++rr) {
    const int64_t r = base + rr;
    if (r >= nr) break;
    const double a = row_norm2<TS>(phi, ldp, nphi, r, lane);
    const double b = mode == QR_ALIASED ? a : (mode == QR_PLAIN ? 1.0 : row_norm2<TS>(psi, lds, npsi, r, lane));
    if (lane == rr) mine = a * b;
  }
  const int64_t r = base + lane;
  double bad = 0.0;
  if (r < nr) {
    if (!isfinite(mine)) {
      bad = 1.0;
      mine = 0.0;
    }
    d[r] = mine;
  } else {
    mine = -1.0;
  }
  block_top2_store(mine, r, bad, part);
}

// One column of L.  Phase 1: one wavefront per row for K(r, p) (lanes over
// the orbitals, Phi(p) and Psi(p) from LDS; the sketch's row X(p) in place).
// Phase 2: one thread per row
// for the projection on the earlier columns (column-major L, coalesced; the
// pivot's row of L broadcast from LDS in chunks).
template <class TS, int MODE>
__global__ __launch_bounds__(QR_TILE) void qrcp_step(const TS* __restrict__ phi, int64_t ldp, int nphi,
                                                    const TS* __restrict__ psi, int64_t lds, int npsi,
                                                    int64_t nr, int k, const QrcpState* __restrict__ st,
                                                    double* __restrict__ L, double* __restrict__ d,
                                                    const double* __restrict__ lp, double* __restrict__ part) {
  if (st->done) return;  // uniform: written by the previous select launch
  extern __shared__ double lds_mem[];
  constexpr bool CPLX = MODE != QR_ALIASED;
  constexpr bool TWO = MODE == QR_HADAMARD;  // a second orbital set
  constexpr int CW = CPLX ? 2 : 1;
  constexpr bool STAGE = MODE != QR_PLAIN;  // copy the pivot's orbital rows to LDS
  double2* sphi = reinterpret_cast<double2*>(lds_mem);
  double2* spsi = sphi + (STAGE ? nphi : 0);
  double* slp = reinterpret_cast<double*>(spsi + (TWO ? npsi : 0));
  const int64_t p = st->p;
  const double dp = st->dp;
  const int tid = threadIdx.x;
  const int lane = tid & (ISDF_WAVE - 1);
  const int wv = tid / ISDF_WAVE;

  if (STAGE)
    for (int i = tid; i < nphi; i += QR_TILE) sphi[i] = Cplx<TS>::load(phi + 2 * (p * ldp + i));
  if (TWO)
    for (int i = tid; i < npsi; i += QR_TILE) spsi[i] = Cplx<TS>::load(psi + 2 * (p * lds + i));
  __syncthreads();
  // the sketch's pivot row (m complex FP64 values, possibly more than LDS
  // holds) is read in place: every wavefront reads the same row, which
  // stays in the caches
  const double2* __restrict__ qphi;
  if constexpr (STAGE)
    qphi = sphi;
  else
    qphi = reinterpret_cast<const double2*>(phi) + p * ldp;

  // ---- phase 1: c = K(r, p): a conj(b), |a|^2 or a, a = Phi(r).conj(Phi(p)), b likewise
  const int64_t base = (int64_t)blockIdx.x * QR_TILE + wv * ISDF_WAVE;
  double cre = 0.0, cim = 0.0;
  for (int rr = 0; rr < ISDF_WAVE; rr += QR_UNROLL) {
    double ar[QR_UNROLL], ai[QR_UNROLL], br[QR_UNROLL], bi[QR_UNROLL];
#pragma unroll
    for (int u = 0; u < QR_UNROLL; ++u) {
      ar[u] = ai[u] = br[u] = bi[u] = 0.0;
      const int64_t r = base + rr + u;
      if (r < nr) {
        for (int i = lane; i < nphi; i += ISDF_WAVE) {
          const double2 z = Cplx<TS>::load(phi + 2 * (r * ldp + i));
          const double2 q = qphi[i];
          ar[u] += z.x * q.x + z.y * q.y;
          ai[u] += z.y * q.x - z.x * q.y;
        }
        if (TWO)
          for (int i = lane; i < npsi; i += ISDF_WAVE) {
            const double2 z = Cplx<TS>::load(psi + 2 * (r * lds + i));
            const double2 q = spsi[i];
            br[u] += z.x * q.x + z.y * q.y;
            bi[u] += z.y * q.x - z.x * q.y;
          }
      }
    }
#pragma unroll
    for (int u = 0; u < QR_UNROLL; ++u) {
      const double sar = wave_sum(ar[u]), sai = wave_sum(ai[u]);
      if (TWO) {
        const double sbr = wave_sum(br[u]), sbi = wave_sum(bi[u]);
        if (lane == rr + u) {
          cre = sar * sbr + sai * sbi;  // a conj(b)
          cim = sai * sbr - sar * sbi;
        }
      } else if (MODE == QR_PLAIN) {
        if (lane == rr + u) {
          cre = sar;                    // X(r) . conj(X(p))
          cim = sai;
        }
      } else if (lane == rr + u) {
        cre = sar * sar + sai * sai;    // |a|^2: Psi = Phi
      }
    }
  }
  // lane l of wavefront w now holds row base + l; move to thread-per-row order
  // (the same thread: row = blockIdx.x * QR_TILE + tid).
  const int64_t r = (int64_t)blockIdx.x * QR_TILE + tid;
  const bool live = r < nr;

  // ---- phase 2: c -= sum_{j<k} L(r, j) conj(L(p, j)); lp holds conj(L(p, j))
  double sre = 0.0, sim = 0.0;
  for (int j0 = 0; j0 < k; j0 += QR_LPC) {
    const int jn = min(QR_LPC, k - j0);
    __syncthreads();
    for (int t = tid; t < jn * CW; t += QR_TILE) slp[t] = lp[(int64_t)j0 * CW + t];
    __syncthreads();
    if (live) {
      const double* col = L + ((int64_t)j0 * nr + r) * CW;
      int j = 0;
      for (; j + 8 <= jn; j += 8) {
        double v[8 * CW];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (CPLX) {
            const double2 x = *reinterpret_cast<const double2*>(col + (int64_t)(j + u) * nr * CW);
            v[2 * u] = x.x;
            v[2 * u + 1] = x.y;
          } else {
            v[u] = col[(int64_t)(j + u) * nr];
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (CPLX) {
            const double qr = slp[2 * (j + u)], qi = slp[2 * (j + u) + 1];
            sre += v[2 * u] * qr - v[2 * u + 1] * qi;
            sim += v[2 * u] * qi + v[2 * u + 1] * qr;
          } else {
            sre += v[u] * slp[j + u];
          }
        }
      }
      for (; j < jn; ++j) {
        if (CPLX) {
          const double2 x = *reinterpret_cast<const double2*>(col + (int64_t)j * nr * CW);
          const double qr = slp[2 * j], qi = slp[2 * j + 1];
          sre += x.x * qr - x.y * qi;
          sim += x.x * qi + x.y * qr;
        } else {
          sre += col[(int64_t)j * nr] * slp[j];
        }
      }
    }
  }

  double dn = -1.0, bad = 0.0;
  if (live) {
    const double dr = d[r];
    double lre, lim = 0.0;
    if (r == p) {
      lre = sqrt(dp);  // the Cholesky diagonal, |R_kk|
      dn = -1.0;       // chosen
    } else if (dr < 0.0) {
      lre = 0.0;       // an earlier pivot: zero residual
      dn = -1.0;
    } else {
      const double inv = 1.0 / sqrt(dp);
      lre = (cre - sre) * inv;
      lim = CPLX ? (cim - sim) * inv : 0.0;
      const double t = dr - (lre * lre + lim * lim);
      if (isfinite(t)) {
        dn = fmax(t, 0.0);  // rounding below zero: an exhausted direction
      } else {
        bad = 1.0;
        dn = 0.0;
      }
    }
    double* out = L + ((int64_t)k * nr + r) * CW;
    if (CPLX)
      *reinterpret_cast<double2*>(out) = make_double2(lre, lim);
    else
      *out = lre;
    d[r] = dn;
  }
  block_top2_store(dn, r, bad, part);
}

// Global top-2 over the workgroup partials, the pivot decision of step k and
// the gather of the new pivot's row of L (conjugated) for the next column.
template <bool CPLX>
__global__ __launch_bounds__(QR_SEL) void qrcp_select(const double* __restrict__ part, int nblk, int k, int n_mu,
                                                     double rtol2, double near_tie_rel, int64_t nr,
                                                     const double* __restrict__ L, double* __restrict__ d,
                                                     double* __restrict__ lp, QrcpState* __restrict__ st,
                                                     int32_t* __restrict__ idx, double* __restrict__ rdiag,
                                                     double* __restrict__ gap, isdf_qrcp_info* __restrict__ info) {
  if (st->done) return;
  constexpr int CW = CPLX ? 2 : 1;
  __shared__ Top2 red[QR_SEL / ISDF_WAVE];
  __shared__ double rbad[QR_SEL / ISDF_WAVE];
  __shared__ int accept_s;
  __shared__ int64_t p_s;
  const int tid = threadIdx.x;
  Top2 t;
  t.d1 = -1.0;
  t.r1 = INT64_MAX;
  t.d2 = -1.0;
  double bad = 0.0;
  for (int b = tid; b < nblk; b += QR_SEL) {
    Top2 u;
    u.d1 = part[4 * b];
    u.r1 = u.d1 >= 0.0 ? (int64_t)part[4 * b + 1] : INT64_MAX;
    u.d2 = part[4 * b + 2];
    t = top2_merge(t, u);
    bad += part[4 * b + 3];
  }
  t = top2_wave(t);
  bad = wave_sum(bad);
  const int w = tid / ISDF_WAVE;
  if ((tid & (ISDF_WAVE - 1)) == 0) {
    red[w] = t;
    rbad[w] = bad;
  }
  __syncthreads();
  if (tid == 0) {
    Top2 a = red[0];
    double nb = rbad[0];
    for (int i = 1; i < QR_SEL / ISDF_WAVE; ++i) {
      a = top2_merge(a, red[i]);
      nb += rbad[i];
    }
    if (k == 0) st->d0 = a.d1 > 0.0 ? a.d1 : 0.0;
    const double d0 = st->d0;
    int accept = 0;
    if (nb > 0.0) {
      st->status = ISDF_E_NONFINITE;
    } else if (a.d1 > 0.0 && a.d1 > rtol2 * d0 && a.r1 < nr) {
      accept = 1;
    }
    if (accept) {
      const double g = (a.d1 - fmax(a.d2, 0.0)) / a.d1;
      idx[k] = (int32_t)a.r1;
      rdiag[k] = sqrt(a.d1);
      if (gap) gap[k] = g;
      if (g <= near_tie_rel) st->near_ties += 1;
      st->p = (int32_t)a.r1;
      st->dp = a.d1;
      st->rank = k + 1;
      d[a.r1] = -1.0;
    } else {
      st->done = 1;
    }
    accept_s = accept;
    p_s = a.r1;
    if (!accept || k == n_mu - 1) {
      info->status = st->status;
      info->rank = st->rank;
      info->near_ties = st->near_ties;
      info->reserved = 0;
      info->r00 = sqrt(st->d0);
    }
  }
  __syncthreads();
  if (accept_s) {
    if (k < n_mu - 1) {
      const int64_t p = p_s;
      for (int j = tid; j < k; j += QR_SEL) {
        const double* src = L + ((int64_t)j * nr + p) * CW;
        lp[(int64_t)j * CW] = src[0];
        if (CPLX) lp[(int64_t)j * CW + 1] = -src[1];
      }
    }
  } else {
    for (int j = k + tid; j < n_mu; j += QR_SEL) {
      idx[j] = -1;
      rdiag[j] = 0.0;
      if (gap) gap[j] = 0.0;
    }
  }
}

__global__ void qrcp_reset(QrcpState* st) {
  st->p = -1;
  st->done = 0;
  st->rank = 0;
  st->near_ties = 0;
  st->status = ISDF_OK;
  st->pad = 0;
  st->dp = 0.0;
  st->d0 = 0.0;
}

// LDS of one qrcp_step workgroup: Phi(p), Psi(p) and a chunk of the pivot's row of L.
static size_t qrcp_lds_bytes(int n_phi, int n_psi, int mode) {
  return sizeof(double2) * (size_t)((mode == QR_PLAIN ? 0 : n_phi) + (mode == QR_HADAMARD ? n_psi : 0)) +
         sizeof(double) * QR_LPC * (mode == QR_ALIASED ? 1 : 2);
}
static constexpr size_t QR_MAX_LDS = 64 * 1024;

struct QrcpPlan {
  double* L;
  double* d;
  double* lp;
  double* part;
  QrcpState* st;
  size_t bytes;
};

static QrcpPlan plan_qrcp(void* ws, int64_t nr, int n_mu, bool cplx) {
  Carver c(ws, (size_t)-1);
  const int cw = cplx ? 2 : 1;
  const int64_t nblk = ceil_div(nr, QR_TILE);
  QrcpPlan pl;
  pl.L = c.take<double>((size_t)(n_mu > 1 ? n_mu - 1 : 1) * nr * cw);
  pl.d = c.take<double>((size_t)nr);
  pl.lp = c.take<double>((size_t)n_mu * cw);
  pl.part = c.take<double>((size_t)4 * nblk);
  pl.st = c.take<QrcpState>(1);
  pl.bytes = c.used;
  return pl;
}

template <class TS, int MODE>
static int qrcp_run(const TS* phi, int64_t ldp, int nphi, const TS* psi, int64_t lds, int npsi, int64_t nr, int n_mu,
                    double rtol, double near_tie_rel, int32_t* idx, double* rdiag, double* gap,
                    isdf_qrcp_info* info, const QrcpPlan& pl, hipStream_t s) {
  const int nblk = (int)ceil_div(nr, QR_TILE);
  constexpr bool CPLX = MODE != QR_ALIASED;
  const size_t lds_bytes = qrcp_lds_bytes(nphi, npsi, MODE);
  const double rtol2 = rtol * rtol;
  hipLaunchKernelGGL(qrcp_reset, dim3(1), dim3(1), 0, s, pl.st);
  if (!launch_ok()) return ISDF_E_HIP;
  hipLaunchKernelGGL((qrcp_init<TS>), dim3(nblk), dim3(QR_TILE), 0, s, phi, ldp, nphi, psi, lds, npsi, MODE, nr,
                     pl.d, pl.part);
  if (!launch_ok()) return ISDF_E_HIP;
  for (int k = 0; k < n_mu; ++k) {
    hipLaunchKernelGGL((qrcp_select<CPLX>), dim3(1), dim3(QR_SEL), 0, s, (const double*)pl.part, nblk, k, n_mu,
                       rtol2, near_tie_rel, nr, (const double*)pl.L, pl.d, pl.lp, pl.st, idx, rdiag, gap, info);
    if (!launch_ok()) return ISDF_E_HIP;
    if (k == n_mu - 1) break;
    hipLaunchKernelGGL((qrcp_step<TS, MODE>), dim3(nblk), dim3(QR_TILE), lds_bytes, s, phi, ldp, nphi, psi, lds,
                       npsi, nr, k, (const QrcpState*)pl.st, pl.L, pl.d, (const double*)pl.lp, pl.part);
    if (!launch_ok()) return ISDF_E_HIP;
  }
  return ISDF_OK;
}

}  // namespace
}  // namespace isdf

using namespace isdf;


extern "C" size_t isdf_qrcp_workspace(const isdf_grid* grid, int32_t n_mu, int32_t aliased) {
  if (!grid || n_mu <= 0) return 0;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (nr <= 0) return 0;
  return plan_qrcp(nullptr, nr, n_mu, !aliased).bytes;
}

extern "C" int isdf_qrcp(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi, int32_t n_phi,
                         const void* psi, int64_t ld_psi, int32_t n_psi, int32_t n_mu, double rtol,
                         double near_tie_rel, int32_t* idx, double* rdiag, double* gap, isdf_qrcp_info* info,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  if (!grid) return ISDF_E_ARG;
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] <= 0) return ISDF_E_ARG;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (dt != ISDF_C128 && dt != ISDF_C64) return ISDF_E_ARG;
  if (!phi || !psi || !idx || !rdiag || !info) return ISDF_E_ARG;
  if (n_phi <= 0 || n_psi <= 0 || ld_phi < n_phi || ld_psi < n_psi) return ISDF_E_ARG;
  if (n_mu <= 0 || n_mu > nr || nr >= ((int64_t)1 << 31)) return ISDF_E_ARG;
  if (!(rtol >= 0.0 && rtol < 1.0) || !(near_tie_rel >= 0.0)) return ISDF_E_ARG;
  const bool aliased = phi == psi && ld_phi == ld_psi && n_phi == n_psi;
  if (qrcp_lds_bytes(n_phi, n_psi, aliased ? QR_ALIASED : QR_HADAMARD) > QR_MAX_LDS) return ISDF_E_UNSUPPORTED;
  const QrcpPlan need = plan_qrcp(nullptr, nr, n_mu, !aliased);
  if (!ws || ws_bytes < need.bytes) return ISDF_E_WORKSPACE;
  const QrcpPlan pl = plan_qrcp(ws, nr, n_mu, !aliased);
  hipStream_t s = (hipStream_t)stream;
  if (dt == ISDF_C128) {
    const double *a = (const double*)phi, *b = (const double*)psi;
    return aliased ? qrcp_run<double, QR_ALIASED>(a, ld_phi, n_phi, b, ld_psi, n_psi, nr, n_mu, rtol, near_tie_rel,
                                                  idx, rdiag, gap, info, pl, s)
                   : qrcp_run<double, QR_HADAMARD>(a, ld_phi, n_phi, b, ld_psi, n_psi, nr, n_mu, rtol, near_tie_rel,
                                                   idx, rdiag, gap, info, pl, s);
  }
  const float *a = (const float*)phi, *b = (const float*)psi;
  return aliased ? qrcp_run<float, QR_ALIASED>(a, ld_phi, n_phi, b, ld_psi, n_psi, nr, n_mu, rtol, near_tie_rel,
                                               idx, rdiag, gap, info, pl, s)
                 : qrcp_run<float, QR_HADAMARD>(a, ld_phi, n_phi, b, ld_psi, n_psi, nr, n_mu, rtol, near_tie_rel,
                                                idx, rdiag, gap, info, pl, s);
}

namespace isdf {
namespace {

// R[k][i] = g[i][k] + 0 i (the sketch columns as complex "rows" for the
// Gram right-hand side), iota[k] = k.
__global__ void sketch_rows(const double* __restrict__ g, int n, int m, double* __restrict__ R,
                            int32_t* __restrict__ iota) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / n), i = (int)(e % n);
    R[2 * e] = g[(int64_t)i * m + k];
    R[2 * e + 1] = 0.0;
    if (e < m) iota[e] = (int32_t)e;
  }
}

struct SketchPlan {
  double* X;  // [N_r][m] interleaved complex: Z Omega
  double *Rphi, *Rpsi, *Ephi, *Epsi;
  int32_t* iota;
  int* ab;
  QrcpPlan q;
  size_t bytes;
};

static SketchPlan plan_sketch(void* ws, int64_t nr, int n_mu, int n_phi, int n_psi, int m) {
  Carver c(ws, (size_t)-1);
  SketchPlan pl;
  const int m16 = (int)ceil_div(m, 16) * 16;
  pl.X = c.take<double>((size_t)nr * 2 * m);
  pl.Rphi = c.take<double>((size_t)m * 2 * n_phi);
  pl.Rpsi = c.take<double>((size_t)m * 2 * n_psi);
  pl.Ephi = c.take<double>((size_t)2 * m16 * 2 * n_phi);
  pl.Epsi = c.take<double>((size_t)2 * m16 * 2 * n_psi);
  pl.iota = c.take<int32_t>((size_t)m);
  pl.ab = c.take<int>(64);
  const size_t head = c.used;
  pl.q = plan_qrcp(ws ? (char*)ws + align_up(head, 256) : nullptr, nr, n_mu, true);
  pl.bytes = align_up(head, 256) + pl.q.bytes;
  return pl;
}

template <class TS>
static int sketch_run(const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                      const double* g_phi, const double* g_psi, int m, int64_t nr, int n_mu, double rtol,
                      double near_tie_rel, int32_t* idx, double* rdiag, double* gap, isdf_qrcp_info* info,
                      const SketchPlan& pl, hipStream_t s) {
  const int m16 = (int)ceil_div(m, 16) * 16;
  if (!fill<int>(pl.ab, 1, 0, s)) return ISDF_E_HIP;
  // (every entry of iota is written: m <= m n)
  const unsigned bphi = (unsigned)std::min<int64_t>(ceil_div((int64_t)m * n_phi, 256), 4096);
  const unsigned bpsi = (unsigned)std::min<int64_t>(ceil_div((int64_t)m * n_psi, 256), 4096);
  hipLaunchKernelGGL(sketch_rows, dim3(bphi), dim3(256), 0, s, g_phi, n_phi, m, pl.Rphi, pl.iota);
  hipLaunchKernelGGL(sketch_rows, dim3(bpsi), dim3(256), 0, s, g_psi, n_psi, m, pl.Rpsi, pl.iota);
  if (!launch_ok()) return ISDF_E_HIP;
  if (!pack<double, double>(pl.Rphi, n_phi, n_phi, pl.iota, m, m, m16, pl.Ephi, s)) return ISDF_E_HIP;
  if (!pack<double, double>(pl.Rpsi, n_psi, n_psi, pl.iota, m, m, m16, pl.Epsi, s)) return ISDF_E_HIP;
  // X = (Phi g_phi) .* conj(Psi g_psi), FP64 (two right-hand sides even when Psi = Phi)
  SplitWork none{};
  if (!gram<ISDF_P_FP64, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, false, pl.Ephi, pl.Epsi, m16, m, nullptr, nr, 0,
                             (int)nr, pl.X, 2 * (int64_t)m, G_CPLX, pl.ab, s, nullptr, &none))
    return ISDF_E_HIP;
  return qrcp_run<double, QR_PLAIN>(pl.X, m, m, pl.X, m, m, nr, n_mu, rtol, near_tie_rel, idx, rdiag, gap, info,
                                    pl.q, s);
}

}  // namespace
}  // namespace isdf

extern "C" size_t isdf_qrcp_sketch_workspace(const isdf_grid* grid, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                                             int32_t m) {
  if (!grid || n_mu <= 0 || n_phi <= 0 || n_psi <= 0 || m <= 0) return 0;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (nr <= 0) return 0;
  return plan_sketch(nullptr, nr, n_mu, n_phi, n_psi, m).bytes;
}

extern "C" int isdf_qrcp_sketch(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi, int32_t n_phi,
                                const void* psi, int64_t ld_psi, int32_t n_psi, const double* g_phi,
                                const double* g_psi, int32_t m, int32_t n_mu, double rtol, double near_tie_rel,
                                int32_t* idx, double* rdiag, double* gap, isdf_qrcp_info* info, void* ws,
                                size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  if (!grid) return ISDF_E_ARG;
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] <= 0) return ISDF_E_ARG;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (dt != ISDF_C128 && dt != ISDF_C64) return ISDF_E_ARG;
  if (!phi || !psi || !g_phi || !g_psi || !idx || !rdiag || !info) return ISDF_E_ARG;
  if (n_phi <= 0 || n_psi <= 0 || ld_phi < n_phi || ld_psi < n_psi || m <= 0) return ISDF_E_ARG;
  if (n_mu <= 0 || n_mu > nr || nr >= ((int64_t)1 << 31)) return ISDF_E_ARG;
  if (!(rtol >= 0.0 && rtol < 1.0) || !(near_tie_rel >= 0.0)) return ISDF_E_ARG;
  const SketchPlan need = plan_sketch(nullptr, nr, n_mu, n_phi, n_psi, m);
  if (!ws || ws_bytes < need.bytes) return ISDF_E_WORKSPACE;
  const SketchPlan pl = plan_sketch(ws, nr, n_mu, n_phi, n_psi, m);
  hipStream_t s = (hipStream_t)stream;
  if (dt == ISDF_C128)
    return sketch_run<double>((const double*)phi, ld_phi, n_phi, (const double*)psi, ld_psi, n_psi, g_phi, g_psi, m,
                              nr, n_mu, rtol, near_tie_rel, idx, rdiag, gap, info, pl, s);
  return sketch_run<float>((const float*)phi, ld_phi, n_phi, (const float*)psi, ld_psi, n_psi, g_phi, g_psi, m, nr,
                           n_mu, rtol, near_tie_rel, idx, rdiag, gap, info, pl, s);
}
