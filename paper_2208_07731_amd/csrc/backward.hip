// Adjoint of the least-squares fit Theta = G M^-1 (eq. theta of
// arXiv:2208.07731) with the interpolation points fixed.  The paper has no
// adjoint; this is reverse-mode differentiation of the forward formulas, in
// PyTorch's complex-gradient convention (dL/dRe + i dL/dIm):
//
//   S = Thetabar M^-1,  Mbar = -Theta^H S,  Gbar = S,  Gbar[idx] += Mbar,
//   Abar = Gbar .* B,  Bbar = conj(Gbar) .* A,
//   dPhi = Abar Phi_mu,  dPhi[idx] += Abar^H Phi,  (same for Psi with Bbar).
//
// G, A, B are recomputed one r-block at a time and never stored whole, or,
// for callers that kept them from the forward (isdf_zc_ab), read from there
// and overwritten in place; the r-block loop and every reduction order are
// the same either way, so both give bitwise equal gradients.
// General upstream Thetabar: per block Theta = G M^-1 and S = Thetabar M^-1
// (FP64 GEMMs), the split-K partials of Theta^T S, Abar / Bbar in place.
// Fused loss L = sum_r g_r sum_mu |Theta_r,mu|^2 (Thetabar = 2 g Theta):
// S = 2 g . (G M^-2) and Theta^T S = 2 M^-1 H M^-2 with H = G^T diag(g) G,
// so Theta is never formed: per block one FP64 GEMM G M^-2 whose epilogue
// writes Abar / Bbar and the loss, and the lower half of H (split-K).
// Either way the block's rows of dPhi = Abar Phi_mu and the partials of
// Abar^T Phi follow; every split-K reduction runs in a fixed order, so the
// result is deterministic.  The Mbar terms touch only the N_mu
// interpolation rows and are applied once after the last block.
#include "fitlib.h"

namespace isdf {
namespace {

constexpr int MAX_SPLITS = 32;

// Abar / Bbar from S and the block's Gram blocks, in place.
//  aliased: S real [R][n_mu]; A complex -> Abar = S A (over A)
//  general: S complex; Abar = S B (over B), Bbar = conj(S) A (over A)
__global__ void adj_hadamard(const double* __restrict__ S, double* __restrict__ A, double* __restrict__ B,
                             int64_t R, int n_mu, int aliased) {
  const int64_t total = R * n_mu;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double2* a = reinterpret_cast<double2*>(A) + e;
    if (aliased) {
      const double s = S[e];
      double2 v = *a;
      *a = make_double2(s * v.x, s * v.y);
    } else {
      const double2 s = reinterpret_cast<const double2*>(S)[e];
      double2* b = reinterpret_cast<double2*>(B) + e;
      const double2 av = *a, bv = *b;
      *b = make_double2(s.x * bv.x - s.y * bv.y, s.x * bv.y + s.y * bv.x);
      *a = make_double2(s.x * av.x + s.y * av.y, s.x * av.y - s.y * av.x);
    }
  }
}

// Real rows of Phi at the interpolation points: X[mu][k] = Phi_real[idx[mu]][k].
template <class TS, class T>
__global__ void gather_rows(const TS* __restrict__ phi, int64_t ld, int n, const int32_t* __restrict__ idx,
                            int n_mu, int64_t nr, T* __restrict__ X) {
  const int64_t total = (int64_t)n_mu * 2 * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mu = (int)(e / (2 * n)), k = (int)(e % (2 * n));
    int64_t p = idx[mu];
    if (p < 0 || p >= nr) p = 0;
    X[e] = (T)phi[2 * p * ld + k];
  }
}

// out = (accumulate ? out : 0) + sum_z part[z] in increasing z.
__global__ void reduce_splits(double* __restrict__ out, const double* __restrict__ part, int64_t n, int splits,
                              int accumulate, const int* abort) {
  if (*abort) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = accumulate ? out[i] : 0.0;
    for (int z = 0; z < splits; ++z) s += part[z * n + i];
    out[i] = s;
  }
}

// Fused-loss S = 2 g . (G (C C^H)^-2) never stored: its epilogue forms
// Abar / Bbar in place (as adj_hadamard does) and the loss partial
// sum_r g_r sum_c (G (C C^H)^-2)_rc G_rc  (= sum_r g_r |Theta_r|^2).
// In the complex case the partner lane (column 2 nu + 1 - c) supplies the
// other half of S_{r nu}.
struct EpiSAdj {
  const double* G;
  int64_t ldg;
  double* A;
  double* B;
  int64_t ldab;
  const double* g;
  int M, N;
  int aliased;
  double* partial;
  double* amax;  // optional [2]: max |re|, |im| of Abar and of Bbar written here (binary16 scales)
  template <class Cfg, class Acc>
  __device__ __forceinline__ void apply(const Acc (&acc)[Cfg::MI][Cfg::NI], const TileAt& at) const {
    __shared__ double red[Cfg::THREADS / ISDF_WAVE];
    double sl = 0.0, ma = 0.0, mb = 0.0;
    if (aliased) {
      // One 16 x 16 tile at a time, its loads (indices clamped into the
      // block, so without branches) all issued before its stores: a store
      // into A, written in place, would otherwise keep every later load of
      // G or A from starting before it.  Arithmetic and the order of the
      // loss sum are those of one element at a time.
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) {
          const int n = at.n_wave + j * 16 + (at.lane & 15);
          const int nc = n < N ? n : N - 1;
          double gm[4], gv[4];
          double2 xv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = at.m_wave + i * 16 + Cfg::orow(at.lane, r);
            const int mc = m < M ? m : M - 1;
            gm[r] = g[mc];
            gv[r] = G[(int64_t)mc * ldg + nc];
            xv[r] = *reinterpret_cast<const double2*>(A + (int64_t)mc * ldab + 2 * nc);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = at.m_wave + i * 16 + Cfg::orow(at.lane, r);
            if (m < M && n < N) {
              const double v = (double)acc[i][j][r];
              const double s = 2.0 * gm[r] * v;
              sl += gm[r] * v * gv[r];
              const double2 o = make_double2(s * xv[r].x, s * xv[r].y);
              *reinterpret_cast<double2*>(A + (int64_t)m * ldab + 2 * n) = o;
              ma = fmax(ma, fmax(fabs(o.x), fabs(o.y)));
            }
          }
          __builtin_amdgcn_sched_barrier(0);  // one tile's loads in flight at a time
        }
    } else {
      // Psi != Phi: one element at a time (lane pairs exchange S)
#pragma unroll
      for (int i = 0; i < Cfg::MI; ++i)
#pragma unroll
        for (int j = 0; j < Cfg::NI; ++j) {
          const int n = at.n_wave + j * 16 + (at.lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = at.m_wave + i * 16 + Cfg::orow(at.lane, r);
            const bool ok = m < M && n < N;
            const double gm = ok ? g[m] : 0.0;
            const double v = (double)acc[i][j][r];
            const double s = 2.0 * gm * v;
            if (ok) sl += gm * v * G[(int64_t)m * ldg + n];
            const double so = __shfl_xor(s, 1, ISDF_WAVE);
            if (ok) {
              const int nu = n >> 1, c = n & 1;
              const double sr = c ? so : s, si = c ? s : so;
              if (c == 0) {
                double2* bp = reinterpret_cast<double2*>(B + (int64_t)m * ldab + 2 * nu);
                const double2 bv = *bp;
                const double2 o = make_double2(sr * bv.x - si * bv.y, sr * bv.y + si * bv.x);
                *bp = o;
                ma = fmax(ma, fmax(fabs(o.x), fabs(o.y)));
              } else {
                double2* ap = reinterpret_cast<double2*>(A + (int64_t)m * ldab + 2 * nu);
                const double2 av = *ap;
                const double2 o = make_double2(sr * av.x + si * av.y, sr * av.y - si * av.x);
                *ap = o;
                mb = fmax(mb, fmax(fabs(o.x), fabs(o.y)));
              }
            }
          }
        }
    }
    sl = wave_sum(sl);
    if (at.lane == 0) red[threadIdx.x >> 6] = sl;
    if (amax) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        ma = fmax(ma, __shfl_xor(ma, o, ISDF_WAVE));
        mb = fmax(mb, __shfl_xor(mb, o, ISDF_WAVE));
      }
      if (at.lane == 0) {
        if (ma > 0.0) atomic_max_pos(amax, ma);
        if (mb > 0.0) atomic_max_pos(amax + 1, mb);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < Cfg::THREADS / ISDF_WAVE; ++w) t += red[w];
      partial[blockIdx.x] = t;
    }
  }
};

// Largest |x| and |x rowscale[k]| over the rows of a real r-major block
// (binary16 scales of the two split operands of H), folded into out[0] and
// out[1] (positive doubles order like their bit patterns).
__global__ void absmax_real2(const double* __restrict__ x, int64_t ld, int n, int64_t rows,
                             const double* __restrict__ rowscale, double* out) {
  double m = 0.0, mg = 0.0;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const double gr = fabs(rowscale[r]);
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const double v = fabs(x[r * ld + k]);
      m = fmax(m, v);
      mg = fmax(mg, v * gr);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m = fmax(m, __shfl_xor(m, o, ISDF_WAVE));
    mg = fmax(mg, __shfl_xor(mg, o, ISDF_WAVE));
  }
  if ((threadIdx.x & 63) == 0) {
    if (mg > 0.0) atomic_max_pos(out, mg);
    if (m > 0.0) atomic_max_pos(out + 1, m);
  }
}

// Upper triangle of an n x n matrix from its lower triangle.
__global__ void mirror_lower(double* __restrict__ H, int n, const int* abort) {
  if (*abort) return;
  const int64_t total = (int64_t)n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (j > i) H[e] = H[(int64_t)j * n + i];
  }
}

// loss += sum of the per-tile partials, in a fixed order (one workgroup of
// 256 threads, four independent loads in flight per thread).
constexpr int LOSS_THREADS = 256;
__global__ __launch_bounds__(LOSS_THREADS) void add_loss(FitState* st, const double* __restrict__ partial, int n) {
  __shared__ double red[LOSS_THREADS / ISDF_WAVE];
  if (st->abort) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 3 * LOSS_THREADS < n; i += 4 * LOSS_THREADS) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += partial[i + u * LOSS_THREADS];
  }
  for (int u = 0; i < n; i += LOSS_THREADS, ++u) s[u] += partial[i];
  double t = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
  if ((threadIdx.x & (ISDF_WAVE - 1)) == 0) red[threadIdx.x / ISDF_WAVE] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < LOSS_THREADS / ISDF_WAVE; ++w) a += red[w];
    st->loss += a;
  }
}

// Corrections at the interpolation rows from Mbar = -combine(P):
//  aliased: dA = Mbar .* A_mu (Mbar real)
//  general: Mbar_{mu nu} = -[(P_rr + P_ii) + i (P_ri - P_ir)],
//           dA = Mbar .* B_mu, dB = conj(Mbar) .* A_mu
__global__ void mbar_hadamard(const double* __restrict__ P, const double* __restrict__ Amu,
                              const double* __restrict__ Bmu, double* __restrict__ dA, double* __restrict__ dB,
                              int n_mu, int aliased, const int* abort) {
  if (*abort) return;
  const int64_t total = (int64_t)n_mu * n_mu;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mu = (int)(e / n_mu), nu = (int)(e % n_mu);
    const double2 a = reinterpret_cast<const double2*>(Amu)[e];
    if (aliased) {
      const double m = -P[e];
      reinterpret_cast<double2*>(dA)[e] = make_double2(m * a.x, m * a.y);
    } else {
      const int64_t n1 = 2 * (int64_t)n_mu;
      const double prr = P[(2 * mu) * n1 + 2 * nu], pii = P[(2 * mu + 1) * n1 + 2 * nu + 1];
      const double pri = P[(2 * mu) * n1 + 2 * nu + 1], pir = P[(2 * mu + 1) * n1 + 2 * nu];
      const double mr = -(prr + pii), mi = -(pri - pir);
      const double2 b = reinterpret_cast<const double2*>(Bmu)[e];
      reinterpret_cast<double2*>(dA)[e] = make_double2(mr * b.x - mi * b.y, mr * b.y + mi * b.x);
      reinterpret_cast<double2*>(dB)[e] = make_double2(mr * a.x + mi * a.y, mr * a.y - mi * a.x);
    }
  }
}

// dX[idx[mu]][i] += T1[mu][i] + (Abar^H X)[mu][i], the latter combined from
// Q[2 mu + c][2 i + c'] = sum_r Abar_c(r, mu) X_c'(r, i).
template <class TS>
__global__ void scatter_rows(TS* __restrict__ dX, int64_t ld, int n, const int32_t* __restrict__ idx, int n_mu,
                             int64_t nr, const double* __restrict__ Q, const double* __restrict__ T1,
                             const int* abort) {
  if (*abort) return;
  const int64_t total = (int64_t)n_mu * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mu = (int)(e / n), i = (int)(e % n);
    const int64_t q0 = (int64_t)(2 * mu) * (2 * n), q1 = q0 + 2 * n;
    const double re = Q[q0 + 2 * i] + Q[q1 + 2 * i + 1] + T1[(int64_t)mu * 2 * n + 2 * i];
    const double im = Q[q0 + 2 * i + 1] - Q[q1 + 2 * i] + T1[(int64_t)mu * 2 * n + 2 * i + 1];
    const int64_t row = idx[mu];
    if (row < 0 || row >= nr) continue;  // reported by check_idx, which also aborts the call
    TS* p = dX + 2 * (row * ld + i);
    const double2 old = Cplx<TS>::load(p);
    Cplx<TS>::store(p, old.x + re, old.y + im);
  }
}

template <class TS>
__global__ void copy_rows(TS* __restrict__ dst, int64_t ldd, const TS* __restrict__ src, int64_t lds, int64_t rows,
                          int n) {
  const int64_t total = rows * 2 * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / (2 * n), k = e % (2 * n);
    dst[2 * r * ldd + k] = src[2 * r * lds + k];
  }
}

// K extent of the transposed planes of a block of `rows` grid rows, and
// their row pitch: one 128-byte line more, so that blocks of 2^k rows do not
// put every plane row at the same power-of-two stride (8-14 % less L2-miss
// traffic in the products over grid rows at 65536-row blocks).
static inline int kext_rows(int64_t rows) { return (int)ceil_div(rows, 32) * 32; }
static inline int ldk_of(int64_t rows) { return kext_rows(rows) + 64; }

// Split factor of a split-engine product with `tiles` 128 x 128 output tiles
// of mn elements in total, contracted over K grid rows.  The engine holds one
// workgroup per CU (slots / 2 of them, slots counting two FP64 tiles per CU),
// so a launch takes ceil(tiles s / CUs) waves of workgroups: the factor is the
// power of two, with K slices of at least 4096 rows, that minimises the
// modelled time waves (K / s) t_row + s mn 16 B / bw (the partial sums'
// write and read), a larger one taken only for a modelled gain above 2 %.
// t_row is the measured time of one tile per K row (FP16x3 34 ns, BF16x6
// 51 ns); e.g. the 136 lower tiles of a 2048 x 2048 H over 262144 rows run in
// 9 waves of 16 slices instead of 3 waves of 4.
static int split_k_for(int64_t tiles, int64_t K, int64_t mn, int slots, int mode) {
  const int64_t cus = slots / 2 > 0 ? slots / 2 : 1;
  const double t_row = mode == SPLIT_BF16X6 ? 51e-9 : 34e-9;
  const double bw = 4e12;
  int best = 1;
  double best_t = (double)ceil_div(tiles, cus) * (double)K * t_row;
  for (int s = 2; s <= MAX_SPLITS && ceil_div(K, s) >= 4096; s *= 2) {
    const double t = (double)ceil_div(tiles * s, cus) * ((double)K / s) * t_row + s * (double)mn * 16.0 / bw;
    if (t < 0.98 * best_t) {
      best = s;
      best_t = t;
    }
  }
  return best;
}

static unsigned blocks_for(int64_t n) {
  int64_t b = ceil_div(n, 256);
  return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

// Workgroup slots of the current device: two 128 x 128 FP64 tiles per CU.
static int device_slots() {
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cu <= 0)
    cu = 256;
  return 2 * cu;
}

// Split-K factor of a 128 x 128-tiled product with `tiles` output tiles of
// mn elements in total and K-deep sums: 1 or a multiple of 8 (one K slice per
// XCD at a time), slices of at least 512 rows, chosen to minimise
// the modelled time ceil(tiles s / slots) (K / s) t_row + s mn 16 B / bw,
// i.e. whole waves of workgroups against the partial sums' write and read.
static int splits_for(int64_t tiles, int64_t K, int64_t mn, int slots) {
  const double t_row = 2.0 * 128 * 128 / (60e12 / slots);  // s per k-row and tile
  const double bw = 4e12;                                   // B/s for the partials
  int best = 1;
  double best_t = 0.0;
  for (int s = 1; s <= MAX_SPLITS; s = s < 8 ? 8 : s + 8) {
    if (s > 1 && ceil_div(K, s) < 512) break;
    const double waves = (double)ceil_div(tiles * s, (int64_t)slots);
    const double t = waves * ((double)K / s) * t_row + (s > 1 ? s * (double)mn * 16.0 / bw : 0.0);
    if (s == 1 || t < best_t * (1.0 - 1e-9)) {
      best = s;
      best_t = t;
    }
  }
  return best;
}

// Split factors the adjoint uses for blocks of `rows` rows.
struct BwdSplits {
  int h;  // Theta^T S (general) or H = G^T g G (fused, lower tiles)
  int q;  // Abar^T X per orbital set
};

static BwdSplits bwd_splits(int64_t rows, int64_t n1, int n_mu, int n, bool fused, int slots) {
  const int64_t t1 = ceil_div(n1, 128);
  BwdSplits b;
  b.h = splits_for(fused ? gemm_tiles((int)t1, (int)t1, 1) : t1 * t1, rows, n1 * n1, slots);
  b.q = splits_for(ceil_div(2 * (int64_t)n_mu, 128) * ceil_div(2 * (int64_t)n, 128), rows,
                   2 * (int64_t)n_mu * 2 * n, slots);
  return b;
}

// Planes of the adjoint's orbital products dX = Abar F (split precisions):
// the r-block's Abar (or Bbar) rows and the packed F of each orbital set,
// all with K = 2 N_mu rounded up to 32 (kx) and row pitch ldp.
struct AdjPlanes {
  void* abar;   // [NP][rows_cap][ldp]
  void* f_phi;  // [NP][2 n_phi][ldp]
  void* f_psi;  // [NP][2 n_psi][ldp]
  int ldp, kx;
  int64_t rows_cap;
};

static AdjPlanes carve_adj(Carver& c, isdf_prec prec, int n_phi, int n_psi, bool aliased, int n_mu,
                           int64_t rows_cap) {
  AdjPlanes a{};
  if (prec != ISDF_P_BF16X6 && prec != ISDF_P_FP16X3) return a;
  const int np = prec == ISDF_P_BF16X6 ? 3 : 2;
  a.ldp = ldp_of(n_mu);
  a.kx = kext_of(n_mu);
  a.rows_cap = rows_cap;
  a.abar = c.take<char>(plane_bytes(np, rows_cap, a.ldp));
  a.f_phi = c.take<char>(plane_bytes(np, 2 * (int64_t)n_phi, a.ldp));
  a.f_psi = aliased ? a.f_phi : c.take<char>(plane_bytes(np, 2 * (int64_t)n_psi, a.ldp));
  return a;
}

struct BwdPlan {
  FitState* st;
  int* marker;   // [N_r] occupancy of the interpolation rows (check_idx)
  void *Ephi, *Epsi, *Fphi, *Fpsi, *Xphi, *Xpsi;
  double *G, *Th, *A, *B, *P, *Ppart, *Qphi, *Qpsi, *Qpart, *Amu, *Bmu, *dA, *dB, *T1, *lpart, *W2;
  // binary16 split: operand maxima and power-of-two scales
  //  amax [8]: block rows of Phi, Psi; interpolation rows (E) of Phi, Psi; Abar, Bbar; g G, G
  //  sc [20]: Gram (rows Phi, E_phi, rows Psi, E_psi); Abar F (Abar, E_phi, Bbar, E_psi);
  //           Abar^T X (Abar, rows Phi, Bbar, rows Psi); H (g G, G, -, -); Gram of the
  //           interpolation rows (E_phi, E_phi, E_psi, E_psi)
  double* amax;
  double* sc;
  void* tp;      // transposed planes of the products over grid rows (H, Abar^T X), split precisions
  double* tpart; // split-K partials of those products (null: never split)
  SplitWork sw;  // orbital-row and Gram right-hand-side planes (split precisions)
  AdjPlanes ap;  // Abar / Bbar and F planes (split precisions)
  int slots;     // workgroup slots the split factors were chosen for
  size_t bytes;
};

static BwdPlan plan_bwd(void* ws, size_t cap, int64_t nr, int n_mu, int n_phi, int n_psi, bool aliased,
                        isdf_prec prec, int64_t rblock, int slots, bool saved = false) {
  const size_t tsize = tsize_of(prec);
  // largest split factors over the block sizes that occur (both losses)
  int sh = 1, sq = 1;
  for (int64_t rows : {rblock, nr - (ceil_div(nr, rblock) - 1) * rblock})
    for (bool fused : {false, true}) {
      const int64_t n1b = aliased ? n_mu : 2 * (int64_t)n_mu;
      const BwdSplits b1 = bwd_splits(rows, n1b, n_mu, n_phi, fused, slots);
      const BwdSplits b2 = bwd_splits(rows, n1b, n_mu, n_psi, fused, slots);
      sh = b1.h > sh ? b1.h : sh;
      sq = b1.q > sq ? b1.q : sq;
      sq = b2.q > sq ? b2.q : sq;
    }
  Carver c(ws, cap);
  BwdPlan P{};
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  const int64_t n1 = aliased ? n_mu : 2 * (int64_t)n_mu;
  const int nmax = n_phi > n_psi ? n_phi : n_psi;
  P.st = c.take<FitState>(1);
  P.marker = c.take<int>(nr);
  P.amax = c.take<double>(8);
  P.sc = c.take<double>(20);
  P.Ephi = c.take<char>((size_t)2 * nmu16 * 2 * n_phi * tsize);
  P.Fphi = c.take<char>((size_t)2 * n_phi * 2 * n_mu * tsize);
  P.Xphi = c.take<char>((size_t)n_mu * 2 * n_phi * tsize);
  if (!aliased) {
    P.Epsi = c.take<char>((size_t)2 * nmu16 * 2 * n_psi * tsize);
    P.Fpsi = c.take<char>((size_t)2 * n_psi * 2 * n_mu * tsize);
    P.Xpsi = c.take<char>((size_t)n_mu * 2 * n_psi * tsize);
  }
  if (!saved) {  // else the caller's saved Gram blocks stand in for G, A, B
    P.G = c.take<double>((size_t)rblock * n1);
    P.A = c.take<double>((size_t)rblock * 2 * n_mu);
    if (!aliased) P.B = c.take<double>((size_t)rblock * 2 * n_mu);
  }
  P.Th = c.take<double>((size_t)rblock * n1);
  P.P = c.take<double>((size_t)n1 * n1);
  P.W2 = c.take<double>((size_t)n1 * n1);
  P.Ppart = c.take<double>((size_t)sh * n1 * n1);
  P.slots = slots;
  P.Qphi = c.take<double>((size_t)2 * n_mu * 2 * n_phi);
  if (!aliased) P.Qpsi = c.take<double>((size_t)2 * n_mu * 2 * n_psi);
  P.Qpart = c.take<double>((size_t)sq * 2 * n_mu * 2 * nmax);
  P.Amu = c.take<double>((size_t)n_mu * 2 * n_mu);
  if (!aliased) P.Bmu = c.take<double>((size_t)n_mu * 2 * n_mu);
  P.dA = c.take<double>((size_t)n_mu * 2 * n_mu);
  if (!aliased) P.dB = c.take<double>((size_t)n_mu * 2 * n_mu);
  P.T1 = c.take<double>((size_t)n_mu * 2 * nmax);
  P.lpart = c.take<double>((size_t)ceil_div(rblock, 128) * ceil_div(n1, 128));
  P.sw = carve_split(c, prec, n_phi, n_psi, aliased, n_mu, rblock > n_mu ? rblock : n_mu);
  P.ap = carve_adj(c, prec, n_phi, n_psi, aliased, n_mu, rblock);
  if (prec == ISDF_P_BF16X6 || prec == ISDF_P_FP16X3) {
    // one buffer serves H's two operands and then each orbital set's Abar^T X
    const int np = prec == ISDF_P_BF16X6 ? 3 : 2;
    const int64_t cols = 2 * n1 > 2 * (int64_t)n_mu + 2 * nmax ? 2 * n1 : 2 * (int64_t)n_mu + 2 * nmax;
    P.tp = c.take<char>((size_t)np * cols * ldk_of(rblock) * 2);
    // split-K partials: the largest split factor over the block sizes that
    // occur, with the output tile split_xty launches for this precision
    const int bm = SplitTile<SPLIT_FP16X3>::BM, bn = SplitTile<SPLIT_FP16X3>::BN;
    static_assert(SplitTile<SPLIT_BF16X6>::BM == bm && SplitTile<SPLIT_BF16X6>::BN == bn, "one tile");
    // (Abar^T X per orbital set: a set with fewer columns has fewer tiles and
    // may take a larger factor, so both sets are sized)
    const int mode = prec == ISDF_P_BF16X6 ? SPLIT_BF16X6 : SPLIT_FP16X3;
    const int64_t th = split_tiles((int)ceil_div(n1, bm), (int)ceil_div(n1, bn), bm / bn, 1);
    int64_t need = 0;
    for (int64_t rows : {rblock, nr - (ceil_div(nr, rblock) - 1) * rblock}) {
      const int sh2 = split_k_for(th, kext_rows(rows), n1 * n1, slots, mode);
      if (sh2 > 1 && sh2 * n1 * n1 > need) need = sh2 * n1 * n1;
      for (int n : {n_phi, aliased ? n_phi : n_psi}) {
        const int64_t mn = 2 * (int64_t)n_mu * 2 * n;
        const int64_t tq = ceil_div(2 * (int64_t)n_mu, bm) * ceil_div(2 * (int64_t)n, bn);
        const int sq2 = split_k_for(tq, kext_rows(rows), mn, slots, mode);
        if (sq2 > 1 && sq2 * mn > need) need = sq2 * mn;
      }
    }
    if (need > 0) P.tpart = c.take<double>((size_t)need);
  }
  P.bytes = c.used;
  return P;
}

// Transposed split of X (and, with out2, of X without its row scale in the
// same pass).
template <int SPLIT, class TS>
static bool split_t(const TS* x, int64_t ld, int ncols, int rows, const double* rowscale, void* out, int ldk,
                    const double* scale, hipStream_t s, void* out2 = nullptr, const double* scale2 = nullptr) {
  typedef typename SplitT<SPLIT>::P P;
  dim3 grid((unsigned)ceil_div(ldk, 64), (unsigned)ceil_div(ncols, 64));
  const int64_t ps = (int64_t)ncols * ldk;
  if (out2)
    hipLaunchKernelGGL((split_planes_t<SPLIT, TS, T_DUAL>), grid, dim3(256), 0, s, x, ld, ncols, rows, rowscale,
                       (P*)out, ldk, ps, scale, (P*)out2, ldk, ps, scale2);
  else
    hipLaunchKernelGGL((split_planes_t<SPLIT, TS, T_ONE>), grid, dim3(256), 0, s, x, ld, ncols, rows, rowscale,
                       (P*)out, ldk, ps, scale, (P*)nullptr, 0, (int64_t)0, (const double*)nullptr);
  return launch_ok();
}

// Transposed planes of X (out, as split_t) and its row planes (rout [NP]
// [rows_cap][ldp], as split_rows) from one read of X.
template <int SPLIT>
static bool split_t_rows(const double* x, int64_t ld, int ncols, int rows, void* out, int ldk, const double* scale,
                         void* rout, int ldp, int64_t rows_cap, const double* rscale, hipStream_t s) {
  typedef typename SplitT<SPLIT>::P P;
  if (ldp % 8 != 0 || ldp > ceil_div(ncols, 64) * 64 || rows > rows_cap) return false;
  dim3 grid((unsigned)ceil_div(ldk, 64), (unsigned)ceil_div(ncols, 64));
  hipLaunchKernelGGL((split_planes_t<SPLIT, double, T_ROWS>), grid, dim3(256), 0, s, x, ld, ncols, rows,
                     (const double*)nullptr, (P*)out, ldk, (int64_t)ncols * ldk, scale, (P*)rout, ldp,
                     rows_cap * ldp, rscale);
  return launch_ok();
}

// C (=, or += when accumulate) X^T Y over the `rows` grid rows of r-major
// blocks X [rows][mx] and Y [rows][ny], on 16-bit matrix cores: both split
// transposed into `tp` (X scaled by rowscale when given; binary16 operand
// scales sc[0], sc[1]), then one split product, split over K into partial
// slices (fixed-order reduction) when split_k_for finds whole waves of
// workgroups better filled that way.  lower_only (X = Y up to rowscale,
// mx = ny): the lower tiles only.  x_split: X's planes are in tp already.
template <int SPLIT, class TY>
static bool split_xty(const double* X, int64_t ldx, int mx, const double* rowscale, const TY* Y, int64_t ldy, int ny,
                      int rows, double* C, int64_t ldc, bool accumulate, int lower_only, void* tp, double* part,
                      const double* sc, int slots, const int* ab, hipStream_t s, bool x_split = false) {
  typedef typename SplitT<SPLIT>::P P;
  constexpr int NP = SplitT<SPLIT>::NP;
  const int ldk = ldk_of(rows);
  P* ta = (P*)tp;
  P* tb = ta + (int64_t)NP * mx * ldk;
  if (x_split) {  // X's planes are in tp already (split_t_rows)
    if (!split_t<SPLIT>(Y, ldy, ny, rows, nullptr, tb, ldk, sc ? sc + 1 : nullptr, s)) return false;
  } else if ((const void*)X == (const void*)Y && sizeof(TY) == sizeof(double) && ldx == ldy && mx == ny) {
    // X^T diag(g) X: both operands' planes from one read of X
    if (!split_t<SPLIT>(X, ldx, mx, rows, rowscale, ta, ldk, sc, s, tb, sc ? sc + 1 : nullptr)) return false;
  } else {
    if (!split_t<SPLIT>(X, ldx, mx, rows, rowscale, ta, ldk, sc, s)) return false;
    if (!split_t<SPLIT>(Y, ldy, ny, rows, nullptr, tb, ldk, sc ? sc + 1 : nullptr, s)) return false;
  }
  PlaneOp<P> a{ta, ldk, (int64_t)mx * ldk, nullptr}, b{tb, ldk, (int64_t)ny * ldk, nullptr};
  typedef SplitTile<SPLIT> T;
  const int kx = kext_rows(rows);
  const int64_t tiles =
      split_tiles((int)ceil_div(mx, T::BM), (int)ceil_div(ny, T::BN), T::BM / T::BN, lower_only && mx == ny);
  const int sp = part ? split_k_for(tiles, kx, (int64_t)mx * ny, slots, SPLIT) : 1;
  const int64_t cn = (int64_t)mx * ldc;
  if (sp == 1) {
    EpiStore<double> epi{C, ldc, mx, ny, 1.0, accumulate ? 1.0 : 0.0, nullptr, 0, 0};
    return launch_split<SPLIT, T::BM, T::BN, T::WM, T::WN, 1>(mx, ny, kx, a, b, a, b, 0, sc, epi, ab, s, lower_only);
  }
  EpiStore<double> epi{part, ldc, mx, ny, 1.0, 0.0, nullptr, cn, 0};
  if (!launch_split<SPLIT, T::BM, T::BN, T::WM, T::WN, 1>(mx, ny, kx, a, b, a, b, 0, sc, epi, ab, s, lower_only, sp))
    return false;
  hipLaunchKernelGGL(reduce_splits, dim3(blocks_for(cn)), dim3(256), 0, s, C, (const double*)part, cn, sp,
                     accumulate ? 1 : 0, ab);
  return launch_ok();
}

// dX rows = Abar F (Abar: rows x 2 N_mu real form, F: packed Phi_mu) in the
// orbital precision.  Split precisions: Abar is split into planes here, F's
// planes (fplanes) were split once per call; scales = binary16 operand
// scales (s_Abar, s_F), FP16 split only.
template <int PREC, class TS>
static bool adj_rows(int rows, const double* Abar, int n_mu, const typename Prec<PREC>::E* F, const void* fplanes,
                     int n, TS* dX, int64_t ld_dx, const double* scales, const AdjPlanes& ap, const int* ab,
                     hipStream_t s, bool abar_split = false) {
  typedef typename Prec<PREC>::E T;
  constexpr int SPLIT = Prec<PREC>::SPLIT;
  const int64_t two_mu = 2 * (int64_t)n_mu;
  if constexpr (SPLIT >= 0) {
    typedef typename SplitT<SPLIT>::P P;
    const double* sc = SPLIT == SPLIT_FP16X3 ? scales : nullptr;
    if (!abar_split &&
        !split_rows<SPLIT, double>(Abar, n_mu, n_mu, nullptr, rows, 0, rows, ap.abar, ap.ldp, ap.rows_cap, sc, s))
      return false;
    EpiStore<TS> epi{dX, 2 * ld_dx, rows, 2 * n, 1.0, 0.0, nullptr, 0, 0};
    PlaneOp<P> a{(const P*)ap.abar, ap.ldp, ap.rows_cap * ap.ldp, nullptr};
    PlaneOp<P> b{(const P*)fplanes, ap.ldp, 2 * (int64_t)n * ap.ldp, nullptr};
    typedef SplitTile<SPLIT> T;
    return launch_split<SPLIT, T::BM, T::BN, T::WM, T::WN, 1>(rows, 2 * n, ap.kx, a, b, a, b, 0, sc, epi, ab, s);
  } else {
    (void)fplanes;
    (void)ap;
    return tgemm<T, KC, KC>(rows, 2 * n, two_mu, Abar, two_mu, F, two_mu, dX, 2 * ld_dx, 1.0, 0.0, ab, s);
  }
}

// One orbital set's share of the block: dX rows = Abar F, Q += Abar^T X
// (split precisions: both on 16-bit matrix cores, Abar^T X through
// transposed planes; else Abar^T X in the compute type, split over K).
template <int PREC, class TS>
static bool orbital_block(const double* Abar, int n_mu, const typename Prec<PREC>::E* F, const void* fplanes,
                          const TS* X, int64_t ld_x, int n, TS* dX, int64_t ld_dx, int64_t r, int rows, double* Q,
                          double* Qpart, const double* scales, const double* scales_t, const AdjPlanes& ap, int sp,
                          bool first, void* tp, double* tpart, int slots, const int* ab, hipStream_t s) {
  const int64_t two_mu = 2 * (int64_t)n_mu;
  constexpr int SPLIT = Prec<PREC>::SPLIT;
  if constexpr (SPLIT >= 0) {
    // Abar's transposed planes (Abar^T X) and row planes (Abar F) from one
    // read of Abar; binary16 scales (s_Abar, s_X) = scales_t[0..1], (s_Abar,
    // s_F) = scales[0..1]
    const bool h = SPLIT == SPLIT_FP16X3;
    if (!split_t_rows<SPLIT>(Abar, two_mu, (int)two_mu, rows, tp, ldk_of(rows), h ? scales_t : nullptr, ap.abar,
                             ap.ldp, ap.rows_cap, h ? scales : nullptr, s))
      return false;
    if (!adj_rows<PREC, TS>(rows, Abar, n_mu, F, fplanes, n, dX + 2 * r * ld_dx, ld_dx, scales, ap, ab, s, true))
      return false;
    return split_xty<SPLIT, TS>(Abar, two_mu, (int)two_mu, nullptr, X + 2 * r * ld_x, 2 * ld_x, 2 * n, rows, Q,
                                2 * (int64_t)n, !first, 0, tp, tpart, h ? scales_t : nullptr, slots, ab, s, true);
  } else {
    if (!adj_rows<PREC, TS>(rows, Abar, n_mu, F, fplanes, n, dX + 2 * r * ld_dx, ld_dx, scales, ap, ab, s))
      return false;
    (void)scales_t;
    (void)tp;
    (void)tpart;
    (void)slots;
    const int64_t qn = two_mu * 2 * n;
    if (!tgemm<typename Prec<PREC>::Q, XC, XC>((int)two_mu, 2 * n, rows, Abar, two_mu, X + 2 * r * ld_x, 2 * ld_x,
                                               Qpart, 2 * (int64_t)n, 1.0, 0.0, ab, s, sp, qn))
      return false;
    hipLaunchKernelGGL(reduce_splits, dim3(blocks_for(qn)), dim3(256), 0, s, Q, Qpart, qn, sp, first ? 0 : 1, ab);
    return launch_ok();
  }
}

// Mbar terms of one orbital set at the interpolation rows (small: N_mu rows).
template <int PREC, class TS>
static bool orbital_fix(const double* dAbar, int n_mu, const typename Prec<PREC>::E* F,
                        const typename Prec<PREC>::E* Xmu, int n, TS* dX, int64_t ld_dx, const int32_t* idx, int64_t nr,
                        double* Q, double* T1, const int* ab, hipStream_t s) {
  typedef typename Prec<PREC>::E T;
  const int64_t two_mu = 2 * (int64_t)n_mu;
  if (!tgemm<T, KC, KC>(n_mu, 2 * n, two_mu, dAbar, two_mu, F, two_mu, T1, 2 * (int64_t)n, 1.0, 0.0, ab, s))
    return false;
  if (!tgemm<T, XC, XC>((int)two_mu, 2 * n, n_mu, dAbar, two_mu, Xmu, 2 * (int64_t)n, Q, 2 * (int64_t)n, 1.0, 1.0,
                        ab, s))
    return false;
  hipLaunchKernelGGL(scatter_rows<TS>, dim3(blocks_for((int64_t)n_mu * n)), dim3(256), 0, s, dX, ld_dx, n, idx, n_mu,
                     nr, (const double*)Q, (const double*)T1, ab);
  return launch_ok();
}

// Phases of one adjoint call: BWD_BEGIN sets up (state, index check, packed
// right-hand sides, (C C^H)^-2) and starts the reductions, BWD_END applies the
// Mbar terms at the interpolation rows and writes info; the rows
// [row_lo, row_hi) in between are processed rblock at a time.  G, A, B (and
// theta_bar) rows are read from Gs + (r - gbase) n1 etc. when given (kept
// from the forward), else recomputed into the workspace.
enum { BWD_BEGIN = 1, BWD_END = 2 };

template <int PREC, class TS, class TT>
static int bwd_run(int64_t nr, const TS* phi, int64_t ld_phi, int n_phi, const TS* psi, int64_t ld_psi, int n_psi,
                   bool aliased, const int32_t* idx, int n_mu, const double* minv, const TT* tbar, int64_t ld_tbar,
                   const double* g, TS* dphi, int64_t ld_dphi, TS* dpsi, int64_t ld_dpsi, double* loss,
                   int64_t rblock, double* Gs, double* As, double* Bs, isdf_fit_info* info, const BwdPlan& P,
                   int64_t row_lo, int64_t row_hi, int64_t gbase, unsigned phases, hipStream_t s) {
  const int nmu16 = (int)ceil_div(n_mu, 16) * 16;
  const int n1 = aliased ? n_mu : 2 * n_mu;
  const int* ab = &P.st->abort;
  typedef typename Prec<PREC>::E T;
  T *Ephi = (T*)P.Ephi, *Fphi = (T*)P.Fphi, *Xphi = (T*)P.Xphi;
  T *Epsi = aliased ? Ephi : (T*)P.Epsi, *Fpsi = aliased ? Fphi : (T*)P.Fpsi, *Xpsi = aliased ? Xphi : (T*)P.Xpsi;
  if (phases & BWD_BEGIN) {
    hipLaunchKernelGGL(fit_state_init, dim3(1), dim3(1), 0, s, P.st);
    // interpolation indices must be distinct grid points: every launch that
    // reads or writes rows through idx is a no-op once check_idx has aborted
    // the call, and fit_finish reports ISDF_E_BAD_IDX
    if (!fill<int>(P.marker, nr, 0, s)) return ISDF_E_HIP;
    hipLaunchKernelGGL(check_idx, dim3((unsigned)ceil_div(n_mu, 256)), dim3(256), 0, s, idx, n_mu, nr, P.marker, P.st);
    if (!pack<TS, T>(phi, ld_phi, n_phi, idx, n_mu, nr, nmu16, Ephi, s)) return ISDF_E_HIP;
    hipLaunchKernelGGL((pack_adj_rhs<TS, T>), dim3(blocks_for((int64_t)4 * n_phi * n_mu)), dim3(256), 0, s, phi,
                       ld_phi, n_phi, idx, n_mu, nr, Fphi);
    hipLaunchKernelGGL((gather_rows<TS, T>), dim3(blocks_for((int64_t)2 * n_phi * n_mu)), dim3(256), 0, s, phi,
                       ld_phi, n_phi, idx, n_mu, nr, Xphi);
    if (!aliased) {
      if (!pack<TS, T>(psi, ld_psi, n_psi, idx, n_mu, nr, nmu16, Epsi, s)) return ISDF_E_HIP;
      hipLaunchKernelGGL((pack_adj_rhs<TS, T>), dim3(blocks_for((int64_t)4 * n_psi * n_mu)), dim3(256), 0, s, psi,
                         ld_psi, n_psi, idx, n_mu, nr, Fpsi);
      hipLaunchKernelGGL((gather_rows<TS, T>), dim3(blocks_for((int64_t)2 * n_psi * n_mu)), dim3(256), 0, s, psi,
                         ld_psi, n_psi, idx, n_mu, nr, Xpsi);
    }
    if (!launch_ok()) return ISDF_E_HIP;
    // binary16 scales of the interpolation rows (E, F, the rows' Gram at the
    // end); the grid rows' scales follow block by block
    if (!gram_scales_rows<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, 0, 0, (const double*)Ephi,
                                    (const double*)Epsi, nmu16, P.amax, P.sc, s))
      return ISDF_E_HIP;
    if (Prec<PREC>::SPLIT == SPLIT_FP16X3)
      hipLaunchKernelGGL(pow2_scales, dim3(1), dim3(1), 0, s, (const double*)P.amax, P.sc + 16, 2, 2,
                         aliased ? 2 : 3, aliased ? 2 : 3);
    if (!split_rhs<PREC>((const double*)Ephi, (const double*)Epsi, n_phi, n_psi, aliased, P.sc, &P.sw, s))
      return ISDF_E_HIP;
    if constexpr (Prec<PREC>::SPLIT >= 0) {  // F planes, scaled like the orbitals (sc[1], sc[3])
      constexpr int SPLIT = Prec<PREC>::SPLIT;
      const double* sc = SPLIT == SPLIT_FP16X3 ? P.sc : nullptr;
      if (!split_rows<SPLIT, double>((const double*)Fphi, n_mu, n_mu, nullptr, 2 * n_phi, 0, 2 * n_phi, P.ap.f_phi,
                                     P.ap.ldp, 2 * n_phi, sc ? sc + 1 : nullptr, s))
        return ISDF_E_HIP;
      if (!aliased && !split_rows<SPLIT, double>((const double*)Fpsi, n_mu, n_mu, nullptr, 2 * n_psi, 0, 2 * n_psi,
                                                 P.ap.f_psi, P.ap.ldp, 2 * n_psi, sc ? sc + 3 : nullptr, s))
        return ISDF_E_HIP;
    }
    if (!tbar && !dgemm<KC, KC, double>(n1, n1, n1, minv, n1, minv, n1, P.W2, n1, 1.0, 0.0, 0, ab, s))
      return ISDF_E_HIP;  // (C C^H)^-2
  }  // BWD_BEGIN
  for (int64_t r = row_lo; r < row_hi; r += rblock) {
    const int rows = (int)(row_hi - r < rblock ? row_hi - r : rblock);
    const bool first = (phases & BWD_BEGIN) && r == row_lo;  // the reductions start here
    // Gram blocks of the r-block: A (and B) kept, G for Theta; saved by the
    // forward (isdf_zc_ab) or recomputed here
    double* Gb = Gs ? Gs + (r - gbase) * n1 : P.G;
    double* Ab = As ? As + (r - gbase) * 2 * n_mu : P.A;
    double* Bb = aliased ? nullptr : (Bs ? Bs + (r - gbase) * 2 * n_mu : P.B);
    double* Abar = aliased ? Ab : Bb;  // after the Hadamard step
    double* Bbar = Ab;
    // binary16 scales of this block's orbital rows (sc[0], sc[2])
    if (!gram_scales_rows<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, r, rows, (const double*)Ephi,
                                    (const double*)Epsi, nmu16, P.amax, P.sc, s))
      return ISDF_E_HIP;
    if (!Gs && !gram<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, Ephi, Epsi, nmu16, n_mu, nullptr, nr,
                               r, rows, Gb, n1, aliased ? G_REAL : G_CPLX, ab, s, P.sc, &P.sw, Ab, Bb))
      return ISDF_E_HIP;
    const BwdSplits sp_phi = bwd_splits(rows, n1, n_mu, n_phi, !tbar, P.slots);
    const BwdSplits sp_psi = bwd_splits(rows, n1, n_mu, n_psi, !tbar, P.slots);
    constexpr int SPLIT = Prec<PREC>::SPLIT;
    if (!tbar) {
      // H += G^T diag(g) G (lower tiles, fixed-order reduction): FP64 split-K,
      // or, with split orbital contractions, on 16-bit matrix cores like them
      // (a sum of non-negative terms; nothing here involves (C C^H)^-1)
      if constexpr (SPLIT >= 0) {
        const double* hsc = nullptr;
        if (SPLIT == SPLIT_FP16X3) {  // binary16 scales of g G and G
          if (!fill<double>(P.amax + 6, 2, 0.0, s)) return ISDF_E_HIP;
          hipLaunchKernelGGL(absmax_real2, dim3((unsigned)(rows < 2048 ? rows : 2048)), dim3(256), 0, s,
                             (const double*)Gb, (int64_t)n1, n1, (int64_t)rows, g + r, P.amax + 6);
          hipLaunchKernelGGL(pow2_scales, dim3(1), dim3(1), 0, s, (const double*)P.amax, P.sc + 12, 6, 7, 6, 7);
          if (!launch_ok()) return ISDF_E_HIP;
          hsc = P.sc + 12;
        }
        if (!split_xty<SPLIT, double>(Gb, n1, n1, g + r, Gb, n1, n1, rows, P.P, n1, !first, 1, P.tp, P.tpart, hsc,
                                      P.slots, ab, s))
          return ISDF_E_HIP;
      } else {
        const int sp = sp_phi.h;
        const int64_t pn = (int64_t)n1 * n1;
        if (!tgemm<double, XC, XC>(n1, n1, rows, Gb, n1, Gb, n1, P.Ppart, n1, 1.0, 0.0, ab, s, sp, pn, g + r, 1))
          return ISDF_E_HIP;
        hipLaunchKernelGGL(reduce_splits, dim3(blocks_for(pn)), dim3(256), 0, s, P.P, P.Ppart, pn, sp,
                           first ? 0 : 1, ab);
      }
      // S = 2 g . (G (C C^H)^-2): Abar / Bbar in place, the loss and (binary16
      // split) the largest |Abar|, |Bbar| for their scales, in the epilogue
      if (SPLIT == SPLIT_FP16X3 && !fill<double>(P.amax + 4, 2, 0.0, s)) return ISDF_E_HIP;
      EpiSAdj epi{Gb,  n1, Ab, Bb, 2 * (int64_t)n_mu, g + r, rows, n1, aliased ? 1 : 0, P.lpart,
                  SPLIT == SPLIT_FP16X3 ? P.amax + 4 : nullptr};
      Operand<double> a{Gb, n1, nullptr, nullptr}, b{P.W2, n1, nullptr, nullptr};
      if (!launch_gemm<double, 128, 128, 16, 2, 2, double, KC, double, KC, 1>(rows, n1, n1, a, b, a, b, 0, epi, 0, ab,
                                                                             s))
        return ISDF_E_HIP;
      const int ltiles = (int)(ceil_div(rows, 128) * ceil_div(n1, 128));
      hipLaunchKernelGGL(add_loss, dim3(1), dim3(LOSS_THREADS), 0, s, P.st, (const double*)P.lpart, ltiles);
      if (!launch_ok()) return ISDF_E_HIP;
    } else {
      // Theta = G M^-1, S = Thetabar M^-1 (over G), P += Theta^T S, Abar / Bbar in place
      if (!dgemm<KC, KC, double>(rows, n1, n1, Gb, n1, minv, n1, P.Th, n1, 1.0, 0.0, 0, ab, s)) return ISDF_E_HIP;
      const int64_t ldt = aliased ? ld_tbar : 2 * ld_tbar;
      if (!dgemm<KC, KC, double, TT>(rows, n1, n1, tbar + (r - gbase) * ldt, ldt, minv, n1, Gb, n1, 1.0, 0.0, 0, ab,
                                     s))
        return ISDF_E_HIP;
      const int sp = sp_phi.h;
      const int64_t pn = (int64_t)n1 * n1;
      if (!tgemm<double, XC, XC>(n1, n1, rows, P.Th, n1, Gb, n1, P.Ppart, n1, 1.0, 0.0, ab, s, sp, pn))
        return ISDF_E_HIP;
      hipLaunchKernelGGL(reduce_splits, dim3(blocks_for(pn)), dim3(256), 0, s, P.P, P.Ppart, pn, sp, first ? 0 : 1,
                         ab);
      hipLaunchKernelGGL(adj_hadamard, dim3(blocks_for((int64_t)rows * n_mu)), dim3(256), 0, s, (const double*)Gb,
                         Ab, Bb, (int64_t)rows, n_mu, aliased ? 1 : 0);
      if (!launch_ok()) return ISDF_E_HIP;
    }
    if (SPLIT == SPLIT_FP16X3) {  // binary16 scales of Abar, Phi, Bbar, Psi
      if (tbar) {  // (the fused loss found the maxima in its epilogue)
        if (!fill<double>(P.amax + 4, 2, 0.0, s)) return ISDF_E_HIP;
        if (!absmax<double>(Abar, n_mu, n_mu, rows, P.amax + 4, s)) return ISDF_E_HIP;
        if (!aliased && !absmax<double>(Bbar, n_mu, n_mu, rows, P.amax + 5, s)) return ISDF_E_HIP;
      }
      hipLaunchKernelGGL(pow2_scales, dim3(1), dim3(1), 0, s, (const double*)P.amax, P.sc + 4, 4, 2,
                         aliased ? 4 : 5, aliased ? 2 : 3);
      hipLaunchKernelGGL(pow2_scales, dim3(1), dim3(1), 0, s, (const double*)P.amax, P.sc + 8, 4, 0,
                         aliased ? 4 : 5, aliased ? 0 : 1);
    }
    if (!orbital_block<PREC, TS>(Abar, n_mu, Fphi, P.ap.f_phi, phi, ld_phi, n_phi, dphi, ld_dphi, r, rows, P.Qphi,
                                 P.Qpart, P.sc + 4, P.sc + 8, P.ap, sp_phi.q, first, P.tp, P.tpart, P.slots, ab, s))
      return ISDF_E_HIP;
    if (!aliased && !orbital_block<PREC, TS>(Bbar, n_mu, Fpsi, P.ap.f_psi, psi, ld_psi, n_psi, dpsi, ld_dpsi, r, rows,
                                             P.Qpsi, P.Qpart, P.sc + 6, P.sc + 10, P.ap, sp_psi.q, first, P.tp,
                                             P.tpart, P.slots, ab, s))
      return ISDF_E_HIP;
  }
  if (!(phases & BWD_END)) return ISDF_OK;
  if (!tbar) {
    // Theta^T S = 2 M^-1 H M^-2 with H = G^T diag(g) G
    const int64_t pn = (int64_t)n1 * n1;
    hipLaunchKernelGGL(mirror_lower, dim3(blocks_for(pn)), dim3(256), 0, s, P.P, n1, ab);
    if (!dgemm<KC, KC, double>(n1, n1, n1, P.P, n1, P.W2, n1, P.Ppart, n1, 1.0, 0.0, 0, ab, s)) return ISDF_E_HIP;
    if (!dgemm<KC, XC, double>(n1, n1, n1, minv, n1, P.Ppart, n1, P.P, n1, 2.0, 0.0, 0, ab, s)) return ISDF_E_HIP;
  }
  // Mbar terms at the interpolation rows
  if (!gram<PREC, TS>(phi, ld_phi, n_phi, psi, ld_psi, n_psi, aliased, Ephi, Epsi, nmu16, n_mu, idx, nr, 0, n_mu,
                      nullptr, n1, G_CPLX, ab, s, P.sc + 16, &P.sw, P.Amu, aliased ? nullptr : P.Bmu))
    return ISDF_E_HIP;
  hipLaunchKernelGGL(mbar_hadamard, dim3(blocks_for((int64_t)n_mu * n_mu)), dim3(256), 0, s, (const double*)P.P,
                     (const double*)P.Amu, (const double*)P.Bmu, P.dA, P.dB, n_mu, aliased ? 1 : 0, ab);
  if (!launch_ok()) return ISDF_E_HIP;
  if (!orbital_fix<PREC, TS>(P.dA, n_mu, Fphi, Xphi, n_phi, dphi, ld_dphi, idx, nr, P.Qphi, P.T1, ab, s))
    return ISDF_E_HIP;
  if (!aliased && !orbital_fix<PREC, TS>(P.dB, n_mu, Fpsi, Xpsi, n_psi, dpsi, ld_dpsi, idx, nr, P.Qpsi, P.T1, ab, s))
    return ISDF_E_HIP;
  if (aliased && dpsi != dphi) {
    hipLaunchKernelGGL((copy_rows<TS>), dim3(blocks_for(nr * 2 * n_phi)), dim3(256), 0, s, dpsi, ld_dpsi,
                       (const TS*)dphi, ld_dphi, nr, n_phi);
  }
  hipLaunchKernelGGL(fit_finish, dim3(1), dim3(1), 0, s, P.st, info, loss, 1);
  if (!launch_ok()) return ISDF_E_HIP;
  return ISDF_OK;
}

static size_t bwd_workspace(const isdf_grid* grid, int32_t n_mu, int32_t n_phi, int32_t n_psi, int32_t aliased,
                            isdf_prec prec, int64_t rblock, bool saved) {
  if (!grid || n_mu <= 0 || n_phi <= 0 || n_psi <= 0 || rblock <= 0) return 0;
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] <= 0) return 0;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  if (rblock > nr) rblock = nr;
  return plan_bwd(nullptr, 0, nr, n_mu, n_phi, n_psi, aliased != 0, prec, rblock, device_slots(), saved).bytes;
}

static int bwd_dispatch(const isdf_grid* grid, isdf_dtype dt, const void* phi, int64_t ld_phi, int32_t n_phi,
                        const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx, int32_t n_mu,
                        isdf_prec prec, const double* minv, const void* theta_bar, int64_t ld_tbar, const double* g,
                        void* dphi, int64_t ld_dphi, void* dpsi, int64_t ld_dpsi, double* loss, int64_t rblock,
                        double* Gs, double* As, double* Bs, bool saved, isdf_fit_info* info, void* ws,
                        size_t ws_bytes, void* stream, int64_t row0 = 0, int64_t nrows = -1,
                        unsigned phases = BWD_BEGIN | BWD_END) {
  int64_t nr = 0;
  if (!fit_args_ok(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, &nr)) return ISDF_E_ARG;
  if (!minv || !info || !dphi || !dpsi || rblock <= 0) return ISDF_E_ARG;
  if (!theta_bar && !g) return ISDF_E_ARG;
  if (theta_bar && ld_tbar < n_mu) return ISDF_E_ARG;
  if (ld_dphi < n_phi || ld_dpsi < n_psi) return ISDF_E_ARG;
  if (prec == ISDF_P_FP64 && dt != ISDF_C128) return ISDF_E_ARG;
  const bool aliased = phi == psi && ld_phi == ld_psi && n_phi == n_psi;
  if (!aliased && dphi == dpsi) return ISDF_E_ARG;
  if (nrows < 0) nrows = nr;  // the whole grid in one call
  if (row0 < 0 || row0 > nr || nrows > nr - row0) return ISDF_E_ARG;
  if (saved && nrows > 0 && (!Gs || !As || (!aliased && !Bs))) return ISDF_E_ARG;
  if (!saved) Gs = As = Bs = nullptr;
  if (rblock > nr) rblock = nr;
  BwdPlan P = plan_bwd(ws, ws_bytes, nr, n_mu, n_phi, n_psi, aliased, prec, rblock, device_slots(), saved);
  if (!ws || P.bytes > ws_bytes) return ISDF_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
#define ISDF_BWD_ARGS(TS)                                                                                        \
  nr, (const TS*)phi, ld_phi, n_phi, (const TS*)psi, ld_psi, n_psi, aliased, idx, n_mu, minv, (const TS*)theta_bar, \
      ld_tbar, g, (TS*)dphi, ld_dphi, (TS*)dpsi, ld_dpsi, loss, rblock, Gs, As, Bs, info, P, row0, row0 + nrows,      \
      row0, phases, s
  if (dt == ISDF_C128) {
    switch (prec) {
      case ISDF_P_FP64: return bwd_run<ISDF_P_FP64, double, double>(ISDF_BWD_ARGS(double));
      case ISDF_P_FP32: return bwd_run<ISDF_P_FP32, double, double>(ISDF_BWD_ARGS(double));
      case ISDF_P_BF16X6: return bwd_run<ISDF_P_BF16X6, double, double>(ISDF_BWD_ARGS(double));
      default: return bwd_run<ISDF_P_FP16X3, double, double>(ISDF_BWD_ARGS(double));
    }
  }
  switch (prec) {
    case ISDF_P_FP32: return bwd_run<ISDF_P_FP32, float, float>(ISDF_BWD_ARGS(float));
    case ISDF_P_BF16X6: return bwd_run<ISDF_P_BF16X6, float, float>(ISDF_BWD_ARGS(float));
    default: return bwd_run<ISDF_P_FP16X3, float, float>(ISDF_BWD_ARGS(float));
  }
#undef ISDF_BWD_ARGS
}

}  // namespace
}  // namespace isdf

using namespace isdf;

extern "C" size_t isdf_fit_backward_workspace(const isdf_grid* grid, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                                              int32_t aliased, int32_t prec_in, int64_t rblock) {
  if (!prec_valid(prec_in)) return 0;
  const isdf_prec prec = (isdf_prec)prec_in;
  return bwd_workspace(grid, n_mu, n_phi, n_psi, aliased, prec, rblock, false);
}

extern "C" int isdf_fit_backward(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi,
                                 int32_t n_phi, const void* psi, int64_t ld_psi, int32_t n_psi, const int32_t* idx,
                                 int32_t n_mu, int32_t prec_in, const double* minv, const void* theta_bar,
                                 int64_t ld_tbar, const double* g, void* dphi, int64_t ld_dphi, void* dpsi,
                                 int64_t ld_dpsi, double* loss, int64_t rblock, isdf_fit_info* info, void* ws,
                                 size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  if (!prec_valid(prec_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const isdf_prec prec = (isdf_prec)prec_in;
  return bwd_dispatch(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, minv, theta_bar, ld_tbar, g,
                      dphi, ld_dphi, dpsi, ld_dpsi, loss, rblock, nullptr, nullptr, nullptr, false, info, ws, ws_bytes,
                      stream);
}

extern "C" size_t isdf_fit_backward_gram_workspace(const isdf_grid* grid, int32_t n_mu, int32_t n_phi,
                                                   int32_t n_psi, int32_t aliased, int32_t prec_in, int64_t rblock) {
  if (!prec_valid(prec_in)) return 0;
  const isdf_prec prec = (isdf_prec)prec_in;
  return bwd_workspace(grid, n_mu, n_phi, n_psi, aliased, prec, rblock, true);
}

extern "C" int isdf_fit_backward_gram(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi,
                                      int32_t n_phi, const void* psi, int64_t ld_psi, int32_t n_psi,
                                      const int32_t* idx, int32_t n_mu, int32_t prec_in, const double* minv,
                                      const void* theta_bar, int64_t ld_tbar, const double* g, void* dphi,
                                      int64_t ld_dphi, void* dpsi, int64_t ld_dpsi, double* loss, int64_t rblock,
                                      double* G, double* A, double* B, isdf_fit_info* info, void* ws,
                                      size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  if (!prec_valid(prec_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const isdf_prec prec = (isdf_prec)prec_in;
  return bwd_dispatch(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, minv, theta_bar, ld_tbar, g,
                      dphi, ld_dphi, dpsi, ld_dpsi, loss, rblock, G, A, B, true, info, ws, ws_bytes, stream);
}

extern "C" int isdf_fit_backward_rows(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi,
                                      int32_t n_phi, const void* psi, int64_t ld_psi, int32_t n_psi,
                                      const int32_t* idx, int32_t n_mu, int32_t prec_in, const double* minv,
                                      const void* theta_bar, int64_t ld_tbar, const double* g, void* dphi,
                                      int64_t ld_dphi, void* dpsi, int64_t ld_dpsi, double* loss, int64_t row0,
                                      int64_t nrows, int64_t rblock, double* G, double* A, double* B, uint32_t flags,
                                      isdf_fit_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  if (!prec_valid(prec_in)) return ISDF_E_ARG;
  if (flags & ~(ISDF_BWD_FIRST | ISDF_BWD_LAST)) return ISDF_E_ARG;
  if (nrows < 0 || rblock <= 0) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  const isdf_prec prec = (isdf_prec)prec_in;
  const unsigned phases = ((flags & ISDF_BWD_FIRST) ? BWD_BEGIN : 0u) | ((flags & ISDF_BWD_LAST) ? BWD_END : 0u);
  return bwd_dispatch(grid, dt, phi, ld_phi, n_phi, psi, ld_psi, n_psi, idx, n_mu, prec, minv, theta_bar, ld_tbar, g,
                      dphi, ld_dphi, dpsi, ld_dpsi, loss, rblock, G, A, B, true, info, ws, ws_bytes, stream, row0, nrows,
                      phases);
}
