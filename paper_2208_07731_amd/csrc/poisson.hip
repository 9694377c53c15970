// V_mu(r) = int zeta_mu(r') / |r - r'| dr' for every column of Theta
// (eq. V_mu of arXiv:2208.07731, the step after the fit in the paper's
// hybrid-DFT flow), on the periodic grid:
//
//   V-hat(G) = 4 pi zeta-hat(G) / |G|^2,  G = 0 dropped (neutral background).
//
// Theta is r-major [N_r][N_mu] (the fit's layout), so every grid line along
// an axis holds N_mu independent signals side by side.  Five line passes,
// each reading and writing the whole array once (the work is HBM-bound):
//   1. FFT along k   (Theta -> W)          4. inverse FFT along j (W -> W)
//   2. FFT along j   (W -> W)              5. inverse FFT along k (W -> V)
//   3. FFT along i, multiply by 4 pi / (N_r |G|^2), inverse FFT along i
// A workgroup loads one line of n points for 32, 16 or 8 columns (n <= 64,
// 128, 256) into LDS (one 32 KB buffer, passes in place) and runs a
// mixed-radix Stockham FFT (radices 8, 4, 2, 3, 5, 7) there; inverse
// transforms are conj(FFT(conj x)).  Real Theta (Psi = Phi) is packed two
// columns per complex signal: the operator is real and even in G, so the
// real and imaginary parts of the result are the two columns' potentials.
#include <type_traits>

#include "common.h"

namespace isdf {
namespace {

constexpr int FFT_CT = 32;         // column padding of the work array (tiles of 32, 16 or 8 columns)
constexpr int FFT_THREADS = 256;
constexpr int FFT_MAXPASS = 12;
constexpr int FFT_NMAX = 256;      // n x 8 columns x 16 B <= 32 KB of LDS

struct FftAxis {
  int n;
  int npass;
  int radix[FFT_MAXPASS];
  int ns[FFT_MAXPASS];     // sub-transform length before the pass
  int tw[FFT_MAXPASS];     // offset of the pass twiddles exp(-2 pi i x / (ns R)), x < ns R
  int root[FFT_MAXPASS];   // offset of the radix roots exp(-2 pi i q / R), q < R
};

struct FftPlan {
  FftAxis ax[3];
  int ntw;                 // table entries (double2)
};

static bool factor_axis(int n, FftAxis& a, int& off) {
  a.n = n;
  a.npass = 0;
  int ns = 1, m = n;
  static const int radices[] = {8, 4, 2, 3, 5, 7};
  while (m > 1) {
    int r = 0;
    for (int c : radices)
      if (m % c == 0) {
        r = c;
        break;
      }
    if (r == 0 || a.npass == FFT_MAXPASS) return false;
    a.radix[a.npass] = r;
    a.ns[a.npass] = ns;
    a.tw[a.npass] = off;
    off += ns * r;
    a.root[a.npass] = off;
    off += r;
    ++a.npass;
    ns *= r;
    m /= r;
  }
  return true;
}

static bool make_plan(const isdf_grid* g, FftPlan& p) {
  int off = 0;
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] > FFT_NMAX || !factor_axis(g->n[a], p.ax[a], off)) return false;
  }
  p.ntw = off;
  return true;
}

// Twiddle and root tables of the three axes.
__global__ void fft_tables(FftPlan p, double2* __restrict__ tab) {
  for (int a = 0; a < 3; ++a) {
    const FftAxis& ax = p.ax[a];
    for (int s = 0; s < ax.npass; ++s) {
      const int m = ax.ns[s] * ax.radix[s], R = ax.radix[s];
      for (int x = threadIdx.x; x < m; x += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * x / m, &sn, &cs);
        tab[ax.tw[s] + x] = make_double2(cs, sn);
      }
      for (int q = threadIdx.x; q < R; q += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * q / R, &sn, &cs);
        tab[ax.root[s] + q] = make_double2(cs, sn);
      }
    }
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }  // a * (-i)

__device__ __forceinline__ void dft4(double2& v0, double2& v1, double2& v2, double2& v3) {
  const double2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = mul_mi(csub(v1, v3));
  v0 = cadd(a0, a2);
  v2 = csub(a0, a2);
  v1 = cadd(a1, a3);
  v3 = csub(a1, a3);
}

// Forward DFT of v[0..R), R a compile-time radix (values stay in registers).
template <int R>
__device__ __forceinline__ void dft(double2 (&v)[R], const double2* __restrict__ roots) {
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const double h = 0.70710678118654752440;  // 1 / sqrt(2)
    // o_q *= exp(-2 pi i q / 8)
    o1 = make_double2(h * (o1.x + o1.y), h * (o1.y - o1.x));
    o2 = mul_mi(o2);
    o3 = make_double2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
  } else {
    double2 w[R];
#pragma unroll
    for (int q = 0; q < R; ++q) w[q] = roots[q];
    double2 out[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double2 s = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) s = cadd(s, cmul(v[r], w[(q * r) % R]));
      out[q] = s;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = out[q];
  }
}

// One Stockham pass of radix R over the CT columns of LDS buffer `a`, in
// place: each thread reads its butterflies' inputs into registers, the
// workgroup synchronises, and the outputs go back into `a`.  A thread owns
// at most ceil(8 / R) butterflies (n CT <= 2048 elements over 256 threads).
template <int R, int CT>
__device__ __forceinline__ void stockham_pass(double2* a, int n, int ns, const double2* __restrict__ tw,
                                              const double2* __restrict__ roots) {
  const int c = threadIdx.x % CT, grp = threadIdx.x / CT;
  constexpr int NGRP = FFT_THREADS / CT;
  constexpr int NB = (8 + R - 1) / R;
  const int m = n / R;
  double2 v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = grp + q * NGRP;
    if (j < m) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = a[(j + r * m) * CT + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = grp + q * NGRP;
    if (j < m) {
      const int k = j % ns;
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[k * r]);
      }
      dft<R>(v[q], roots);
      const int d = (j / ns) * ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) a[(d + r * ns) * CT + c] = v[q][r];
    }
  }
  __syncthreads();
}

// Forward FFT, in place, of the CT columns held in LDS buffer `a` (n points
// each, element (x, c) at a[x * CT + c]).
// POW2: every radix is 8, 4 or 2 (a kernel without the register-hungry
// generic radices).
template <int CT, bool POW2>
__device__ void fft_lds(double2* a, const FftAxis& ax, const double2* __restrict__ tab) {
  const int n = ax.n;
  for (int s = 0; s < ax.npass; ++s) {
    const double2* tw = tab + ax.tw[s];
    const double2* roots = tab + ax.root[s];
    const int R = ax.radix[s];
    if (R == 8) stockham_pass<8, CT>(a, n, ax.ns[s], tw, roots);
    else if (R == 4) stockham_pass<4, CT>(a, n, ax.ns[s], tw, roots);
    else if (R == 2) stockham_pass<2, CT>(a, n, ax.ns[s], tw, roots);
    else if constexpr (!POW2) {
      if (R == 3) stockham_pass<3, CT>(a, n, ax.ns[s], tw, roots);
      else if (R == 5) stockham_pass<5, CT>(a, n, ax.ns[s], tw, roots);
      else stockham_pass<7, CT>(a, n, ax.ns[s], tw, roots);
    }
  }
}

// Line geometry: point x of line `line` along axis `axis`.
struct Lines {
  int n0, n1, n2;
  __device__ __forceinline__ int64_t point(int axis, int64_t line, int x) const {
    if (axis == 2) return line * n2 + x;                             // line = i n1 + j
    if (axis == 1) return (line / n2) * (int64_t)n1 * n2 + (int64_t)x * n2 + line % n2;  // line = i n2 + k
    return (int64_t)x * n1 * n2 + line;                              // line = j n2 + k
  }
};

enum { SRC_W = 0, SRC_REAL = 1, SRC_CPLX = 2 };
enum { DST_W = 0, DST_REAL = 1, DST_CPLX = 2 };

// One line pass.  dir: 0 forward, 1 inverse, 2 forward + Poisson kernel +
// inverse (axis 0 only).  Source / destination: the work array W, stored in
// tiles of 32 columns ([ncols / 32][N_r][32] double2, so that a k-line of a
// tile is contiguous), or Theta / V as real pairs or complex of type TS.
template <class TS, int SRC, int DST, int CT, bool POW2>
__global__ __launch_bounds__(FFT_THREADS) void fft_pass(const void* __restrict__ src, int64_t lds, void* __restrict__ dst,
                                                        int64_t ldd, const double2* __restrict__ W_in,
                                                        double2* __restrict__ W_out, int64_t ncols, int n_mu,
                                                        Lines L, int axis, int dir, FftPlan plan,
                                                        const double2* __restrict__ tab, double3 gscale,
                                                        double inv_nr) {
  extern __shared__ double2 lds_buf[];
  const FftAxis& ax = plan.ax[axis];
  const int n = ax.n;
  double2* a = lds_buf;
  const int64_t line = blockIdx.x;
  const int64_t nr = (int64_t)L.n0 * L.n1 * L.n2;
  const int64_t c0 = (int64_t)blockIdx.y * CT;
  const bool conj_in = dir == 1;
  // load: at most 8 elements per thread (n CT <= 2048), all issued before
  // the LDS stores so that they are in flight together
  constexpr int PER = 8;
  const int total = n * CT;
  double2 t[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    t[q] = make_double2(0.0, 0.0);
    if (e < total) {
      const int x = e / CT, c = e % CT;
      const int64_t p = L.point(axis, line, x), col = c0 + c;
      if (SRC == SRC_W) {
        t[q] = W_in[((col >> 5) * nr + p) * 32 + (col & 31)];
      } else if (SRC == SRC_REAL) {
        const TS* row = (const TS*)src + p * lds;
        if (2 * col < n_mu) t[q].x = (double)row[2 * col];
        if (2 * col + 1 < n_mu) t[q].y = (double)row[2 * col + 1];
      } else {
        if (col < n_mu) t[q] = Cplx<TS>::load((const TS*)src + 2 * (p * lds + col));
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    if (e < total) a[e] = conj_in ? make_double2(t[q].x, -t[q].y) : t[q];
  }
  __syncthreads();
  fft_lds<CT, POW2>(a, ax, tab);
  double2* res = a;
  if (dir == 2) {
    // res holds the spectrum along axis 0 (all three axes transformed):
    // multiply by 4 pi / (N_r |G|^2), then conj for the inverse transform
    const int64_t j = line / L.n2, k = line % L.n2;
    const int mj = j < (L.n1 + 1) / 2 ? (int)j : (int)j - L.n1;
    const int mk = k < (L.n2 + 1) / 2 ? (int)k : (int)k - L.n2;
    const double gjk = (mj * gscale.y) * (mj * gscale.y) + (mk * gscale.z) * (mk * gscale.z);
    for (int e = threadIdx.x; e < n * CT; e += FFT_THREADS) {
      const int x = e / CT;
      const int mi = x < (n + 1) / 2 ? x : x - n;
      const double g2 = (mi * gscale.x) * (mi * gscale.x) + gjk;
      const double kv = g2 > 0.0 ? 4.0 * M_PI * inv_nr / g2 : 0.0;
      const double2 v = res[e];
      res[e] = make_double2(kv * v.x, -kv * v.y);
    }
    __syncthreads();
    fft_lds<CT, POW2>(res, ax, tab);
  }
  const bool conj_out = dir >= 1;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    if (e < total) t[q] = res[e];
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * FFT_THREADS;
    if (e >= total) continue;
    const int x = e / CT, c = e % CT;
    const int64_t p = L.point(axis, line, x), col = c0 + c;
    double2 v = t[q];
    if (conj_out) v.y = -v.y;
    if (DST == DST_W) {
      W_out[((col >> 5) * nr + p) * 32 + (col & 31)] = v;
    } else if (DST == DST_REAL) {
      TS* row = (TS*)dst + p * ldd;
      if (2 * col < n_mu) row[2 * col] = (TS)v.x;
      if (2 * col + 1 < n_mu) row[2 * col + 1] = (TS)v.y;
    } else {
      if (col < n_mu) Cplx<TS>::store((TS*)dst + 2 * (p * ldd + col), v.x, v.y);
    }
  }
}

struct PoissonWork {
  double2* tab;
  double2* W;
  int64_t ncols;
  size_t bytes;
};

static PoissonWork plan_poisson(void* ws, size_t cap, int64_t nr, int n_mu, bool cplx, int ntw) {
  Carver c(ws, cap);
  PoissonWork w{};
  const int64_t cols = cplx ? n_mu : ceil_div(n_mu, 2);
  w.ncols = ceil_div(cols, FFT_CT) * FFT_CT;  // a multiple of both column tiles
  w.tab = c.take<double2>(ntw > 0 ? ntw : 1);
  w.W = c.take<double2>((size_t)nr * w.ncols);
  w.bytes = c.used;
  return w;
}

template <class TS>
static int poisson_run(const isdf_grid* g, const TS* theta, int64_t ld_theta, int n_mu, bool cplx, TS* V,
                       int64_t ld_v, const FftPlan& plan, const PoissonWork& w, hipStream_t s) {
  const Lines L{g->n[0], g->n[1], g->n[2]};
  const int64_t nr = (int64_t)L.n0 * L.n1 * L.n2;
  const double3 gs = make_double3(2.0 * M_PI / (L.n0 * g->h[0]), 2.0 * M_PI / (L.n1 * g->h[1]),
                                  2.0 * M_PI / (L.n2 * g->h[2]));
  const double inv_nr = 1.0 / (double)nr;
  hipLaunchKernelGGL(fft_tables, dim3(1), dim3(256), 0, s, plan, w.tab);
  if (!launch_ok()) return ISDF_E_HIP;
  // Columns per workgroup: 32 (512-byte row segments) for n <= 64, else 16
  // (n <= 128), else 8: n x columns <= 2048 elements, 32 KB of LDS.
  bool pow2 = true;
  for (int a = 0; a < 3; ++a)
    for (int q = 0; q < plan.ax[a].npass; ++q) pow2 = pow2 && (plan.ax[a].radix[q] % 2 == 0);
  auto launch = [&](auto src_tag, auto dst_tag, auto ct_tag, auto pow2_tag, int axis, int dir, const void* src,
                    int64_t lds_, void* dst, int64_t ldd) {
    constexpr int S = decltype(src_tag)::value, D = decltype(dst_tag)::value, CTV = decltype(ct_tag)::value;
    constexpr bool P2 = decltype(pow2_tag)::value;
    const int n = plan.ax[axis].n;
    hipLaunchKernelGGL((fft_pass<TS, S, D, CTV, P2>), dim3((unsigned)(nr / n), (unsigned)(w.ncols / CTV)),
                       dim3(FFT_THREADS), (size_t)n * CTV * sizeof(double2), s, src, lds_, dst, ldd,
                       (const double2*)w.W, w.W, w.ncols, n_mu, L, axis, dir, plan, (const double2*)w.tab, gs,
                       inv_nr);
  };
  auto run = [&](auto src_tag, auto dst_tag, int axis, int dir, const void* src, int64_t lds_, void* dst,
                 int64_t ldd) -> bool {
    const int n = plan.ax[axis].n;
    typedef std::integral_constant<int, 32> c32;
    typedef std::integral_constant<int, 16> c16;
    typedef std::integral_constant<int, 8> c8;
    if (pow2) {
      std::true_type p2;
      if (n <= 64) launch(src_tag, dst_tag, c32(), p2, axis, dir, src, lds_, dst, ldd);
      else if (n <= 128) launch(src_tag, dst_tag, c16(), p2, axis, dir, src, lds_, dst, ldd);
      else launch(src_tag, dst_tag, c8(), p2, axis, dir, src, lds_, dst, ldd);
    } else {
      std::false_type p2;
      if (n <= 64) launch(src_tag, dst_tag, c32(), p2, axis, dir, src, lds_, dst, ldd);
      else if (n <= 128) launch(src_tag, dst_tag, c16(), p2, axis, dir, src, lds_, dst, ldd);
      else launch(src_tag, dst_tag, c8(), p2, axis, dir, src, lds_, dst, ldd);
    }
    return launch_ok();
  };
  typedef std::integral_constant<int, SRC_W> sW;
  typedef std::integral_constant<int, DST_W> dW;
  // 1. forward along k, Theta -> W
  bool ok = cplx ? run(std::integral_constant<int, SRC_CPLX>(), dW(), 2, 0, theta, ld_theta, nullptr, 0)
                 : run(std::integral_constant<int, SRC_REAL>(), dW(), 2, 0, theta, ld_theta, nullptr, 0);
  // 2. forward along j; 3. along i with the kernel; 4. inverse along j
  ok = ok && run(sW(), dW(), 1, 0, nullptr, 0, nullptr, 0);
  ok = ok && run(sW(), dW(), 0, 2, nullptr, 0, nullptr, 0);
  ok = ok && run(sW(), dW(), 1, 1, nullptr, 0, nullptr, 0);
  // 5. inverse along k, W -> V
  ok = ok && (cplx ? run(sW(), std::integral_constant<int, DST_CPLX>(), 2, 1, nullptr, 0, V, ld_v)
                   : run(sW(), std::integral_constant<int, DST_REAL>(), 2, 1, nullptr, 0, V, ld_v));
  return ok ? ISDF_OK : ISDF_E_HIP;
}

}  // namespace
}  // namespace isdf

using namespace isdf;

extern "C" size_t isdf_poisson_workspace(const isdf_grid* grid, int32_t n_mu, int32_t is_complex) {
  if (!grid || n_mu <= 0) return 0;
  FftPlan plan{};
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] <= 0) return 0;
  if (!make_plan(grid, plan)) return 0;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  return plan_poisson(nullptr, 0, nr, n_mu, is_complex != 0, plan.ntw).bytes;
}

extern "C" int isdf_poisson(const isdf_grid* grid, int32_t dt_in, const void* theta, int64_t ld_theta, int32_t n_mu,
                            int32_t is_complex, void* V, int64_t ld_v, void* ws, size_t ws_bytes, void* stream) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  if (!grid || !theta || !V || n_mu <= 0 || ld_theta < n_mu || ld_v < n_mu) return ISDF_E_ARG;
  if (dt != ISDF_C128 && dt != ISDF_C64) return ISDF_E_ARG;
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] <= 0 || !(grid->h[a] > 0.0)) return ISDF_E_ARG;
  FftPlan plan{};
  if (!make_plan(grid, plan)) return ISDF_E_UNSUPPORTED;  // an axis > 256 or with a prime factor > 7
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  const int64_t lines_max = nr / 1;
  if (lines_max > INT32_MAX) return ISDF_E_ARG;
  const bool cplx = is_complex != 0;
  PoissonWork w = plan_poisson(ws, ws_bytes, nr, n_mu, cplx, plan.ntw);
  if (!ws || w.bytes > ws_bytes) return ISDF_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (dt == ISDF_C128)
    return poisson_run<double>(grid, (const double*)theta, ld_theta, n_mu, cplx, (double*)V, ld_v, plan, w, s);
  return poisson_run<float>(grid, (const float*)theta, ld_theta, n_mu, cplx, (float*)V, ld_v, plan, w, s);
}
