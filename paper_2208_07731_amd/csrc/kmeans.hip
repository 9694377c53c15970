// Weighted K-means over grid points (Sec. 2.2 and Alg. 1 of arXiv:2208.07731)
// and the K-means weight functions (eqs. weight function, weight function 2).
//
// Kernels, in launch order:
//   km_weight  one HBM pass over the orbital rows -> w[N_r] (FP64)
//   km_init    seeds, counters and per-cluster bounding boxes
//   km_assign  classification, one 4x4x4 brick of grid points per wavefront:
//              first round, argmin over every centroid staged through LDS;
//              later rounds, over the centroids of the cells near the brick
//              (km_bin); also the objective partials, tie counts,
//              changed-label count, evaluated-pair counts and per-cluster
//              bounding boxes (integer atomics, order independent)
//   km_update  weighted centroids: one wavefront per cluster scans its
//              bounding box in a fixed order -> deterministic FP64 sums
//   km_bin     the updated centroids sorted into a coarse grid of cells
//   km_snap    member nearest to each final centroid (lowest index on ties)
//   km_final   info struct
// A round that changes no label sets a device flag that turns the remaining
// launches into no-ops, so the host enqueues a fixed sequence and never
// synchronises.
#include <float.h>
#include <limits.h>

#include <mutex>

#include "common.h"

namespace isdf {

struct KmState {
  int done;        // remaining rounds are no-ops
  int converged;
  int iters;       // updates applied
  int last_t;      // last classification that ran
  int nonfinite;
  int empty_final;
  int pad0, pad1;
};

struct KmArrays {
  KmState* st;
  int* changed;    // [T+1]
  int* ties;       // [T+1]
  int* nearc;      // [T+1]
  int* empty;      // [T+1]
  double* jhist;   // [T+1]
  double* cent;    // [K][3]
  int* labels;     // [N_r]
  double* w;       // [N_r]
  int* bbox;       // [K][6]: imin, imax, jmin, jmax, kmin, kmax
  double* jpart;   // [assign blocks]
  int* cell_start;  // [cells + 1]: centroids of cell q at cell_c[cell_start[q] .. cell_start[q + 1])
  double4* cell_c;  // [K]: (x, y, z, index) of the centroids, by cell
  unsigned long long* pairs;  // [assign blocks] point-centroid distances evaluated, over all classifications
  unsigned long long* tests;  // [assign blocks] brick-centroid bound tests, over all classifications
};

struct KmGeom {
  int n0, n1, n2;
  int nb0, nb1, nb2;  // bricks per axis (4 points each)
  double s0, s1, s2;  // metric weights (h_a / min h)^2
  int aniso;
  int cell;           // edge of a centroid cell in grid points
  int nc0, nc1, nc2;  // cells per axis
};

constexpr int ASSIGN_THREADS = 512;  // 8 wavefronts = 8 bricks
constexpr int CTILE = 2048;          // centroids staged per LDS tile
constexpr int MAX_CELLS = 8192;      // centroid cells (counted in LDS by km_bin)
constexpr int BIN_THREADS = 1024;

// Squared distance with the same operation order as the definition
// ((s0 dx^2 + s1 dy^2) + s2 dz^2); contraction off so that the value is the
// correctly rounded result of each operation.
__device__ __forceinline__ double sqd(double dx, double dy, double dz, const KmGeom& g) {
#pragma clang fp contract(off)
  if (g.aniso) return (g.s0 * (dx * dx) + g.s1 * (dy * dy)) + g.s2 * (dz * dz);
  return (dx * dx + dy * dy) + dz * dz;
}

// ------------------------------------------------------------------ weight
template <class T>
__device__ __forceinline__ double row_pow_sum(const T* __restrict__ row, int n, int sub, int sw,
                                              int alpha) {
  double acc = 0.0;
  for (int i = sub; i < n; i += sw) {
    double2 z = Cplx<T>::load(row + 2 * (int64_t)i);
    double s = z.x * z.x + z.y * z.y;
    double v;
    if (alpha == 2) v = s;
    else if (alpha == 1) v = sqrt(s);
    else if (alpha == 3) v = s * sqrt(s);
    else v = s * s;
    acc += v;
  }
  return acc;
}

// Segmented sum over `sw` consecutive lanes (sw a power of two <= 64).
__device__ __forceinline__ double seg_sum(double v, int sw) {
  for (int o = sw >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, ISDF_WAVE);
  return v;
}

// Sub-wave of width sw per row; alpha = 2 for SSM/PSM.
template <class T>
__global__ __launch_bounds__(256) void km_weight(const T* __restrict__ phi, int64_t ldp, int nphi,
                                                 const T* __restrict__ psi, int64_t lds, int npsi,
                                                 int aliased, int kind, int sw, int64_t nr,
                                                 double* __restrict__ w, KmState* st) {
  const int lane = threadIdx.x & 63;
  const int sub = lane & (sw - 1);
  const int rows_per_wave = ISDF_WAVE / sw;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int alpha = kind == ISDF_W_SM ? 1 : kind == ISDF_W_SCM ? 3 : kind == ISDF_W_SQM ? 4 : 2;
  int bad = 0;
  for (int64_t r0 = wave * rows_per_wave; r0 < nr; r0 += nwaves * rows_per_wave) {
    int64_t r = r0 + lane / sw;
    double a = 0.0, b = 0.0;
    if (r < nr) {
      a = row_pow_sum<T>(phi + 2 * r * ldp, nphi, sub, sw, alpha);
      if (!aliased) b = row_pow_sum<T>(psi + 2 * r * lds, npsi, sub, sw, alpha);
    }
    a = seg_sum(a, sw);
    if (!aliased) b = seg_sum(b, sw);
    if (aliased) b = a;
    double v = kind == ISDF_W_PSM ? a * b : a + b;
    if (r < nr && sub == 0) {
      w[r] = v;
      if (!isfinite(v)) bad = 1;
    }
  }
  if (bad) atomicOr(&st->nonfinite, 1);
}

// Checks a caller-given weight for NaN / Inf / negative values.
__global__ void km_check_weight(const double* __restrict__ w, int64_t nr, KmState* st) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nr;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = w[i];
    if (!isfinite(v) || v < 0.0) bad = 1;
  }
  if (bad) atomicOr(&st->nonfinite, 1);
}

// ------------------------------------------------------------------ init
__global__ void km_init(KmArrays a, const double* __restrict__ c0, int K, int T, int64_t nr, int nparts) {
  int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) {
    int nf = a.st->nonfinite;  // written by the weight pass before this launch
    a.st->done = nf ? 1 : 0;
    a.st->converged = 0;
    a.st->iters = 0;
    a.st->last_t = -1;
    a.st->empty_final = 0;
  }
  for (int64_t i = tid; i <= T; i += stride) {
    a.changed[i] = 0;
    a.ties[i] = 0;
    a.nearc[i] = 0;
    a.empty[i] = 0;
    a.jhist[i] = -1.0;
  }
  for (int64_t i = tid; i < nparts; i += stride) {
    a.pairs[i] = 0;
    a.tests[i] = 0;
  }
  for (int64_t i = tid; i < 3 * (int64_t)K; i += stride) a.cent[i] = c0[i];
  for (int64_t i = tid; i < K; i += stride) {
    int* b = a.bbox + 6 * i;
    b[0] = INT_MAX; b[1] = INT_MIN; b[2] = INT_MAX; b[3] = INT_MIN; b[4] = INT_MAX; b[5] = INT_MIN;
  }
  for (int64_t i = tid; i < nr; i += stride) a.labels[i] = -1;
}

// ------------------------------------------------------------------ assign
// Exact per-brick candidate pruning.  For the brick's bounding box B and a
// centroid c: lb(c) = min_{p in B} D(p, c), ub(c) = max_{p in B} D(p, c).
// U is an upper bound of every brick point's nearest distance d1(p):
//  * first round: U = min_c ub(c), since d1(p) <= D(p, c) <= ub(c) for any c;
//  * later rounds: U = max_{p in B} D(p, c(old(p))), the distance of each
//    point to the centroid of the cluster it was given in the previous round,
//    evaluated with the centroids as they are now (just updated); that is a
//    distance to one of the current centroids, so d1(p) <= D(p, c(old(p))) <= U
//    however far that centroid moved.
// A centroid with lb(c) > U is then strictly farther than some centroid for
// every point of the brick and can be skipped.  The test uses U (1 + margin)
// with margin well above rounding and above the near-tie band, so labels,
// exact ties and near-tie counts are those of the full scan.  Survivors are
// evaluated in increasing centroid order (lowest index wins ties).
constexpr int SURV = 128;  // per-wavefront survivor list
static_assert(SURV <= CTILE / (ASSIGN_THREADS / ISDF_WAVE), "survivor coordinates fit a wave's tile slice");

__device__ __forceinline__ double axis_lb(double c, double lo, double hi) {
  const double d = fmax(fmax(lo - c, c - hi), 0.0);
  return d * d;
}
__device__ __forceinline__ double axis_ub(double c, double lo, double hi) {
  const double d = fmax(fabs(c - lo), fabs(c - hi));
  return d * d;
}

__global__ __launch_bounds__(ASSIGN_THREADS) void km_assign(KmArrays a, KmGeom g, int K, int t,
                                                            double near_rel) {
  if (a.st->done) return;
  __shared__ double cx[CTILE], cy[CTILE], cz[CTILE];
  __shared__ double jw[ASSIGN_THREADS / ISDF_WAVE];
  __shared__ int surv[ASSIGN_THREADS / ISDF_WAVE][SURV];
  __shared__ int cellst[ASSIGN_THREADS / ISDF_WAVE][ISDF_WAVE], celloff[ASSIGN_THREADS / ISDF_WAVE][ISDF_WAVE];
  __shared__ unsigned long long wpairs[ASSIGN_THREADS / ISDF_WAVE], wtests[ASSIGN_THREADS / ISDF_WAVE];
  __shared__ int wcount[ASSIGN_THREADS / ISDF_WAVE][3];

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t brick = (int64_t)blockIdx.x * (ASSIGN_THREADS / ISDF_WAVE) + wv;
  const int64_t nbricks = (int64_t)g.nb0 * g.nb1 * g.nb2;
  int bi = 0, bj = 0, bk = 0;
  if (brick < nbricks) {
    bk = (int)(brick % g.nb2);
    int64_t q = brick / g.nb2;
    bj = (int)(q % g.nb1);
    bi = (int)(q / g.nb1);
  }
  const int pi = bi * 4 + (lane >> 4), pj = bj * 4 + ((lane >> 2) & 3), pk = bk * 4 + (lane & 3);
  const bool valid = brick < nbricks && pi < g.n0 && pj < g.n1 && pk < g.n2;
  const double px = (double)pi, py = (double)pj, pz = (double)pk;
  // bounding box of the brick's grid points
  const double lo0 = bi * 4, lo1 = bj * 4, lo2 = bk * 4;
  const double hi0 = min(bi * 4 + 3, g.n0 - 1), hi1 = min(bj * 4 + 3, g.n1 - 1), hi2 = min(bk * 4 + 3, g.n2 - 1);
  const double margin = 1.0 + fmax(1e-5, 4.0 * near_rel);
  int* list = surv[wv];

  double d1 = INFINITY, d2 = INFINITY;
  int lab = 0;
  const int64_t p = ((int64_t)pi * g.n1 + pj) * g.n2 + pk;
  unsigned long long n_eval = 0, n_test = 0;  // survivors evaluated, bound tests (wave-uniform)
  if (t > 0) {
    // U: the largest distance of a brick point to the centroid of the
    // cluster it was given in the previous round, with the centroids as
    // they are now (just updated): a distance to a current centroid, so it
    // bounds every brick point's nearest distance
    double own = -INFINITY;
    if (valid) {
      const int old = a.labels[p];
      own = sqd(px - a.cent[3 * (int64_t)old], py - a.cent[3 * (int64_t)old + 1],
                pz - a.cent[3 * (int64_t)old + 2], g);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) own = fmax(own, __shfl_xor(own, o, ISDF_WAVE));
    const double cut = own * margin;
    // a centroid with lb <= cut lies within sqrt(cut / s_a) of the brick on
    // every axis a, so only the cells of that box can hold one
    int c_lo[3], c_hi[3];
    const double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2}, sa[3] = {g.s0, g.s1, g.s2};
    const int nca[3] = {g.nc0, g.nc1, g.nc2};
    int nbox = 1;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double r = cut > 0.0 ? sqrt(cut / sa[ax]) * (1.0 + 1e-12) + 1e-9 : 0.0;
      c_lo[ax] = max(0, (int)floor((lo[ax] - r) / g.cell));
      c_hi[ax] = min(nca[ax] - 1, (int)floor((hi[ax] + r) / g.cell));
      if (!(cut >= 0.0) || c_hi[ax] < c_lo[ax]) nbox = 0;  // no valid point in the brick
      else nbox *= c_hi[ax] - c_lo[ax] + 1;
    }
    const int e1 = c_hi[1] - c_lo[1] + 1, e2 = c_hi[2] - c_lo[2] + 1;
    int* cst = cellst[wv];
    int* cof = celloff[wv];
    // survivors' coordinates: this wave's slice of the first round's tile arrays
    double* sx = cx + wv * (CTILE / (ASSIGN_THREADS / ISDF_WAVE));
    double* sy = cy + wv * (CTILE / (ASSIGN_THREADS / ISDF_WAVE));
    double* sz = cz + wv * (CTILE / (ASSIGN_THREADS / ISDF_WAVE));
    int nlist = 0;
    for (int b0 = 0; b0 < nbox; b0 += ISDF_WAVE) {
      // one cell of the box per lane: its first entry and its count
      const int q = b0 + lane;
      int cs = 0, cn = 0;
      if (q < nbox) {
        const int qk = q % e2, qj = (q / e2) % e1, qi = q / (e1 * e2);
        const int cell = ((c_lo[0] + qi) * g.nc1 + (c_lo[1] + qj)) * g.nc2 + (c_lo[2] + qk);
        cs = a.cell_start[cell];
        cn = a.cell_start[cell + 1] - cs;
      }
      int incl = cn;  // inclusive prefix sum over the lanes
#pragma unroll
      for (int o = 1; o < ISDF_WAVE; o <<= 1) {
        const int v = __shfl_up(incl, o, ISDF_WAVE);
        if (lane >= o) incl += v;
      }
      const int total = __shfl(incl, ISDF_WAVE - 1, ISDF_WAVE);
      const int ncell = min(ISDF_WAVE, nbox - b0);
      cst[lane] = cs;
      cof[lane] = incl - cn;
      __builtin_amdgcn_wave_barrier();
      for (int c0 = 0; c0 < total; c0 += ISDF_WAVE) {
        const int qq = c0 + lane;
        bool keep = false;
        double4 cand = make_double4(0.0, 0.0, 0.0, 0.0);
        if (qq < total) {
          int lo_i = 0, hi_i = ncell - 1;  // last cell lane whose offset <= qq
          while (lo_i < hi_i) {
            const int mid = (lo_i + hi_i + 1) >> 1;
            if (cof[mid] <= qq) lo_i = mid;
            else hi_i = mid - 1;
          }
          cand = a.cell_c[cst[lo_i] + (qq - cof[lo_i])];
          const double lb = (g.s0 * axis_lb(cand.x, lo0, hi0) + g.s1 * axis_lb(cand.y, lo1, hi1)) +
                            g.s2 * axis_lb(cand.z, lo2, hi2);
          keep = lb <= cut;
        }
        n_test += (unsigned long long)min(ISDF_WAVE, total - c0);
        const unsigned long long bal = __ballot(keep);
        const int cnt = __popcll(bal);
        if (nlist + cnt > SURV) {  // evaluate the list (wave-uniform)
          for (int e = 0; e < nlist; ++e) {
            const int m = list[e];
            const double d = sqd(px - sx[e], py - sy[e], pz - sz[e], g);
            if (d < d1 || (d == d1 && m < lab)) {
              d2 = d1;
              d1 = d;
              lab = m;
            } else {
              d2 = fmin(d2, d);
            }
          }
          n_eval += (unsigned long long)nlist;
          nlist = 0;
          __builtin_amdgcn_wave_barrier();
        }
        if (keep) {  // survivor: its index and coordinates into this wave's list
          const int at = nlist + __popcll(bal & ((1ull << lane) - 1ull));
          list[at] = (int)cand.w;
          sx[at] = cand.x;
          sy[at] = cand.y;
          sz[at] = cand.z;
        }
        nlist += cnt;
        __builtin_amdgcn_wave_barrier();
      }
      __builtin_amdgcn_wave_barrier();
    }
    for (int e = 0; e < nlist; ++e) {
      const int m = list[e];
      const double d = sqd(px - sx[e], py - sy[e], pz - sz[e], g);
      if (d < d1 || (d == d1 && m < lab)) {
        d2 = d1;
        d1 = d;
        lab = m;
      } else {
        d2 = fmin(d2, d);
      }
    }
    n_eval += (unsigned long long)nlist;
  } else {
    // first round: U = the smallest over centroids of the farthest brick
    // distance, then every centroid tile's survivors in increasing index
    double U = INFINITY;
    for (int c0 = 0; c0 < K; c0 += CTILE) {
      const int cn = min(CTILE, K - c0);
      __syncthreads();
      for (int i = threadIdx.x; i < cn; i += ASSIGN_THREADS) {
        cx[i] = a.cent[3 * (int64_t)(c0 + i) + 0];
        cy[i] = a.cent[3 * (int64_t)(c0 + i) + 1];
        cz[i] = a.cent[3 * (int64_t)(c0 + i) + 2];
      }
      __syncthreads();
      for (int m = lane; m < cn; m += ISDF_WAVE) {
        const double ub = (g.s0 * axis_ub(cx[m], lo0, hi0) + g.s1 * axis_ub(cy[m], lo1, hi1)) +
                          g.s2 * axis_ub(cz[m], lo2, hi2);
        U = fmin(U, ub);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) U = fmin(U, __shfl_xor(U, o, ISDF_WAVE));
    const double cut = U * margin;
    const bool one_tile = K <= CTILE;  // the tile is still in LDS
    for (int c0 = 0; c0 < K; c0 += CTILE) {
      const int cn = min(CTILE, K - c0);
      if (!one_tile) {
        __syncthreads();
        for (int i = threadIdx.x; i < cn; i += ASSIGN_THREADS) {
          cx[i] = a.cent[3 * (int64_t)(c0 + i) + 0];
          cy[i] = a.cent[3 * (int64_t)(c0 + i) + 1];
          cz[i] = a.cent[3 * (int64_t)(c0 + i) + 2];
        }
        __syncthreads();
      }
      int nlist = 0;
      n_test += (unsigned long long)cn;
      for (int mb = 0; mb < cn; mb += ISDF_WAVE) {
        const int m = mb + lane;
        bool keep = false;
        if (m < cn) {
          const double lb = (g.s0 * axis_lb(cx[m], lo0, hi0) + g.s1 * axis_lb(cy[m], lo1, hi1)) +
                            g.s2 * axis_lb(cz[m], lo2, hi2);
          keep = lb <= cut;
        }
        const unsigned long long bal = __ballot(keep);
        const int cnt = __popcll(bal);
        if (nlist + cnt > SURV) {  // flush the list (wave-uniform)
          for (int q = 0; q < nlist; ++q) {
            const int mm = list[q];
            const double d = sqd(px - cx[mm], py - cy[mm], pz - cz[mm], g);
            d2 = fmin(d2, fmax(d, d1));
            const bool better = d < d1;
            d1 = better ? d : d1;
            lab = better ? c0 + mm : lab;
          }
          n_eval += (unsigned long long)nlist;
          nlist = 0;
        }
        if (keep) list[nlist + __popcll(bal & ((1ull << lane) - 1ull))] = m;
        nlist += cnt;
      }
      for (int q = 0; q < nlist; ++q) {
        const int mm = list[q];
        const double d = sqd(px - cx[mm], py - cy[mm], pz - cz[mm], g);
        d2 = fmin(d2, fmax(d, d1));
        const bool better = d < d1;
        d1 = better ? d : d1;
        lab = better ? c0 + mm : lab;
      }
      n_eval += (unsigned long long)nlist;
    }
  }
  {  // this wave's counts, summed per workgroup below (no atomics on shared counters)
    const int nvalid = __popcll(__ballot(valid));
    if (lane == 0) {
      wpairs[wv] = nvalid > 0 ? n_eval * (unsigned long long)nvalid : 0ull;
      wtests[wv] = nvalid > 0 ? n_test : 0ull;
    }
  }

  double jv = 0.0;
  bool chg = false, tie = false, nr_tie = false;
  if (valid) {
    int old = a.labels[p];
    chg = old != lab;
    a.labels[p] = lab;
    jv = a.w[p] * d1;
    tie = d1 == d2;
    nr_tie = (d2 < INFINITY) && (d2 - d1 <= near_rel * d2);
  }
  // objective partial: fixed-order block sum
  jv = wave_sum(jv);
  if (lane == 0) jw[wv] = jv;
  unsigned long long bc = __ballot(chg), bt = __ballot(tie), bn = __ballot(nr_tie);
  if (lane == 0) {  // summed per workgroup below: one atomic per workgroup and counter
    wcount[wv][0] = __popcll(bc);
    wcount[wv][1] = __popcll(bt);
    wcount[wv][2] = __popcll(bn);
  }
  // per-cluster bounding boxes: one atomic set per distinct label in the
  // brick.  Lane l holds brick point (l / 16, (l / 4) % 4, l % 4), so the
  // extent of a label's points on each axis follows from its lane mask with
  // scalar bit operations.
  unsigned long long act = __ballot(valid);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int L = __shfl(lab, leader, ISDF_WAVE);
    const unsigned long long mm = __ballot(valid && lab == L);
    if (lane == leader) {
      int i_lo = 4, i_hi = -1, j_lo = 4, j_hi = -1, k_lo = 4, k_hi = -1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if ((mm >> (16 * q)) & 0xFFFFull) {
          i_lo = min(i_lo, q);
          i_hi = max(i_hi, q);
        }
        if (mm & (0x000F000F000F000Full << (4 * q))) {
          j_lo = min(j_lo, q);
          j_hi = max(j_hi, q);
        }
        if (mm & (0x1111111111111111ull << q)) {
          k_lo = min(k_lo, q);
          k_hi = max(k_hi, q);
        }
      }
      int* b = a.bbox + 6 * (int64_t)L;
      atomicMin(b + 0, bi * 4 + i_lo); atomicMax(b + 1, bi * 4 + i_hi);
      atomicMin(b + 2, bj * 4 + j_lo); atomicMax(b + 3, bj * 4 + j_hi);
      atomicMin(b + 4, bk * 4 + k_lo); atomicMax(b + 5, bk * 4 + k_hi);
    }
    act &= ~mm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    unsigned long long np = 0, nt = 0;
    int nc = 0, ntie = 0, nnear = 0;
    for (int i = 0; i < ASSIGN_THREADS / ISDF_WAVE; ++i) {
      s += jw[i];
      np += wpairs[i];
      nt += wtests[i];
      nc += wcount[i][0];
      ntie += wcount[i][1];
      nnear += wcount[i][2];
    }
    if (nc) atomicAdd(&a.changed[t], nc);
    if (ntie) atomicAdd(&a.ties[t], ntie);
    if (nnear) atomicAdd(&a.nearc[t], nnear);
    a.jpart[blockIdx.x] = s;
    a.pairs[blockIdx.x] += np;  // running totals over the classifications, one slot per workgroup
    a.tests[blockIdx.x] += nt;
    if (blockIdx.x == 0) a.st->last_t = t;
  }
}

// Fixed-order sum of the objective partials by one wavefront.
__device__ double reduce_jpart(const double* __restrict__ jp, int n, int lane) {
  double s = 0.0;
  for (int i = lane; i < n; i += ISDF_WAVE) s += jp[i];
  return wave_sum(s);
}

// Walks the bounding box of cluster `mu` line by line (lines along the last
// axis); each lane visits a fixed subset of the box's grid points in a fixed
// order.  The points are taken SCAN_U at a time: load(p) for all of them
// first (independent loads, in flight together), then use(v, p, i, j, k) in
// the walk's order, so sums keep the order of a plain one-by-one walk.
constexpr int SCAN_U = 4;
template <class L, class F>
__device__ __forceinline__ void scan_bbox(const int* b, const KmGeom& g, int lane, L&& load, F&& use) {
  const int i0 = b[0], i1 = b[1], j0 = b[2], j1 = b[3], k0 = b[4], k1 = b[5];
  if (i0 > i1) return;
  const int ej = j1 - j0 + 1, ek = k1 - k0 + 1;
  const int64_t nlines = (int64_t)(i1 - i0 + 1) * ej;
  // this lane's n-th point: line q0 + n dq, offset kk + n dk within it
  int64_t q0, dq;
  int kk, dk, kspan;
  if (ek <= ISDF_WAVE) {
    const int lpp = ISDF_WAVE / ek;  // lines per pass
    const int lo = lane / ek;
    if (lo >= lpp) return;
    q0 = lo;
    dq = lpp;
    kk = lane - lo * ek;
    dk = 0;
    kspan = 1;
  } else {
    if (lane >= ek) return;
    q0 = 0;
    dq = 1;
    kk = lane;
    dk = ISDF_WAVE;
    kspan = (ek - lane + ISDF_WAVE - 1) / ISDF_WAVE;  // points of this lane per line
  }
  const int64_t total = ((nlines - q0 + dq - 1) / dq) * kspan;
  for (int64_t n0 = 0; n0 < total; n0 += SCAN_U) {
    int64_t pp[SCAN_U];
    int ii[SCAN_U], jj[SCAN_U], kq[SCAN_U];
    decltype(load((int64_t)0)) v[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      const int64_t n = n0 + u < total ? n0 + u : total - 1;  // past the end: repeat the last point
      const int64_t q = q0 + (n / kspan) * dq;
      ii[u] = i0 + (int)(q / ej);
      jj[u] = j0 + (int)(q % ej);
      kq[u] = k0 + kk + (int)(n % kspan) * dk;
      pp[u] = ((int64_t)ii[u] * g.n1 + jj[u]) * g.n2 + kq[u];
      v[u] = load(pp[u]);
    }
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u)
      if (n0 + u < total) use(v[u], pp[u], ii[u], jj[u], kq[u]);
  }
}

// ------------------------------------------------------------------ update
__global__ __launch_bounds__(256) void km_update(KmArrays a, KmGeom g, int K, int t, int nparts) {
  if (a.st->done) return;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  if (blockIdx.x == 0 && wv == 0) {
    double J = reduce_jpart(a.jpart, nparts, lane);
    if (lane == 0) a.jhist[t] = J;
  }
  if (t > 0 && a.changed[t] == 0) {  // fixed point: same labels as the previous round
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.st->done = 1;
      a.st->converged = 1;
    }
    return;
  }
  const int mu = blockIdx.x * 4 + wv;
  if (mu >= K) return;
  int* b = a.bbox + 6 * (int64_t)mu;
  double sw = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
  struct LabW {
    int lab;
    double w;
  };
  scan_bbox(
      b, g, lane, [&](int64_t p) { return LabW{a.labels[p], a.w[p]}; },
      [&](LabW v, int64_t, int i, int j, int k) {
        if (v.lab == mu) {
          const double wp = v.w;
          sw += wp;
          sx += wp * (double)i;
          sy += wp * (double)j;
          sz += wp * (double)k;
        }
      });
  sw = wave_sum(sw);
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  if (lane == 0) {
    if (sw > 0.0) {
      a.cent[3 * (int64_t)mu + 0] = sx / sw;
      a.cent[3 * (int64_t)mu + 1] = sy / sw;
      a.cent[3 * (int64_t)mu + 2] = sz / sw;
    } else {
      atomicAdd(&a.empty[t], 1);
    }
    b[0] = INT_MAX; b[1] = INT_MIN; b[2] = INT_MAX; b[3] = INT_MIN; b[4] = INT_MAX; b[5] = INT_MIN;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.st->iters = t + 1;
}

// ------------------------------------------------------------------ bin
// Sorts the centroids into cells of g.cell^3 grid points (one workgroup):
// counts per cell, an exclusive scan into cell_start, then each centroid's
// (x, y, z, index) at its cell's next free slot.  The order inside a cell
// is unspecified; the classification does not depend on it (it keeps the
// lowest index among equal distances explicitly).
__device__ __forceinline__ int cell_of(double x, double y, double z, const KmGeom& g) {
  const int i = min(g.nc0 - 1, max(0, (int)floor(x / g.cell)));
  const int j = min(g.nc1 - 1, max(0, (int)floor(y / g.cell)));
  const int k = min(g.nc2 - 1, max(0, (int)floor(z / g.cell)));
  return (i * g.nc1 + j) * g.nc2 + k;
}

__global__ __launch_bounds__(BIN_THREADS) void km_bin(KmArrays a, KmGeom g, int K) {
  if (a.st->done) return;
  __shared__ int cnt[MAX_CELLS];
  __shared__ int part[BIN_THREADS];
  const int ncells = g.nc0 * g.nc1 * g.nc2;
  const int tid = threadIdx.x;
  for (int i = tid; i < ncells; i += BIN_THREADS) cnt[i] = 0;
  __syncthreads();
  for (int m = tid; m < K; m += BIN_THREADS) {
    const double* c = a.cent + 3 * (int64_t)m;
    atomicAdd(&cnt[cell_of(c[0], c[1], c[2], g)], 1);
  }
  __syncthreads();
  // exclusive scan: each thread its run of `per` cells, then the run totals
  const int per = (ncells + BIN_THREADS - 1) / BIN_THREADS;
  const int b = tid * per, e = min(ncells, b + per);
  int run = 0;
  for (int i = b; i < e; ++i) run += cnt[i];
  part[tid] = run;
  __syncthreads();
  for (int o = 1; o < BIN_THREADS; o <<= 1) {
    const int v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int off = part[tid] - run;
  for (int i = b; i < e; ++i) {
    const int c = cnt[i];
    cnt[i] = off;  // becomes the fill cursor
    a.cell_start[i] = off;
    off += c;
  }
  if (tid == 0) a.cell_start[ncells] = K;
  __syncthreads();
  for (int m = tid; m < K; m += BIN_THREADS) {
    const double* c = a.cent + 3 * (int64_t)m;
    const int pos = atomicAdd(&cnt[cell_of(c[0], c[1], c[2], g)], 1);
    a.cell_c[pos] = make_double4(c[0], c[1], c[2], (double)m);
  }
}

// ------------------------------------------------------------------ snap
__global__ __launch_bounds__(256) void km_snap(KmArrays a, KmGeom g, int K, int32_t* __restrict__ idx) {
  const int lane = threadIdx.x & 63;
  const int mu = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (mu >= K) return;
  if (a.st->nonfinite) {
    if (lane == 0) idx[mu] = -1;
    return;
  }
  const double cxm = a.cent[3 * (int64_t)mu], cym = a.cent[3 * (int64_t)mu + 1],
               czm = a.cent[3 * (int64_t)mu + 2];
  double bd = INFINITY;
  int64_t bp = -1;
  scan_bbox(
      a.bbox + 6 * (int64_t)mu, g, lane, [&](int64_t p) { return a.labels[p]; },
      [&](int lab, int64_t p, int i, int j, int k) {
        if (lab == mu) {
          double d = sqd((double)i - cxm, (double)j - cym, (double)k - czm, g);
          if (d < bd || (d == bd && p < bp)) {
            bd = d;
            bp = p;
          }
        }
      });
  for (int o = 32; o > 0; o >>= 1) {
    double od = __shfl_xor(bd, o, ISDF_WAVE);
    int64_t op = __shfl_xor(bp, o, ISDF_WAVE);
    bool take = (op >= 0) && (bp < 0 || od < bd || (od == bd && op < bp));
    bd = take ? od : bd;
    bp = take ? op : bp;
  }
  if (lane == 0) {
    idx[mu] = (int32_t)bp;
    if (bp < 0) atomicAdd(&a.st->empty_final, 1);
  }
}

__global__ void km_final(KmArrays a, int nparts, isdf_kmeans_info* info, double* __restrict__ objective,
                         int T) {
  const int lane = threadIdx.x;
  KmState* st = a.st;
  int t = st->last_t;
  double J = reduce_jpart(a.jpart, nparts, lane);
  if (t >= 0 && lane == 0) a.jhist[t] = J;
  if (objective)
    for (int i = lane; i <= T; i += ISDF_WAVE) objective[i] = (i == t) ? J : a.jhist[i];
  unsigned long long np = 0, nt = 0;  // integer sums: exact in any order
  for (int i = lane; i < nparts; i += ISDF_WAVE) {
    np += a.pairs[i];
    nt += a.tests[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    np += __shfl_xor(np, o, ISDF_WAVE);
    nt += __shfl_xor(nt, o, ISDF_WAVE);
  }
  if (lane != 0) return;
  int status = ISDF_OK;
  if (st->nonfinite) status = ISDF_E_NONFINITE;
  else if (st->empty_final) status = ISDF_W_EMPTY_CLUSTER;
  info->status = status;
  info->iters = st->iters;
  info->converged = st->converged;
  info->empty_update = st->iters > 0 ? a.empty[st->iters - 1] : 0;
  info->empty_final = st->empty_final;
  info->ties = t >= 0 ? a.ties[t] : 0;
  info->near_ties = t >= 0 ? a.nearc[t] : 0;
  info->changed = t >= 0 ? a.changed[t] : 0;
  info->objective = t >= 0 ? J : 0.0;
  info->pairs_evaluated = (int64_t)np;
  info->bound_tests = (int64_t)nt;
}

__global__ void copy_f64(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ------------------------------------------------------------------ host
struct KmPlan {
  KmArrays a;
  size_t bytes;
};

static KmPlan plan_kmeans(void* ws, size_t cap, int64_t nr, int K, int T, int nparts,
                          bool own_cent, bool own_labels, bool own_w, bool own_obj) {
  Carver c(ws, cap);
  KmPlan P{};
  P.a.st = c.take<KmState>(1);
  P.a.changed = c.take<int>(T + 1);
  P.a.ties = c.take<int>(T + 1);
  P.a.nearc = c.take<int>(T + 1);
  P.a.empty = c.take<int>(T + 1);
  P.a.jhist = c.take<double>(T + 1);
  P.a.bbox = c.take<int>(6 * (size_t)K);
  P.a.jpart = c.take<double>(nparts);
  P.a.pairs = c.take<unsigned long long>(nparts);
  P.a.tests = c.take<unsigned long long>(nparts);
  P.a.cell_start = c.take<int>(MAX_CELLS + 1);
  P.a.cell_c = c.take<double4>(K);
  if (own_cent) P.a.cent = c.take<double>(3 * (size_t)K);
  if (own_labels) P.a.labels = c.take<int>(nr);
  if (own_w) P.a.w = c.take<double>(nr);
  (void)own_obj;
  P.bytes = c.used;
  return P;
}

static KmGeom make_geom(const isdf_grid* g) {
  KmGeom G{};
  G.n0 = g->n[0];
  G.n1 = g->n[1];
  G.n2 = g->n[2];
  G.nb0 = (G.n0 + 3) / 4;
  G.nb1 = (G.n1 + 3) / 4;
  G.nb2 = (G.n2 + 3) / 4;
  double hmin = fmin(g->h[0], fmin(g->h[1], g->h[2]));
  G.s0 = (g->h[0] / hmin) * (g->h[0] / hmin);
  G.s1 = (g->h[1] / hmin) * (g->h[1] / hmin);
  G.s2 = (g->h[2] / hmin) * (g->h[2] / hmin);
  G.aniso = !(G.s0 == 1.0 && G.s1 == 1.0 && G.s2 == 1.0);
  return G;
}

// Centroid cells: about two centroids per cell (edge ~ (2 N_r / K)^(1/3)
// grid points), at most MAX_CELLS of them.
static void set_cells(KmGeom& G, int K) {
  const double nr = (double)G.n0 * G.n1 * G.n2;
  int e = (int)ceil(cbrt(2.0 * nr / K));
  if (e < 1) e = 1;
  for (;; ++e) {
    const int64_t c = ceil_div(G.n0, e) * ceil_div(G.n1, e) * ceil_div(G.n2, e);
    if (c <= MAX_CELLS) break;
  }
  G.cell = e;
  G.nc0 = (int)ceil_div(G.n0, e);
  G.nc1 = (int)ceil_div(G.n1, e);
  G.nc2 = (int)ceil_div(G.n2, e);
}

static int assign_blocks(const KmGeom& G) {
  int64_t nb = (int64_t)G.nb0 * G.nb1 * G.nb2;
  return (int)ceil_div(nb, ASSIGN_THREADS / ISDF_WAVE);
}

static bool grid_ok(const isdf_grid* g) {
  if (!g) return false;
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] <= 0) return false;
    if (!(g->h[a] > 0.0) || !(g->h[a] < 1e300)) return false;
  }
  int64_t nr = (int64_t)g->n[0] * g->n[1] * g->n[2];
  return nr < (int64_t)INT32_MAX;
}

}  // namespace isdf

using namespace isdf;

extern "C" size_t isdf_kmeans_workspace(const isdf_grid* grid, int32_t n_mu, int32_t max_iter) {
  if (!grid_ok(grid) || n_mu <= 0 || max_iter < 0) return 0;
  int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  KmGeom G = make_geom(grid);
  return plan_kmeans(nullptr, 0, nr, n_mu, max_iter, assign_blocks(G), true, true, true, true).bytes;
}

// Host checks shared by both K-means entry points (nothing touches the device).
static int kmeans_args(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi, int32_t n_phi,
                       const void* psi, int64_t ld_psi, int32_t n_psi, int32_t weight_kind, uint32_t flags,
                       int32_t n_mu, const double* c0, int32_t max_iter, double near_tie_rel, const int32_t* idx,
                       const double* w, const isdf_kmeans_info* info) {
  if (!dtype_valid(dt_in)) return ISDF_E_ARG;
  const isdf_dtype dt = (isdf_dtype)dt_in;
  if (!grid_ok(grid)) return ISDF_E_ARG;
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  const bool wgiven = (flags & ISDF_KM_WEIGHT_GIVEN) != 0;
  if (flags & ~ISDF_KM_WEIGHT_GIVEN) return ISDF_E_ARG;
  if (n_mu <= 0 || n_mu > nr || max_iter < 0 || !c0 || !idx || !info) return ISDF_E_ARG;
  if (!(near_tie_rel >= 0.0)) return ISDF_E_ARG;
  if (wgiven) {
    if (!w) return ISDF_E_ARG;
  } else {
    if (dt != ISDF_C128 && dt != ISDF_C64) return ISDF_E_ARG;
    if (weight_kind < ISDF_W_SSM || weight_kind > ISDF_W_SQM) return ISDF_E_ARG;
    if (!phi || !psi || n_phi <= 0 || n_psi <= 0 || ld_phi < n_phi || ld_psi < n_psi) return ISDF_E_ARG;
  }
  return ISDF_OK;
}

// Enqueues the whole K-means on `st` with the plan's arrays (carved from the
// caller's workspace or from the static scratch).
static int kmeans_enqueue(const isdf_grid* grid, isdf_dtype dt, const void* phi, int64_t ld_phi, int32_t n_phi,
                          const void* psi, int64_t ld_psi, int32_t n_psi, int32_t weight_kind, bool wgiven,
                          int32_t n_mu, const double* c0, int32_t max_iter, double near_tie_rel, int32_t* idx,
                          double* objective, isdf_kmeans_info* info, const KmGeom& G, int nparts, const KmPlan& P,
                          hipStream_t st) {
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  // state must be clean before the weight pass can flag non-finite values
  if (!fill<int>((int*)P.a.st, sizeof(KmState) / sizeof(int), 0, st)) return ISDF_E_HIP;
  if (!wgiven) {
    const bool aliased = phi == psi && ld_phi == ld_psi && n_phi == n_psi;
    int nmax = aliased ? n_phi : (n_phi > n_psi ? n_phi : n_psi);
    int sw = 64;
    while (sw > 1 && sw / 2 >= nmax) sw >>= 1;
    int64_t rows_per_block = (256 / 64) * (64 / sw);
    int64_t blocks = ceil_div(nr, rows_per_block);
    if (blocks > 8192) blocks = 8192;
    if (dt == ISDF_C128)
      hipLaunchKernelGGL(km_weight<double>, dim3((unsigned)blocks), dim3(256), 0, st, (const double*)phi,
                         ld_phi, n_phi, (const double*)psi, ld_psi, n_psi, aliased ? 1 : 0, weight_kind, sw,
                         nr, P.a.w, P.a.st);
    else
      hipLaunchKernelGGL(km_weight<float>, dim3((unsigned)blocks), dim3(256), 0, st, (const float*)phi, ld_phi,
                         n_phi, (const float*)psi, ld_psi, n_psi, aliased ? 1 : 0, weight_kind, sw, nr,
                         P.a.w, P.a.st);
    if (!launch_ok()) return ISDF_E_HIP;
  } else {
    int64_t blocks = ceil_div(nr, 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(km_check_weight, dim3((unsigned)blocks), dim3(256), 0, st, (const double*)P.a.w, nr,
                       P.a.st);
    if (!launch_ok()) return ISDF_E_HIP;
  }
  {
    int64_t work = nr > 3 * (int64_t)n_mu ? nr : 3 * (int64_t)n_mu;
    int64_t blocks = ceil_div(work, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(km_init, dim3((unsigned)blocks), dim3(256), 0, st, P.a, c0, n_mu, max_iter, nr, nparts);
    if (!launch_ok()) return ISDF_E_HIP;
  }
  const int ublocks = (int)ceil_div(n_mu, 4);
  for (int t = 0; t < max_iter; ++t) {
    hipLaunchKernelGGL(km_assign, dim3(nparts), dim3(ASSIGN_THREADS), 0, st, P.a, G, n_mu, t, near_tie_rel);
    hipLaunchKernelGGL(km_update, dim3(ublocks), dim3(256), 0, st, P.a, G, n_mu, t, nparts);
    hipLaunchKernelGGL(km_bin, dim3(1), dim3(BIN_THREADS), 0, st, P.a, G, n_mu);
  }
  hipLaunchKernelGGL(km_assign, dim3(nparts), dim3(ASSIGN_THREADS), 0, st, P.a, G, n_mu, max_iter,
                     near_tie_rel);
  hipLaunchKernelGGL(km_snap, dim3(ublocks), dim3(256), 0, st, P.a, G, n_mu, idx);
  hipLaunchKernelGGL(km_final, dim3(1), dim3(64), 0, st, P.a, nparts, info, objective, max_iter);
  if (!launch_ok()) return ISDF_E_HIP;
  return ISDF_OK;
}

extern "C" int isdf_kmeans(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi,
                           int32_t n_phi, const void* psi, int64_t ld_psi, int32_t n_psi,
                           int32_t weight_kind, uint32_t flags, int32_t n_mu, const double* c0,
                           int32_t max_iter, double near_tie_rel, int32_t* idx, double* centroids,
                           int32_t* labels, double* w, double* objective, isdf_kmeans_info* info,
                           void* ws, size_t ws_bytes, void* stream) {
  ISDF_TRY(kmeans_args(grid, dt_in, phi, ld_phi, n_phi, psi, ld_psi, n_psi, weight_kind, flags, n_mu, c0, max_iter,
                       near_tie_rel, idx, w, info));
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  KmGeom G = make_geom(grid);
  set_cells(G, n_mu);
  const int nparts = assign_blocks(G);
  KmPlan P = plan_kmeans(ws, ws_bytes, nr, n_mu, max_iter, nparts, !centroids, !labels, !w, !objective);
  if (P.bytes > ws_bytes || !ws) return ISDF_E_WORKSPACE;
  if (centroids) P.a.cent = centroids;
  if (labels) P.a.labels = labels;
  if (w) P.a.w = w;
  return kmeans_enqueue(grid, (isdf_dtype)dt_in, phi, ld_phi, n_phi, psi, ld_psi, n_psi, weight_kind,
                        (flags & ISDF_KM_WEIGHT_GIVEN) != 0, n_mu, c0, max_iter, near_tie_rel, idx, objective, info,
                        G, nparts, P, (hipStream_t)stream);
}

// ------------------------------------------------------ allocation-free form
// isdf_kmeans_noalloc keeps what isdf_kmeans carves from the caller's
// workspace (the state, per-round counters, per-cluster bounding boxes and
// objective partials) in this static array instead: one copy per GPU, which
// the GPU holds until the process ends.  Host code never uses the array's
// name as an address: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept below.
constexpr size_t KM_SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[KM_SCRATCH_BYTES];

namespace {
constexpr int KM_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[KM_MAX_DEVICES];  // device address of `scratch` per device (null: not looked up yet)

// Device address of this device's scratch, looked up on the first call on
// the device.  The stream must belong to the current device.
int scratch_address(hipStream_t stream, void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return ISDF_E_HIP;
  if (dev >= KM_MAX_DEVICES) return ISDF_E_UNSUPPORTED;
  if (stream) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return ISDF_E_HIP;
    if (sdev != dev) return ISDF_E_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ISDF_E_HIP;
    g_scratch_at[dev] = p;
  }
  *out = g_scratch_at[dev];
  return ISDF_OK;
}
}  // namespace

extern "C" int isdf_kmeans_noalloc(const isdf_grid* grid, int32_t dt_in, const void* phi, int64_t ld_phi,
                                   int32_t n_phi, const void* psi, int64_t ld_psi, int32_t n_psi,
                                   int32_t weight_kind, uint32_t flags, int32_t n_mu, const double* c0,
                                   int32_t max_iter, double near_tie_rel, int32_t* idx, double* centroids,
                                   int32_t* labels, double* w, double* objective, isdf_kmeans_info* info,
                                   void* stream) {
  ISDF_TRY(kmeans_args(grid, dt_in, phi, ld_phi, n_phi, psi, ld_psi, n_psi, weight_kind, flags, n_mu, c0, max_iter,
                       near_tie_rel, idx, w, info));
  if (!centroids || !labels || !w) return ISDF_E_ARG;  // outputs the workspace form may carve
  const int64_t nr = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  KmGeom G = make_geom(grid);
  set_cells(G, n_mu);
  const int nparts = assign_blocks(G);
  if (plan_kmeans(nullptr, 0, nr, n_mu, max_iter, nparts, false, false, false, false).bytes > KM_SCRATCH_BYTES)
    return ISDF_E_SCRATCH;
  hipStream_t st = (hipStream_t)stream;
  void* base = nullptr;
  ISDF_TRY(scratch_address(st, &base));
  KmPlan P = plan_kmeans(base, KM_SCRATCH_BYTES, nr, n_mu, max_iter, nparts, false, false, false, false);
  P.a.cent = centroids;
  P.a.labels = labels;
  P.a.w = w;
  return kmeans_enqueue(grid, (isdf_dtype)dt_in, phi, ld_phi, n_phi, psi, ld_psi, n_psi, weight_kind,
                        (flags & ISDF_KM_WEIGHT_GIVEN) != 0, n_mu, c0, max_iter, near_tie_rel, idx, objective, info,
                        G, nparts, P, st);
}
