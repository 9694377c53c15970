/*
 * isdf.h -- C ABI of the MI355X (gfx950) ISDF library (libisdf.so).
 *
 * Interpolative separable density fitting of complex Kohn-Sham orbitals,
 * after Jiao et al., arXiv:2208.07731:
 *   Z(r, (i,j)) = phi_i(r) conj(psi_j(r))          (Sec. 2.1)
 *   Z ~ Theta C,  C = rows of Z at N_mu interpolation points r_mu
 *   Theta = Z C^H (C C^H)^-1                        (eq. theta)
 * with Z C^H = (Phi Phi_mu^H) .* conj(Psi Psi_mu^H) (eqs. muRownuCol,
 * muRownuColden), so Z is never formed.  The interpolation points come from
 * weighted K-means over the grid points (Sec. 2.2, Alg. 1) with the
 * sum-of-square-moduli weight (eq. weight function 2, alpha = 2).
 *
 * Conventions shared by every call:
 *  - Every pointer is DEVICE memory unless marked (host).  The caller owns
 *    all memory; the library allocates nothing and keeps no state between
 *    calls (apart from the static scratch of isdf_kmeans_noalloc).
 *  - Every call is asynchronous on `stream` (a hipStream_t, NULL = default
 *    stream).  The return value reports argument errors found on the host
 *    before anything is enqueued (negative codes; nothing is written).
 *    Conditions found by the GPU are written to the device-side `info`
 *    struct, valid once the caller has synchronised `stream`.
 *  - Orbital matrices are r-major: row p of Phi holds phi_1(r_p) ..
 *    phi_{n_phi}(r_p) as interleaved complex numbers (re, im), row p starts
 *    at element p * ld (ld >= n in complex elements).  ISDF_C128 = pairs of
 *    double, ISDF_C64 = pairs of float.
 *  - Grid point p = (i * n[1] + j) * n[2] + k sits at grid coordinates
 *    (i, j, k); spacings h[3] weigh the Euclidean metric per axis by
 *    (h_a / min h)^2 (cubic grids: plain grid units).
 *  - psi == phi (same pointer, ld and count) selects the aliased path:
 *    Theta is real (the fit of |phi|^2-type products) and is stored as real
 *    numbers; otherwise Theta is complex.
 *  - Calls that share a workspace or output buffer must not overlap.
 */
#ifndef ISDF_H
#define ISDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
typedef enum {
  ISDF_OK = 0,
  ISDF_E_ARG = -1,          /* invalid argument (host check, nothing enqueued) */
  ISDF_E_WORKSPACE = -2,    /* ws_bytes below the *_workspace query */
  ISDF_E_HIP = -3,          /* a HIP runtime call failed while enqueueing */
  ISDF_E_UNSUPPORTED = -4,  /* valid request outside what the library implements (e.g. a grid axis isdf_poisson cannot transform) */
  ISDF_E_SCRATCH = -5,      /* request larger than the static scratch of an allocation-free entry point */
  ISDF_E_NOT_PD = 1,        /* device: C C^H not positive definite (see info->pivot) */
  ISDF_E_NONFINITE = 2,     /* device: NaN or Inf in the orbitals / weight */
  ISDF_W_EMPTY_CLUSTER = 3, /* device: a cluster lost all members (idx = -1) */
  ISDF_E_BAD_IDX = 4        /* device: interpolation index out of range or repeated */
} isdf_status;

/* Entry points take isdf_dtype and isdf_prec values as int32_t; any other
 * value is rejected with ISDF_E_ARG (workspace queries return 0). */
typedef enum { ISDF_C128 = 0, ISDF_C64 = 1 } isdf_dtype;

/* Precision of the Gram contractions Phi Phi_mu^H, Psi Psi_mu^H (and of the
 * adjoint contractions with the orbitals).  The factorisation and inverse
 * of C C^H and the product with it are always FP64. */
typedef enum {
  ISDF_P_FP64 = 0,    /* FP64 MFMA */
  ISDF_P_FP32 = 1,    /* FP32 MFMA, FP32 accumulation */
  ISDF_P_BF16X6 = 2,  /* operands split in three BF16 parts, 6 products, FP32 acc */
  ISDF_P_FP16X3 = 3   /* operands split in two scaled FP16 parts, 3 products, FP32 acc */
} isdf_prec;

/* K-means weight w(r) (Sec. 2.2).  SSM is the paper's choice. */
typedef enum {
  ISDF_W_SSM = 0,  /* sum_i |phi_i|^2 + sum_j |psi_j|^2   (eq. weight function 2, alpha=2) */
  ISDF_W_PSM = 1,  /* (sum_i |phi_i|^2)(sum_j |psi_j|^2)  (eq. weight function)           */
  ISDF_W_SM = 2,   /* alpha = 1 */
  ISDF_W_SCM = 3,  /* alpha = 3 */
  ISDF_W_SQM = 4   /* alpha = 4 */
} isdf_weight;

typedef struct {
  int32_t n[3];  /* grid points per axis, N_r = n0 n1 n2 */
  double h[3];   /* spacings (any positive unit); only their ratios matter */
} isdf_grid;

/* -------------------------------------------------------------- K-means */
/* flags of isdf_kmeans */
#define ISDF_KM_WEIGHT_GIVEN 1u /* `w` holds the weight on entry: skip its evaluation */

/* Written by the device at the end of isdf_kmeans. */
typedef struct {
  int32_t status;       /* ISDF_OK, ISDF_W_EMPTY_CLUSTER or ISDF_E_NONFINITE */
  int32_t iters;        /* classify+update rounds applied */
  int32_t converged;    /* 1 if a round left every label unchanged */
  int32_t empty_update; /* clusters of zero total weight at the last update (kept) */
  int32_t empty_final;  /* clusters without member at the final classification */
  int32_t ties;         /* points with two exactly equidistant nearest centroids */
  int32_t near_ties;    /* points with (d2 - d1) <= near_tie_rel * d2 */
  int32_t changed;      /* labels changed by the last round that ran */
  double objective;     /* sum_p w_p |r_p - c_label(p)|^2 at the final classification */
  int64_t pairs_evaluated; /* point-centroid distances evaluated, all classifications
                              (a full scan would take N_r n_mu per classification) */
  int64_t bound_tests;  /* brick-centroid lower-bound tests that chose them */
} isdf_kmeans_info;

/* Bytes of workspace isdf_kmeans needs.  Host-only, never synchronises. */
size_t isdf_kmeans_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t max_iter);

/*
 * Weighted K-means over the grid points (Alg. 1 of the paper):
 *   w    = weight of `weight_kind` from Phi and Psi   (skipped with ISDF_KM_WEIGHT_GIVEN)
 *   c    = c0
 *   repeat up to max_iter times:
 *     label_p = argmin_mu |r_p - c_mu|^2  (Euclidean; lowest mu on ties)     (eq. C_k)
 *     stop if no label changed since the previous round
 *     c_mu = sum_{p in C_mu} w_p r_p / sum_{p in C_mu} w_p  (kept if the sum is 0) (eq. r_k)
 *   final classification with the last centroids, then
 *   idx[mu] = member of C_mu nearest to c_mu (lowest p on ties; -1 if empty).
 * Stopping at a fixed point gives the same result as running all rounds.
 * Arguments:
 *   phi, psi       orbitals (see conventions); psi may equal phi.  Unused
 *                  (may be NULL) when ISDF_KM_WEIGHT_GIVEN is set.
 *   n_mu           number of clusters / interpolation points, 1 <= n_mu <= N_r
 *   c0             [n_mu][3] FP64 initial centroids in grid units (read only)
 *   max_iter       >= 0 rounds
 *   near_tie_rel   relative gap below which a point counts as a near tie (e.g. 1e-6)
 *   idx            [n_mu] int32 out: grid index of each interpolation point
 *   centroids      [n_mu][3] FP64 out, final centroids (NULL: not returned)
 *   labels         [N_r] int32 out, final cluster of every point (NULL: not returned)
 *   w              [N_r] FP64: out (or in with ISDF_KM_WEIGHT_GIVEN); NULL: not returned
 *   objective      [max_iter + 1] FP64 out, objective after each classification,
 *                  unused entries -1 (NULL: not returned)
 *   info           device struct, written at the end
 * Deterministic: equal inputs give bitwise equal outputs.
 */
int isdf_kmeans(const isdf_grid* grid /* host */, int32_t dt,
                const void* phi, int64_t ld_phi, int32_t n_phi,
                const void* psi, int64_t ld_psi, int32_t n_psi,
                int32_t weight_kind, uint32_t flags, int32_t n_mu,
                const double* c0, int32_t max_iter, double near_tie_rel,
                int32_t* idx, double* centroids, int32_t* labels, double* w,
                double* objective, isdf_kmeans_info* info,
                void* ws, size_t ws_bytes, void* stream);

/*
 * isdf_kmeans for callers that cannot allocate device memory (code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * allocation): the same computation and the same results bit for bit, with
 * the same arguments except that there is no workspace.  What isdf_kmeans
 * keeps in the workspace lives in a static 4 MiB device array of the library
 * instead (one per GPU, held until the process ends); the call allocates and
 * frees nothing.
 *   centroids, labels, w   required here (isdf_kmeans may carve them from the
 *                          workspace when they are NULL)
 *   stream                 must belong to the current device (else ISDF_E_ARG)
 * Requests whose scratch (about 56 n_mu + 40 max_iter + N_r / 64 bytes plus
 * 36 KiB) exceeds 4 MiB return ISDF_E_SCRATCH before anything is enqueued.  Every call on a GPU shares that GPU's scratch, and each
 * call re-initialises what it reads: calls that overlap on one GPU (on
 * different streams, or from different host threads without ordering) race
 * and give undefined results; calls ordered on one stream do not.
 */
int isdf_kmeans_noalloc(const isdf_grid* grid /* host */, int32_t dt,
                        const void* phi, int64_t ld_phi, int32_t n_phi,
                        const void* psi, int64_t ld_psi, int32_t n_psi,
                        int32_t weight_kind, uint32_t flags, int32_t n_mu,
                        const double* c0, int32_t max_iter, double near_tie_rel,
                        int32_t* idx, double* centroids, int32_t* labels, double* w,
                        double* objective, isdf_kmeans_info* info, void* stream);

/* ------------------------------------------------------------------ fit */
/* flags of isdf_fit / isdf_fit_backward */
#define ISDF_FIT_FACTOR 1u /* (re)build minv = (C C^H)^-1 from Phi, Psi, idx */

typedef struct {
  int32_t status;   /* ISDF_OK, ISDF_E_NOT_PD, ISDF_E_BAD_IDX */
  int32_t pivot;    /* first non-positive Cholesky pivot (row of minv), else -1 */
  int32_t bad_idx;  /* position in idx of the first invalid entry, else -1 */
  int32_t reserved;
  double pivot_min; /* min and max of the squared Cholesky diagonal of C C^H */
  double pivot_max;
  double loss;      /* isdf_fit_backward with the fused loss: its value */
} isdf_fit_info;

/* Elements (doubles) of the minv buffer: n'^2 with n' = n_mu (aliased) or 2 n_mu. */
size_t isdf_fit_minv_elems(int32_t n_mu, int32_t aliased);

/* Bytes of workspace for isdf_fit / isdf_fit_backward processing at most
 * `rblock` grid rows at a time.  Host-only. */
size_t isdf_fit_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t n_phi,
                          int32_t n_psi, int32_t aliased, int32_t prec, int64_t rblock);
size_t isdf_fit_backward_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t n_phi,
                                   int32_t n_psi, int32_t aliased, int32_t prec, int64_t rblock);

/*
 * Interpolation vectors for grid rows [row0, row0 + nrows):
 *   Theta = (Z C^H)(C C^H)^-1 (eq. theta), Z C^H = A .* conj(B),
 *   A = Phi Phi_mu^H, B = Psi Psi_mu^H (eq. muRownuColden), C C^H = rows idx of Z C^H.
 * Arguments:
 *   idx      [n_mu] int32 distinct grid indices (e.g. from isdf_kmeans)
 *   prec     precision of the Gram contractions (C C^H uses the same one)
 *   minv     [n'][n'] FP64 (n' = n_mu aliased, else 2 n_mu): with ISDF_FIT_FACTOR
 *            it is overwritten by (C C^H)^-1 (complex case: the real 2x2-block
 *            form [[re, im], [-im, re]] of each entry); without the flag it
 *            is read as left by an earlier call with the same inputs.
 *   theta    [nrows][ld_theta] out: real (aliased) or interleaved complex,
 *            double for ISDF_C128, float for ISDF_C64; ld_theta >= n_mu.
 *   rblock   rows processed per internal step (bounded by the workspace query)
 * Rows of Theta are independent given minv: any partition of the grid
 * rows into calls gives the same values.
 */
int isdf_fit(const isdf_grid* grid /* host */, int32_t dt,
             const void* phi, int64_t ld_phi, int32_t n_phi,
             const void* psi, int64_t ld_psi, int32_t n_psi,
             const int32_t* idx, int32_t n_mu, int32_t prec,
             double* minv, uint32_t flags, int64_t row0, int64_t nrows,
             void* theta, int64_t ld_theta, int64_t rblock,
             isdf_fit_info* info, void* ws, size_t ws_bytes, void* stream);

/*
 * The two halves of isdf_fit, as separate calls for callers that stream or
 * reuse Z C^H:
 *
 * isdf_zc: rows [row0, row0 + nrows) of Z C^H = A .* conj(B) (eq. muRownuCol
 * with eq. muRownuColden), Z never formed.  G is [nrows][ldg] FP64: real
 * (aliased, ldg >= n_mu) or interleaved complex (ldg >= 2 n_mu doubles).
 * Workspace: isdf_zc_workspace bytes for calls of up to `nrows` rows.
 */
size_t isdf_zc_workspace(int32_t n_mu, int32_t n_phi, int32_t n_psi, int32_t aliased, int32_t prec,
                         int64_t nrows);
int isdf_zc(const isdf_grid* grid /* host */, int32_t dt,
            const void* phi, int64_t ld_phi, int32_t n_phi,
            const void* psi, int64_t ld_psi, int32_t n_psi,
            const int32_t* idx, int32_t n_mu, int32_t prec,
            int64_t row0, int64_t nrows, double* G, int64_t ldg,
            void* ws, size_t ws_bytes, void* stream);

/*
 * isdf_zc_ab: isdf_zc that also keeps the Gram blocks of the same rows
 * (the P^phi and P^psi of eq. muRownuColden),
 *   A = Phi Phi_mu^H and (Psi != Phi only) B = Psi Psi_mu^H,
 * as [nrows][2 n_mu] interleaved complex FP64 (ld 2 n_mu), for
 * isdf_fit_backward_gram.  Same workspace as isdf_zc.  B is unused (may be
 * NULL) in the aliased case.
 */
int isdf_zc_ab(const isdf_grid* grid /* host */, int32_t dt,
               const void* phi, int64_t ld_phi, int32_t n_phi,
               const void* psi, int64_t ld_psi, int32_t n_psi,
               const int32_t* idx, int32_t n_mu, int32_t prec,
               int64_t row0, int64_t nrows, double* G, int64_t ldg, double* A, double* B,
               void* ws, size_t ws_bytes, void* stream);

/*
 * isdf_apply_minv: Theta = G (C C^H)^-1 for `nrows` rows (the solve of
 * eq. theta), minv as left by isdf_fit with ISDF_FIT_FACTOR, G as written by
 * isdf_zc.  theta: [nrows][ld_theta], real (aliased) or interleaved complex,
 * double (ISDF_C128) or float (ISDF_C64); ld_theta >= n_mu.  One FP64 GEMM
 * launch; no workspace.
 */
int isdf_apply_minv(int32_t n_mu, int32_t aliased, const double* minv, const double* G, int64_t ldg,
                    int64_t nrows, int32_t dt, void* theta, int64_t ld_theta, void* stream);

/*
 * Adjoint of isdf_fit with the interpolation points fixed (the paper gives
 * no adjoint; this is reverse-mode differentiation of eq. theta).  With
 * Theta = G M^-1, G = A .* conj(B), M = G[idx]:
 *   S = Thetabar M^-1,  Mbar = -Theta^H S,  Gbar = S, Gbar[idx] += Mbar,
 *   Abar = Gbar .* B,   Bbar = conj(Gbar) .* A,
 *   dPhi = Abar Phi_mu,  dPhi[idx] += Abar^H Phi,
 *   dPsi = Bbar Psi_mu,  dPsi[idx] += Bbar^H Psi,
 * in PyTorch's complex-gradient convention (dL/dRe + i dL/dIm).
 * Arguments:
 *   minv       as left by isdf_fit with ISDF_FIT_FACTOR on the same inputs
 *   theta_bar  [N_r][ld_tbar] upstream gradient, layout and type of Theta;
 *              NULL selects the fused loss L = sum_r g_r sum_mu |Theta_r,mu|^2
 *   g          [N_r] FP64 loss field (used only when theta_bar is NULL)
 *   dphi, dpsi [N_r][ld] gradients, same type as the orbitals, overwritten;
 *              in the aliased case dpsi may equal dphi (written once).
 *   loss       FP64 device scalar (fused loss only; NULL: not returned)
 *   rblock     grid rows per internal step; Theta is recomputed per block,
 *              never stored whole
 */
int isdf_fit_backward(const isdf_grid* grid /* host */, int32_t dt,
                      const void* phi, int64_t ld_phi, int32_t n_phi,
                      const void* psi, int64_t ld_psi, int32_t n_psi,
                      const int32_t* idx, int32_t n_mu, int32_t prec,
                      const double* minv,
                      const void* theta_bar, int64_t ld_tbar, const double* g,
                      void* dphi, int64_t ld_dphi, void* dpsi, int64_t ld_dpsi,
                      double* loss, int64_t rblock,
                      isdf_fit_info* info, void* ws, size_t ws_bytes, void* stream);

/*
 * isdf_fit_backward from the forward's Gram blocks: the same adjoint, with
 * the Gram product of every r-block replaced by the rows of G, A and B that
 * isdf_zc_ab wrote for the whole grid (G [N_r][n'] with n' = n_mu aliased
 * or 2 n_mu, A and B [N_r][2 n_mu]; B unused when Psi = Phi).  A, B and G
 * are consumed: the adjoint overwrites them in place.  The r-block loop and
 * every reduction order are those of isdf_fit_backward with the same rblock,
 * so the gradients and the loss are bitwise equal to it; the workspace
 * (isdf_fit_backward_gram_workspace) holds no r-block copies of G, A, B.
 * Trades N_r (n' + 2 n_mu [+ 2 n_mu]) doubles kept from the forward for one
 * Gram product per call.
 */
size_t isdf_fit_backward_gram_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t n_phi,
                                        int32_t n_psi, int32_t aliased, int32_t prec, int64_t rblock);
int isdf_fit_backward_gram(const isdf_grid* grid /* host */, int32_t dt,
                           const void* phi, int64_t ld_phi, int32_t n_phi,
                           const void* psi, int64_t ld_psi, int32_t n_psi,
                           const int32_t* idx, int32_t n_mu, int32_t prec,
                           const double* minv,
                           const void* theta_bar, int64_t ld_tbar, const double* g,
                           void* dphi, int64_t ld_dphi, void* dpsi, int64_t ld_dpsi,
                           double* loss, int64_t rblock, double* G, double* A, double* B,
                           isdf_fit_info* info, void* ws, size_t ws_bytes, void* stream);

/* flags of isdf_fit_backward_rows */
#define ISDF_BWD_FIRST 1u /* this call starts the sweep (state, packed rows, accumulators) */
#define ISDF_BWD_LAST 2u  /* this call ends it (interpolation-row terms, info, loss) */

/*
 * isdf_fit_backward_gram streamed over consecutive row blocks, for a forward
 * that runs block by block (isdf_zc_ab, then isdf_apply_minv, on rows
 * [row0, row0 + nrows)): each call takes that block's Gram rows G, A (and B)
 * right after the forward wrote them, so the Gram products are computed once
 * per step and only one block of G, A, B is ever held.  Same adjoint as
 * isdf_fit_backward (reverse mode of eq. theta, interpolation points fixed).
 *   row0, nrows   the block: rows [row0, row0 + nrows) of the grid
 *   rblock        the same value in every call of a sweep, >= nrows of each
 *                 call; the workspace is isdf_fit_backward_gram_workspace
 *                 with this rblock, and it carries the sweep's state
 *                 (accumulators of Theta^H S, Abar^H Phi, the loss) from call
 *                 to call
 *   G, A, B       the block's rows as isdf_zc_ab wrote them ([nrows][n'],
 *                 [nrows][2 n_mu]); consumed (overwritten in place)
 *   theta_bar     NULL (fused loss with field g) or the block's rows of the
 *                 upstream gradient ([nrows][ld_tbar]); the same choice in
 *                 every call of a sweep
 *   g             [N_r] loss field of the whole grid (fused loss)
 *   dphi, dpsi    [N_r][ld] of the whole grid: each call writes its block's
 *                 rows; the call with ISDF_BWD_LAST adds the terms at the
 *                 interpolation rows
 *   flags         ISDF_BWD_FIRST on the first block, ISDF_BWD_LAST on the last
 *                 (both for a single block)
 *   loss, info    written by the ISDF_BWD_LAST call
 * The blocks of a sweep must cover the grid once, in increasing row order,
 * on one stream.  With blocks of rblock rows (the last one ragged) the
 * gradients and the loss are bitwise those of isdf_fit_backward_gram with
 * the same rblock.
 */
int isdf_fit_backward_rows(const isdf_grid* grid /* host */, int32_t dt,
                           const void* phi, int64_t ld_phi, int32_t n_phi,
                           const void* psi, int64_t ld_psi, int32_t n_psi,
                           const int32_t* idx, int32_t n_mu, int32_t prec,
                           const double* minv,
                           const void* theta_bar, int64_t ld_tbar, const double* g,
                           void* dphi, int64_t ld_dphi, void* dpsi, int64_t ld_dpsi,
                           double* loss, int64_t row0, int64_t nrows, int64_t rblock,
                           double* G, double* A, double* B, uint32_t flags,
                           isdf_fit_info* info, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------- residuals */
/*
 * Least-squares residual of the fit without forming Z (follows from
 * eq. theta: Theta C C^H = Z C^H, so ||Theta C||^2 = Re sum conj(Z C^H) . Theta):
 *   out[0] = ||Z - Theta C||_F^2 = sum_r rho_phi(r) rho_psi(r) - Re sum conj(Z C^H) . Theta
 *   out[1] = ||Z||_F^2          = sum_r rho_phi(r) rho_psi(r)
 * with rho_phi = sum_i |phi_i|^2, rho_psi = sum_j |psi_j|^2, Theta the fit of
 * minv (as left by isdf_fit with ISDF_FIT_FACTOR on the same inputs), Z C^H in
 * precision `prec`, Theta and the sums in FP64.  out: device, 2 doubles.
 * Runs r-block by r-block (rblock rows); workspace: isdf_fit_residual_workspace
 * bytes.  Sums are in a fixed order (reproducible bit for bit).
 */
size_t isdf_fit_residual_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                                   int32_t aliased, int32_t prec, int64_t rblock);
int isdf_fit_residual(const isdf_grid* grid /* host */, int32_t dt,
                      const void* phi, int64_t ld_phi, int32_t n_phi,
                      const void* psi, int64_t ld_psi, int32_t n_psi,
                      const int32_t* idx, int32_t n_mu, int32_t prec,
                      const double* minv, int64_t rblock, double* out,
                      isdf_fit_info* info, void* ws, size_t ws_bytes, void* stream);

/*
 * Cluster residual of Appendix A (eqs. errorISDF and proj): every row Z(r)
 * replaced by its projection on the row of its cluster's interpolation point
 * p = idx[labels[r]],
 *   out[0] = R = sum_r [ rho_phi(r) rho_psi(r) - |Z(r) . Z*(p)|^2 / (rho_phi(p) rho_psi(p)) ],
 *   Z(r) . Z*(p) = (Phi(r) . Phi*(p)) conj(Psi(r) . Psi*(p))   (eq. Zmu),
 *   out[1] = number of rows skipped because labels[r] is outside [0, n_mu)
 *            or idx[labels[r]] is outside the grid,
 * labels [N_r] and idx [n_mu] as left by isdf_kmeans.  out: device, 2
 * doubles; workspace: isdf_cluster_residual_workspace() bytes.  FP64 sums in
 * a fixed order.
 */
size_t isdf_cluster_residual_workspace(void);
int isdf_cluster_residual(const isdf_grid* grid /* host */, int32_t dt,
                          const void* phi, int64_t ld_phi, int32_t n_phi,
                          const void* psi, int64_t ld_psi, int32_t n_psi,
                          const int32_t* labels, const int32_t* idx, int32_t n_mu, double* out,
                          void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ potentials */
/*
 * V_mu(r) = int zeta_mu(r') / |r - r'| dr' for every column zeta_mu of Theta
 * (eq. V_mu: the Poisson-like solves ISDF reduces to N_mu), on the periodic
 * grid: V-hat(G) = 4 pi zeta-hat(G) / |G|^2 with G = 2 pi m / (n_a h_a) per
 * axis and the G = 0 term dropped (neutralising background).
 *   theta  [N_r][ld_theta], N_r = n0 n1 n2 in the grid's point order; real
 *          (is_complex = 0, as isdf_fit returns for Psi = Phi) or
 *          interleaved complex; double (ISDF_C128) or float (ISDF_C64)
 *   V      [N_r][ld_v], same type and kind; may not alias theta
 * Every axis must be <= 256 points with prime factors in {2, 3, 5, 7}
 * (else ISDF_E_UNSUPPORTED).  FP64 arithmetic; workspace:
 * isdf_poisson_workspace bytes (0 for an unsupported grid).
 */
size_t isdf_poisson_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t is_complex);
int isdf_poisson(const isdf_grid* grid /* host */, int32_t dt, const void* theta, int64_t ld_theta,
                 int32_t n_mu, int32_t is_complex, void* V, int64_t ld_v, void* ws, size_t ws_bytes,
                 void* stream);

/*
 * ISDF-compressed exchange operator (eq. v2): for every psi_j,
 *   W(r, j) = (V_X psi_j)(r) ~ - sum_mu conj(V_mu(r)) A(r, mu) psi_j(r_mu),
 *   A = Phi Phi_mu^H,
 * with V the potentials isdf_poisson returns for the fit's Theta (eq. v2
 * expands the pair density phi_i* psi_j, the conjugate of the one the fit
 * interpolates, whose interpolation vectors are conj(Theta)).
 *   phi [N_r][ld_phi] (the occupied orbitals), psi [N_r][ld_psi] (the
 *   orbitals the operator acts on), idx [n_mu]: as for isdf_fit
 *   V   [N_r][ld_v], real (v_complex = 0) or interleaved complex, same
 *       storage type as the orbitals
 *   W   [N_r][ld_w] interleaved complex, storage type of the orbitals
 * FP64 arithmetic, rblock grid rows per step; workspace:
 * isdf_exchange_workspace bytes.
 */
size_t isdf_exchange_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                               int64_t rblock);
int isdf_exchange(const isdf_grid* grid /* host */, int32_t dt,
                  const void* phi, int64_t ld_phi, int32_t n_phi,
                  const void* psi, int64_t ld_psi, int32_t n_psi,
                  const int32_t* idx, int32_t n_mu, const void* V, int64_t ld_v, int32_t v_complex,
                  void* W, int64_t ld_w, int64_t rblock, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------- QRCP interpolation points */
/* Written by the device at the end of isdf_qrcp. */
typedef struct {
  int32_t status;    /* ISDF_OK or ISDF_E_NONFINITE */
  int32_t rank;      /* pivots accepted: n_mu unless the residual fell to rtol |R_00| first */
  int32_t near_ties; /* accepted steps whose gap <= near_tie_rel */
  int32_t reserved;
  double r00;        /* |R_00| = max_r |Z(r)| */
} isdf_qrcp_info;

/* Bytes of workspace isdf_qrcp needs (0 for invalid sizes): about
 * (n_mu - 1) N_r doubles, twice that for Psi != Phi.  Host-only. */
size_t isdf_qrcp_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t aliased);

/*
 * Interpolation points by QR factorisation with column pivoting of Z^T
 * (Sec. 2.1, eq. QRCP; the baseline the paper compares K-means against):
 *   Z^T Pi = Q R, |R_00| >= |R_11| >= ...,  idx[k] = grid point of pivot k.
 * Z is not formed: the pivots are those of the pivoted Cholesky
 * factorisation of Z Z^H = (Phi Phi^H) .* conj(Psi Psi^H), whose diagonal
 * after k steps holds the squared residual norms of Z^T's columns.  Step k
 * takes the largest residual (lowest grid index on exact ties).  The paper's
 * randomized variant approximates these exact pivots.
 * Arguments:
 *   phi, psi      orbitals (see conventions); psi == phi selects the aliased
 *                 (real Gram) path
 *   n_mu          pivots wanted, 1 <= n_mu <= N_r
 *   rtol          stop once the largest residual |R_kk| <= rtol |R_00|; the
 *                 Gram formulation resolves |R_kk| down to about 1e-7 |R_00|
 *                 in FP64, so rtol should not be smaller
 *   near_tie_rel  steps whose gap <= near_tie_rel are counted in info
 *   idx           [n_mu] int32 out: pivot grid indices in order; -1 from rank on
 *   rdiag         [n_mu] FP64 out: |R_kk|; 0 from rank on
 *   gap           [n_mu] FP64 out (NULL: not returned): (s1 - s2) / s1 for the
 *                 two largest squared residuals s1 >= s2 at step k, the
 *                 margin of the pivot choice
 *   info          device struct, written at the end
 * FP64 arithmetic throughout; C64 orbitals are widened on load.  Cost:
 * n_mu passes over the orbitals and over the growing factor L (N_r x k),
 * O(n_mu N_r (N_phi + N_psi) + n_mu^2 N_r) (Table 1: QRCP is O(N_mu^2 N_r)).
 * ISDF_E_UNSUPPORTED if Phi(p) and Psi(p) do not fit the step kernel's LDS
 * (N_phi + N_psi above about 3000).  Deterministic: equal inputs give
 * bitwise equal outputs.
 */
int isdf_qrcp(const isdf_grid* grid /* host */, int32_t dt,
              const void* phi, int64_t ld_phi, int32_t n_phi,
              const void* psi, int64_t ld_psi, int32_t n_psi,
              int32_t n_mu, double rtol, double near_tie_rel,
              int32_t* idx, double* rdiag, double* gap, isdf_qrcp_info* info,
              void* ws, size_t ws_bytes, void* stream);

/*
 * Randomized QRCP (Sec. 1 and Sec. 2.1: the standard IP selection the paper
 * compares against): the pivoted QR of eq. QRCP applied to the sketch
 * (Z Omega)^T (m x N_r) instead of Z^T, with Omega the Khatri-Rao product
 *   Omega[(i, j)][k] = g_phi[i][k] g_psi[j][k],
 * so that X = Z Omega = (Phi g_phi) .* conj(Psi g_psi) (N_r x m, one FP64
 * Hadamard Gram product of the fit's kind, two right-hand sides even when
 * psi == phi); then the pivots of the pivoted Cholesky of X X^H, as in
 * isdf_qrcp.
 *   g_phi [n_phi][m], g_psi [n_psi][m]  FP64 device: the random numbers
 *        (the caller draws them, e.g. standard normal)
 *   m    sketch size, m >= 1; at most m pivots exist, so m >= n_mu for a
 *        full set
 *   other arguments and outputs as isdf_qrcp.
 * Cost: 8 N_r m (N_phi + N_psi) flops for X, then n_mu passes over X and
 * over L: more than isdf_qrcp whenever m > (N_phi + N_psi) / 2.  Workspace:
 * isdf_qrcp_sketch_workspace bytes (X, [N_r][m] complex, plus a complex L).
 */
size_t isdf_qrcp_sketch_workspace(const isdf_grid* grid /* host */, int32_t n_mu, int32_t n_phi, int32_t n_psi,
                                  int32_t m);
int isdf_qrcp_sketch(const isdf_grid* grid /* host */, int32_t dt,
                     const void* phi, int64_t ld_phi, int32_t n_phi,
                     const void* psi, int64_t ld_psi, int32_t n_psi,
                     const double* g_phi, const double* g_psi, int32_t m,
                     int32_t n_mu, double rtol, double near_tie_rel,
                     int32_t* idx, double* rdiag, double* gap, isdf_qrcp_info* info,
                     void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- misc */
const char* isdf_version(void);
const char* isdf_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* ISDF_H */
