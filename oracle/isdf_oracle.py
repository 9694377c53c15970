"""Plain FP64 CPU oracle of the ISDF decomposition (weighted K-means + fit + adjoint).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product library
never does, and this file shares no code, table or helper with the HIP path.

Written from arXiv:2208.07731 (Jiao et al., "Complex-valued K-means
clustering of interpolative separable density fitting ...").  Every function
cites the passage it follows.  Arithmetic is numpy/scipy complex128/float64,
one library primitive per step (matmul, Cholesky, triangular solve), with no
blocking or fusion beyond what the cited definition states.

Readings taken where the paper is silent or garbled (each is also listed in
the design notes):
* Z has entries phi_i(r) conj(psi_j(r)) (Sec. 2.1, eq. decomposition / Cmu);
  the least-squares solution of Z ~ Theta C for complex data is
  Theta = Z C^H (C C^H)^-1 (eq. theta written with transposes in real
  notation), and the (r, nu) entry of Z C^H is
  P^phi(r, r_nu) * conj(P^psi(r, r_nu)) (eq. muRownuCol / muRownuColden).
* C C^H is the Hermitian positive definite block of Z C^H at the
  interpolation rows (Sec. 2.4); it is factored by Cholesky.  A non positive
  definite block is reported, never regularised.
* K-means (Alg. 1, eqs. opt / r_k): Euclidean distance on grid coordinates
  (no minimum image), lowest centroid index wins ties, a cluster with zero
  total weight keeps its centroid, at most `max_iter` classify+update rounds
  that stop early at a fixed point, then one final classification; the
  interpolation point of a cluster is its member nearest to the final
  centroid (lowest grid index on ties), because interpolation points are grid
  points (Sec. 2.1) while centroids are not.
* Distances: D = ((s0*dx*dx) + (s1*dy*dy)) + (s2*dz*dz) in grid units with
  s_a = (h_a / min h)^2 (s = 1 on cubic grids, where integer-valued
  coordinates make first-iteration ties exact).
* QRCP interpolation points (Sec. 2.1, eq. QRCP): the exact pivoted QR
  factorisation of Z^T, which the paper's randomized QRCP approximates; the
  numerical rank ends at |R_kk| <= rtol |R_00|.
* The adjoint is not in the paper; it is derived by reverse-mode
  differentiation of the fit with the interpolation points held fixed, in
  PyTorch's complex-gradient convention dL/dRe + i dL/dIm.

Parity status: every function here is pinned by the CPU tests against
closed forms, brute force or library least squares, except where a
docstring says "parity unpinned".
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np
import scipy.linalg as sla

__all__ = [
    "WEIGHT_KINDS", "weight", "grid_points", "metric_scale", "sqdist",
    "assign", "update", "snap", "kmeans", "gather", "gram_blocks", "hadamard",
    "fit", "fit_theta", "fit_backward", "fit_residual", "cluster_residual",
    "cc_condition", "explicit_z", "reciprocal_sq", "poisson", "exchange", "exchange_direct",
    "qrcp", "qrcp_sketch", "khatri_rao_sketch", "qrcp_greedy_excess", "qrcp_sampled_check",
]

# --------------------------------------------------------------------------
# a1: weight function (Sec. 2.2, eq. weight function and eq. weight function 2)
# --------------------------------------------------------------------------
WEIGHT_KINDS = ("ssm", "psm", "sm", "scm", "sqm")


def _abs_pow(x: np.ndarray, alpha: int) -> np.ndarray:
    """|x|^alpha elementwise for complex x, from s = re^2 + im^2."""
    s = x.real * x.real + x.imag * x.imag
    if alpha == 2:
        return s
    if alpha == 1:
        return np.sqrt(s)
    if alpha == 3:
        return s * np.sqrt(s)
    if alpha == 4:
        return s * s
    raise ValueError(alpha)


def weight(phi: np.ndarray, psi: np.ndarray | None = None, kind: str = "ssm") -> np.ndarray:
    """K-means weight w(r), float64 (N_r,).

    * "ssm" (the paper's improved weight, alpha = 2 in eq. weight function 2):
      sum_i |phi_i|^2 + sum_j |psi_j|^2;
    * "sm", "scm", "sqm": the same sum with alpha = 1, 3, 4 (Sec. 2.2);
    * "psm" (the earlier real-valued weight, eq. weight function):
      (sum_i |phi_i|^2) * (sum_j |psi_j|^2).
    psi=None means Psi is Phi.
    """
    if psi is None:
        psi = phi
    if kind == "psm":
        return _abs_pow(phi, 2).sum(axis=1) * _abs_pow(psi, 2).sum(axis=1)
    alpha = {"ssm": 2, "sm": 1, "scm": 3, "sqm": 4}[kind]
    return _abs_pow(phi, alpha).sum(axis=1) + _abs_pow(psi, alpha).sum(axis=1)


# --------------------------------------------------------------------------
# a2-a6: weighted K-means on grid points (Sec. 2.2, eqs. opt, r_k; Alg. 1)
# --------------------------------------------------------------------------
def grid_points(n) -> np.ndarray:
    """Grid coordinates in grid units, float64 (N_r, 3); p = (i*n1 + j)*n2 + k."""
    n0, n1, n2 = (n, n, n) if np.isscalar(n) else tuple(n)
    i, j, k = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    return np.stack([i.reshape(-1), j.reshape(-1), k.reshape(-1)], axis=1).astype(np.float64)


def metric_scale(h=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Per-axis weights s_a = (h_a / min h)^2 of the Euclidean metric."""
    h = np.asarray(h, dtype=np.float64)
    return (h / h.min()) ** 2


def sqdist(pts: np.ndarray, cents: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances (P, K): ((s0*dx*dx) + (s1*dy*dy)) + (s2*dz*dz)."""
    dx = pts[:, None, 0] - cents[None, :, 0]
    dy = pts[:, None, 1] - cents[None, :, 1]
    dz = pts[:, None, 2] - cents[None, :, 2]
    if np.all(s == 1.0):
        return (dx * dx + dy * dy) + dz * dz
    return (s[0] * (dx * dx) + s[1] * (dy * dy)) + s[2] * (dz * dz)


def _threads() -> int:
    return int(os.environ.get("ISDF_ORACLE_THREADS", os.cpu_count() or 1))


def assign(pts: np.ndarray, cents: np.ndarray, s: np.ndarray, chunk: int = 2048):
    """Classification step of Alg. 1 / eq. C_k: label_p = first argmin_mu D_pmu.

    Returns (labels int32, d1 = nearest distance, d2 = second nearest, inf if
    there is one centroid).
    """
    n_pts = pts.shape[0]
    labels = np.empty(n_pts, dtype=np.int32)
    d1 = np.empty(n_pts)
    d2 = np.empty(n_pts)

    def work(lo):
        hi = min(lo + chunk, n_pts)
        D = sqdist(pts[lo:hi], cents, s)
        a = np.argmin(D, axis=1)
        rows = np.arange(hi - lo)
        labels[lo:hi] = a
        d1[lo:hi] = D[rows, a]
        if D.shape[1] > 1:
            D[rows, a] = np.inf
            d2[lo:hi] = D.min(axis=1)
        else:
            d2[lo:hi] = np.inf

    starts = range(0, n_pts, chunk)
    nt = _threads()
    if nt > 1 and n_pts > chunk:
        with _cf.ThreadPoolExecutor(nt) as ex:
            list(ex.map(work, starts))
    else:
        for lo in starts:
            work(lo)
    return labels, d1, d2


def update(pts: np.ndarray, w: np.ndarray, labels: np.ndarray, cents: np.ndarray):
    """Centroid step of Alg. 1 / eq. r_k: r_mu = sum_{C_mu} w r / sum_{C_mu} w.

    A cluster whose total weight is zero keeps its centroid.  Returns
    (new centroids, number of such clusters).
    """
    K = cents.shape[0]
    sw = np.bincount(labels, weights=w, minlength=K)
    out = cents.copy()
    ok = sw > 0
    for a in range(3):
        sa = np.bincount(labels, weights=w * pts[:, a], minlength=K)
        out[ok, a] = sa[ok] / sw[ok]
    return out, int(K - ok.sum())


def snap(pts: np.ndarray, labels: np.ndarray, cents: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Interpolation point of each cluster: its member nearest to the centroid,
    lowest grid index on ties; -1 for an empty cluster (Sec. 2.1: interpolation
    points are grid points; Alg. 1's last step read as this snap)."""
    K = cents.shape[0]
    c = cents[labels]
    dx = pts[:, 0] - c[:, 0]
    dy = pts[:, 1] - c[:, 1]
    dz = pts[:, 2] - c[:, 2]
    if np.all(s == 1.0):
        d = (dx * dx + dy * dy) + dz * dz
    else:
        d = (s[0] * (dx * dx) + s[1] * (dy * dy)) + s[2] * (dz * dz)
    p = np.arange(pts.shape[0])
    order = np.lexsort((p, d, labels))
    lab_sorted = labels[order]
    first = np.ones(order.shape[0], dtype=bool)
    first[1:] = lab_sorted[1:] != lab_sorted[:-1]
    idx = np.full(K, -1, dtype=np.int32)
    idx[lab_sorted[first]] = order[first]
    return idx


def kmeans(n, w: np.ndarray, c0: np.ndarray, max_iter: int, h=(1.0, 1.0, 1.0),
           near_tie_rel: float = 1e-6) -> dict:
    """Weighted K-means on the grid (Alg. 1) with the readings in the module
    docstring.  Returns dict with idx, centroids, labels, d1, d2, J (objective
    of eq. opt at each classification), iters (update rounds run), converged,
    empty (clusters with zero weight at the last update), ties, near_ties,
    near_tie_mask."""
    pts = grid_points(n)
    s = metric_scale(h)
    c = np.array(c0, dtype=np.float64, copy=True)
    prev = None
    J = []
    iters = 0
    converged = False
    empty = 0
    labels = d1 = d2 = None
    for _ in range(max_iter):
        labels, d1, d2 = assign(pts, c, s)
        J.append(float(np.dot(w, d1)))
        if prev is not None and np.array_equal(labels, prev):
            converged = True
            break
        c, empty = update(pts, w, labels, c)
        iters += 1
        prev = labels
    if not converged:
        labels, d1, d2 = assign(pts, c, s)
        J.append(float(np.dot(w, d1)))
    idx = snap(pts, labels, c, s)
    gap = d2 - d1
    near = np.isfinite(d2) & (gap <= near_tie_rel * d2)
    return dict(idx=idx, centroids=c, labels=labels, d1=d1, d2=d2, J=np.array(J),
                iters=iters, converged=converged, empty=empty,
                ties=int(np.count_nonzero(d1 == d2)), near_ties=int(near.sum()),
                near_tie_mask=near)


# --------------------------------------------------------------------------
# a7-a12: least-squares fit of the interpolation vectors (Sec. 2.1,
# eqs. decomMatrix, theta, muRownuCol, muRownuColden; Sec. 2.4)
# --------------------------------------------------------------------------
def gather(x: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Rows of an orbital matrix at the interpolation points (eq. Cmu)."""
    return x[np.asarray(idx)]


def gram_blocks(phi: np.ndarray, psi: np.ndarray, idx: np.ndarray, rows=None):
    """A = Phi Phi_mu^H and B = Psi Psi_mu^H, i.e. P^phi(r, r_nu) and
    P^psi(r, r_nu) of eq. muRownuColden, for all grid rows (or `rows`)."""
    pr = phi if rows is None else phi[rows]
    sr = psi if rows is None else psi[rows]
    A = pr @ gather(phi, idx).conj().T
    B = sr @ gather(psi, idx).conj().T
    return A, B


def hadamard(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """(Z C^H)(r, nu) = P^phi(r, r_nu) conj(P^psi(r, r_nu)) (eq. muRownuCol, with
    the conjugate that complex orbitals require)."""
    return A * B.conj()


def _cc(phi, psi, idx):
    """C C^H: the rows of Z C^H at the interpolation points (Sec. 2.4)."""
    Am, Bm = gram_blocks(phi, psi, idx, rows=np.asarray(idx))
    return hadamard(Am, Bm)


def fit(phi: np.ndarray, psi: np.ndarray, idx: np.ndarray, rows=None) -> dict:
    """Theta = Z C^H (C C^H)^-1 (eq. theta), by Cholesky of C C^H and two
    triangular solves.  Returns dict(theta, G, M, L, A, B) for all rows (or
    the rows listed in `rows`: rows of Theta are independent given C C^H)."""
    A, B = gram_blocks(phi, psi, idx, rows)
    G = hadamard(A, B)
    M = _cc(phi, psi, idx)
    try:
        L = sla.cholesky(M, lower=True, check_finite=True)
    except np.linalg.LinAlgError as e:
        raise np.linalg.LinAlgError("C C^H is not positive definite") from e
    Y = sla.solve_triangular(L, G.conj().T, lower=True)
    theta_h = sla.solve_triangular(L.conj().T, Y, lower=False)
    return dict(theta=theta_h.conj().T, G=G, M=M, L=L, A=A, B=B)


def fit_theta(phi, psi, idx, rows=None) -> np.ndarray:
    return fit(phi, psi, idx, rows)["theta"]


def cc_condition(phi, psi, idx) -> float:
    """2-norm condition number of C C^H (Sec. 2.4's matrix), from its
    eigenvalues; a diagnostic printed beside parity errors."""
    ev = np.linalg.eigvalsh(_cc(phi, psi, idx))
    return float(ev[-1] / ev[0]) if ev[0] > 0 else float("inf")


def fit_residual(phi, psi, idx, theta=None) -> float:
    """||Z - Theta C||_F^2 without forming Z:
    sum_r rho_phi(r) rho_psi(r) - Re sum conj(Z C^H) . Theta, valid for the
    least-squares Theta (diagnostic; the quantity Appendix A bounds)."""
    f = fit(phi, psi, idx)
    th = f["theta"] if theta is None else theta
    rp = (phi.real ** 2 + phi.imag ** 2).sum(axis=1)
    rs = (psi.real ** 2 + psi.imag ** 2).sum(axis=1)
    return float(np.dot(rp, rs) - np.real(np.sum(f["G"].conj() * th)))


def cluster_residual(phi: np.ndarray, psi: np.ndarray, labels: np.ndarray, idx: np.ndarray) -> float:
    """Appendix A, eqs. errorISDF and proj: the residual of representing
    every row Z(r) by its projection on the row of its cluster's
    interpolation point, R = sum_mu sum_{r in C_mu} ||Z(r) - proj Z(r)||^2,
    with proj Z(r) = (Z(r) . Z*(r_mu)) / (Z(r_mu) . Z*(r_mu)) Z(r_mu).

    Without forming Z (eq. Zmu and the first lines of eq. error2):
    Z(r) . Z*(r') = (Phi(r) . Phi*(r')) conj(Psi(r) . Psi*(r')), so
    Z(r) . Z*(r) = rho_phi(r) rho_psi(r) and each term is
    rho_phi(r) rho_psi(r) - |Z(r) . Z*(r_mu)|^2 / (rho_phi(r_mu) rho_psi(r_mu)).
    """
    labels = np.asarray(labels)
    idx = np.asarray(idx)
    p = idx[labels]                                    # interpolation point of each row's cluster
    rp = (phi.real ** 2 + phi.imag ** 2).sum(axis=1)   # rho_phi
    rs = (psi.real ** 2 + psi.imag ** 2).sum(axis=1)   # rho_psi
    a = np.sum(phi * phi[p].conj(), axis=1)            # Phi(r) . Phi*(r_mu)
    b = np.sum(psi * psi[p].conj(), axis=1)            # Psi(r) . Psi*(r_mu)
    zz = a * b.conj()                                  # Z(r) . Z*(r_mu)
    terms = rp * rs - (zz.real ** 2 + zz.imag ** 2) / (rp[p] * rs[p])
    return float(np.sum(terms))


def reciprocal_sq(n, h) -> np.ndarray:
    """|G|^2 on the grid's reciprocal lattice, G_a = 2 pi m_a / (n_a h_a) with
    m_a the FFT-order integers in [-n_a/2, n_a/2); shape (n0, n1, n2)."""
    g = [2.0 * np.pi * np.fft.fftfreq(n[a], d=1.0 / n[a]) / (n[a] * h[a]) for a in range(3)]
    return g[0][:, None, None] ** 2 + g[1][None, :, None] ** 2 + g[2][None, None, :] ** 2


def poisson(theta: np.ndarray, n, h=(1.0, 1.0, 1.0)) -> np.ndarray:
    """V_mu(r) = int zeta_mu(r') / |r - r'| dr' (eq. V_mu) for every column
    zeta_mu of theta [N_r][N_mu] on the periodic grid (p = (i n1 + j) n2 + k,
    spacings h in Bohr): V-hat(G) = 4 pi zeta-hat(G) / |G|^2, with the G = 0
    term dropped (a neutralising background; the paper does not state how the
    periodic integral is regularised).  Same layout and dtype kind as theta."""
    n = tuple(int(x) for x in (n if not np.isscalar(n) else (n, n, n)))
    g2 = reciprocal_sq(n, h)
    kern = np.zeros_like(g2)
    kern[g2 > 0] = 4.0 * np.pi / g2[g2 > 0]
    z = theta.reshape(n + (theta.shape[1],))
    zh = np.fft.fftn(z, axes=(0, 1, 2))
    v = np.fft.ifftn(zh * kern[..., None], axes=(0, 1, 2)).reshape(theta.shape)
    return v.real.copy() if np.isrealobj(theta) else v


def exchange(phi: np.ndarray, psi: np.ndarray, idx: np.ndarray, v: np.ndarray) -> np.ndarray:
    """ISDF-compressed exchange of eq. v2: (V_X psi_j)(r) ~
    -sum_mu V'_mu(r) sum_i phi_i(r) phi_i*(r_mu) psi_j(r_mu), i.e.
    -((V' . A) Psi_mu) with A = Phi Phi_mu^H.  Eq. v2 expands the pair
    density phi_i* psi_j, the complex conjugate of Sec. 2.1's
    z_ij = phi_i psi_j*, whose interpolation vectors are conj(Theta); the
    potentials of those are conj(V) for V = poisson(Theta) (the Poisson
    operator is real), so V' = conj(v).  Returns [N_r][N_psi] complex."""
    idx = np.asarray(idx)
    A = phi @ phi[idx].conj().T
    return -((np.conj(v) * A) @ psi[idx])


def exchange_direct(phi: np.ndarray, psi: np.ndarray, n, h=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Exact exchange of eq. vx / eq. v on the grid, for checking eq. v2:
    (V_X psi_j)(r) = -sum_i phi_i(r) V[phi_i* psi_j](r), with V[.] the
    periodic Poisson potential of poisson().  Tiny inputs only (N_phi N_psi
    potentials)."""
    out = np.zeros((phi.shape[0], psi.shape[1]), dtype=np.complex128)
    for j in range(psi.shape[1]):
        pair = phi.conj() * psi[:, j:j + 1]             # phi_i*(r') psi_j(r'), one column per i
        out[:, j] = -np.sum(phi * poisson(pair, n, h), axis=1)
    return out


def explicit_z(phi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Z (N_r x N_phi N_psi), z_(i,j)(r) = phi_i(r) conj(psi_j(r)) (Sec. 2.1).
    Tiny inputs only: memory is O(N_r N_phi N_psi)."""
    return (phi[:, :, None] * psi.conj()[:, None, :]).reshape(phi.shape[0], -1)


# --------------------------------------------------------------------------
# interpolation points by QR with column pivoting (Sec. 2.1, eq. QRCP; Table 1)
# --------------------------------------------------------------------------
def _suffix_sq(w: np.ndarray) -> np.ndarray:
    """s[k, j] = sum_{i >= k} |w[i, j]|^2: the squared norm of column j of a
    matrix whose rows are coordinates in an orthonormal basis, once the first
    k basis vectors are projected out."""
    a = w.real ** 2 + w.imag ** 2
    return np.cumsum(a[::-1], axis=0)[::-1]


def _qrcp_columns(mt: np.ndarray, n_mu: int, rtol: float) -> dict:
    """Pivoted Householder QR (LAPACK geqp3) of a matrix whose columns are
    the grid points: returns the first n_mu pivots with |R_kk|, decision
    margins and numerical rank, as documented in qrcp()."""
    r, piv = sla.qr(mt, mode="r", pivoting=True)
    m = min(mt.shape)
    r = r[:m]
    kmax = min(n_mu, m)
    s = _suffix_sq(r)
    rdiag = np.zeros(n_mu)
    gap = np.zeros(n_mu)
    idx = np.full(n_mu, -1, dtype=np.int64)
    d = np.abs(np.diag(r))
    rank = 0
    for k in range(kmax):
        if not d[k] > rtol * d[0]:
            break
        rank = k + 1
        idx[k] = piv[k]
        rdiag[k] = d[k]
        rest = s[k, k + 1:]
        s2 = rest.max() if rest.size else 0.0
        gap[k] = (s[k, k] - s2) / s[k, k]
    return dict(idx=idx, rdiag=rdiag, gap=gap, rank=rank)


def qrcp(phi: np.ndarray, psi: np.ndarray, n_mu: int, rtol: float = 1e-7) -> dict:
    """Interpolation points from the QR factorisation with column pivoting
    of Z^T (Sec. 2.1, eq. QRCP): Z^T Pi = Q R with |R_kk| non-increasing; the
    first n_mu pivot columns of Z^T (grid points) are the interpolation
    points.  Z is formed explicitly (tiny inputs only) and factored by
    LAPACK's pivoted Householder QR (geqp3).  The paper's baseline is a
    randomized QRCP that approximates these pivots from a sketch of Z^T
    (qrcp_sketch); this is the exact factorisation it approximates.

    Returns dict:
      idx    [n_mu] int64 grid index of pivot k; -1 from the numerical rank on
      rdiag  [n_mu] |R_kk| (0 from the rank on)
      gap    [n_mu] (s_1 - s_2) / s_1 with s_1 >= s_2 the two largest squared
             residual column norms at step k: the margin of the pivot choice
      rank   number of k < n_mu with |R_kk| > rtol |R_00|
    Exact ties follow LAPACK's column order (not necessarily lowest index).
    """
    return _qrcp_columns(explicit_z(phi, psi).T, n_mu, rtol)   # (N_phi N_psi) x N_r


def khatri_rao_sketch(g_phi: np.ndarray, g_psi: np.ndarray) -> np.ndarray:
    """Omega [(i, j)][k] = g_phi[i, k] g_psi[j, k]: the column-wise Kronecker
    (Khatri-Rao) product of two random matrices, the test matrix that maps
    the N_phi N_psi rows of Z^T to m sketch rows."""
    return (g_phi[:, None, :] * g_psi[None, :, :]).reshape(-1, g_phi.shape[1])


def qrcp_sketch(phi: np.ndarray, psi: np.ndarray, n_mu: int, g_phi: np.ndarray, g_psi: np.ndarray,
                rtol: float = 1e-7) -> dict:
    """Randomized QRCP (Sec. 1 and Sec. 2.1: the standard IP selection the
    paper compares against): the pivoted QR of eq. QRCP applied to the
    sketch (Z Omega)^T, m x N_r, instead of Z^T, with Omega the Khatri-Rao
    product of the real random matrices g_phi [N_phi][m] and g_psi
    [N_psi][m] (the random numbers are inputs).  Z Omega is formed
    explicitly from Z here; its entry (r, k) equals
    (Phi g_phi[:, k])(r) conj((Psi g_psi[:, k])(r)).  Same return value as
    qrcp()."""
    y = explicit_z(phi, psi) @ khatri_rao_sketch(g_phi, g_psi)   # N_r x m
    return _qrcp_columns(y.T, n_mu, rtol)


def _greedy_excess(mt: np.ndarray, idx) -> np.ndarray:
    idx = np.asarray(idx)
    q, _ = np.linalg.qr(mt[:, idx], mode="complete")
    s = _suffix_sq(q.conj().T @ mt)
    ex = np.array([s[k].max() - s[k, idx[k]] for k in range(len(idx))])
    return ex / s[0, idx[0]]


def qrcp_greedy_excess(phi: np.ndarray, psi: np.ndarray, idx, g_phi=None, g_psi=None) -> np.ndarray:
    """Brute-force check of the pivot rule behind eq. QRCP for a given pivot
    order: with Q_k an orthonormal basis of the first k chosen columns of
    Z^T (or of the sketch (Z Omega)^T when g_phi, g_psi are given), pivot k
    must have the largest norm of (I - Q_k Q_k^H) z over all columns z.
    Returns, per step, (max_z s_k(z) - s_k(idx[k])) / s_0(idx[0]), which is
    >= 0 up to rounding and 0 for a greedy order.  Tiny inputs only.  A
    property test: `idx` may come from any implementation."""
    z = explicit_z(phi, psi)
    if g_phi is not None:
        z = z @ khatri_rao_sketch(g_phi, g_psi)
    return _greedy_excess(z.T, idx)


def qrcp_sampled_check(phi: np.ndarray, psi: np.ndarray, idx, rdiag, rows) -> dict:
    """Properties of a pivot sequence that hold at any size, computed
    without Z from its Gram matrix K = Z Z^H = (Phi Phi^H) .* conj(Psi Psi^H)
    (whose pivoted Cholesky factor L has |L_kk| = |R_kk| of eq. QRCP):
      * rdiag[k]^2 equals the k-th squared diagonal of the Cholesky factor of
        K at the pivots (in pivot order): returns the largest difference
        relative to the first (rdiag_rel);
      * greedy rule at the sampled grid rows: the squared residual of every
        sampled non-pivot row after k steps, K_rr - sum_{j<k} |L_rj|^2, is
        at most rdiag[k]^2: returns the largest excess relative to rdiag[0]^2.
    A property test: idx and rdiag may come from any implementation."""
    idx = np.asarray(idx)
    rows = np.setdiff1d(np.asarray(rows), idx)
    kpp = hadamard(*gram_blocks(phi, psi, idx, rows=idx))
    lp = sla.cholesky(kpp, lower=True)
    diag2 = np.abs(np.diag(lp)) ** 2
    rd2 = np.asarray(rdiag, dtype=np.float64) ** 2
    rel = float(np.max(np.abs(diag2 - rd2)) / diag2[0])
    krp = hadamard(*gram_blocks(phi, psi, idx, rows=rows))       # K(rows, P)
    lr = sla.solve_triangular(lp, krp.conj().T, lower=True).conj().T   # L(rows, :) = K(rows, P) L_P^-H
    krr = ((phi[rows].real ** 2 + phi[rows].imag ** 2).sum(axis=1)
           * (psi[rows].real ** 2 + psi[rows].imag ** 2).sum(axis=1))
    a = lr.real ** 2 + lr.imag ** 2
    before = krr[:, None] - np.concatenate([np.zeros((len(rows), 1)), np.cumsum(a, axis=1)[:, :-1]], axis=1)
    excess = float(np.max(before - rd2[None, :]) / rd2[0])
    return dict(rdiag_rel=rel, greedy_excess=excess)


# --------------------------------------------------------------------------
# a13-a16: adjoint of the fit with the interpolation points fixed (derived)
# --------------------------------------------------------------------------
def fit_backward(phi: np.ndarray, psi: np.ndarray, idx: np.ndarray,
                 theta_bar: np.ndarray | None = None, g: np.ndarray | None = None) -> dict:
    """Gradients of a real loss through Theta = G M^-1, G = A . conj(B),
    M = G[idx], A = Phi Phi_mu^H, B = Psi Psi_mu^H.

    theta_bar given: the upstream gradient dL/dRe(Theta) + i dL/dIm(Theta).
    theta_bar None: fused loss L = sum_r g_r sum_mu |Theta_rmu|^2, for which
    theta_bar = 2 g . Theta.
    Returns dict(dphi, dpsi, loss).  The two orbital sets are treated as
    independent inputs even when they hold equal values.
    """
    idx = np.asarray(idx)
    f = fit(phi, psi, idx)
    th, A, B, L = f["theta"], f["A"], f["B"], f["L"]
    loss = None
    if theta_bar is None:
        loss = float(np.sum(g[:, None] * (th.real ** 2 + th.imag ** 2)))
        theta_bar = 2.0 * g[:, None] * th
    # S = theta_bar M^-1  (M Hermitian): S^H = M^-1 theta_bar^H
    S = sla.cho_solve((L, True), theta_bar.conj().T).conj().T
    Mbar = -(th.conj().T @ S)
    Gbar = S.copy()
    Gbar[idx] += Mbar
    Abar = Gbar * B
    Bbar = Gbar.conj() * A
    dphi = Abar @ gather(phi, idx)
    dphi[idx] += Abar.conj().T @ phi
    dpsi = Bbar @ gather(psi, idx)
    dpsi[idx] += Bbar.conj().T @ psi
    return dict(dphi=dphi, dpsi=dpsi, loss=loss)
