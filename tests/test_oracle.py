"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the property and the passage of arXiv:2208.07731 it rests on.
None of them re-types the oracle's own formula: they use explicit Z (brute
force), library least squares, closed forms, invariances and independent
differentiation.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth

EPS = np.finfo(np.float64).eps


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def haar_unitary(rng, n):
    q, r = np.linalg.qr(crandn(rng, n, n))
    return q * (np.diag(r) / np.abs(np.diag(r)))


# --------------------------------------------------------------- weight (a1)
def test_weight_kinds_closed_form():
    """eq. weight function 2 with alpha = 1..4 and eq. weight function (PSM)
    on a one-point grid with |phi| = 5, |psi| = 13 (3-4-5 and 5-12-13)."""
    phi = np.array([[3 + 4j]])
    psi = np.array([[5 - 12j]])
    assert oracle.weight(phi, psi, "ssm")[0] == 25 + 169
    assert oracle.weight(phi, psi, "sm")[0] == 5 + 13
    assert oracle.weight(phi, psi, "scm")[0] == 125 + 2197
    assert oracle.weight(phi, psi, "sqm")[0] == 625 + 28561
    assert oracle.weight(phi, psi, "psm")[0] == 25 * 169


def test_weight_sum_is_orbital_count(water8):
    """Orthonormal columns: sum_r w_r = N_phi + N_psi for SSM (Sec. 2.2)."""
    phi = water8["phi"]
    w = oracle.weight(phi, phi)
    assert abs(w.sum() - 2 * phi.shape[1]) <= 1e-13 * 2 * phi.shape[1]
    rng = np.random.default_rng(7)
    a = synth.random_orthonormal(300, 5, 1)
    b = synth.random_orthonormal(300, 9, 2)
    assert abs(oracle.weight(a, b).sum() - 14) < 1e-13 * 14
    del rng


def test_weight_aliased_is_twice_density(water8):
    """Psi = Phi: w = 2 sum|phi|^2 exactly (x + x = 2x in binary FP)."""
    phi = water8["phi"]
    w = oracle.weight(phi, None)
    rho = (np.abs(phi) ** 2).sum(axis=1)
    assert np.allclose(w, 2 * rho, rtol=1e-14, atol=0)


def test_weight_gauge_invariant():
    """w depends on the orbitals only through the density: Phi -> Phi U
    leaves it unchanged (rel <= 1e-14)."""
    rng = np.random.default_rng(3)
    phi = synth.random_orthonormal(200, 6, 11)
    psi = synth.random_orthonormal(200, 4, 12)
    w = oracle.weight(phi, psi)
    w2 = oracle.weight(phi @ haar_unitary(rng, 6), psi @ haar_unitary(rng, 4))
    assert np.max(np.abs(w2 - w) / w) < 1e-13


# --------------------------------------------------------------- K-means (a2-a6)
def brute_labels(pts, cents):
    """Pure-Python argmin of squared Euclidean distance, lowest index on ties."""
    out = []
    for p in pts:
        best, bi = None, -1
        for m, c in enumerate(cents):
            d = sum((float(p[a]) - float(c[a])) ** 2 for a in range(3))
            if best is None or d < best:
                best, bi = d, m
        out.append(bi)
    return np.array(out)


def test_kmeans_single_cluster_is_weighted_mean():
    """eq. r_k with one cluster: the centroid is the weighted mean of all grid
    points, reached after one update, then a fixed point."""
    rng = np.random.default_rng(0)
    n = 6
    w = rng.uniform(0.1, 2.0, n ** 3)
    pts = oracle.grid_points(n)
    km = oracle.kmeans(n, w, np.array([[0.0, 0.0, 0.0]]), 10)
    ref = np.average(pts, axis=0, weights=w)
    assert np.allclose(km["centroids"][0], ref, rtol=1e-14, atol=0)
    assert km["converged"] and km["iters"] == 1
    # snapped point: nearest grid point to the centroid, by brute force
    d = ((pts - km["centroids"][0]) ** 2).sum(axis=1)
    assert km["idx"][0] == int(np.argmin(d))


def test_kmeans_uniform_blocks_fixed_point():
    """Uniform weight on an 8^3 grid with seeds at {1,6}^3: the Voronoi cells
    are the eight 4^3 blocks, the centroids their centres {1.5, 5.5}^3, and
    the snapped point of each block is its lowest-index corner of the central
    2^3 cube (eight members tie at distance 3/4)."""
    n = 8
    w = np.ones(n ** 3)
    c0 = np.array([[a, b, c] for a in (1, 6) for b in (1, 6) for c in (1, 6)], dtype=float)
    km = oracle.kmeans(n, w, c0, 20)
    exp = np.array([[a, b, c] for a in (1.5, 5.5) for b in (1.5, 5.5) for c in (1.5, 5.5)])
    assert np.array_equal(km["centroids"], exp)
    assert np.array_equal(np.bincount(km["labels"], minlength=8), np.full(8, 64))
    assert km["converged"] and km["iters"] == 1
    corner = [(1 if a < 4 else 5, 1 if b < 4 else 5, 1 if c < 4 else 5) for a, b, c in exp]
    assert list(km["idx"]) == [(i * n + j) * n + k for i, j, k in corner]
    # objective: 8 blocks x 3 axes x 16 lines x (2.25 + 0.25 + 0.25 + 2.25)
    assert km["J"][-1] == 8 * 3 * 16 * (2.25 + 0.25 + 0.25 + 2.25)


def test_kmeans_exact_ties_lowest_index():
    """eq. C_k puts an equidistant point in every nearest cluster; the reading
    taken is the lowest centroid index.  Seeds on grid points make the first
    distances exact integers, so the tie is exact."""
    n = 5
    w = np.ones(n ** 3)
    c0 = np.array([[2.0, 2.0, 0.0], [2.0, 2.0, 4.0]])  # plane k = 2 is equidistant
    km = oracle.kmeans(n, w, c0, 0)
    pts = oracle.grid_points(n)
    mid = pts[:, 2] == 2
    assert np.all(km["labels"][mid] == 0)
    assert km["ties"] == int(mid.sum())


def test_kmeans_objective_monotone_and_bruteforce(water8):
    """Lloyd iterations never increase the objective of eq. opt, and the final
    labels / centroids / snapped points agree with brute force."""
    phi = water8["phi"]
    w = oracle.weight(phi, phi)
    km = oracle.kmeans(water8["wl"].n, w, water8["c0"], 30)
    J = km["J"]
    assert np.all(np.diff(J) <= 1e-12 * J[0])
    assert km["empty"] == 0 and np.all(km["idx"] >= 0)
    assert len(np.unique(km["idx"])) == len(km["idx"])


def test_kmeans_bruteforce_small():
    """Tiny grid: every step against pure-Python loops."""
    rng = np.random.default_rng(5)
    n = 6
    w = rng.uniform(0.0, 1.0, n ** 3) ** 4
    pts = oracle.grid_points(n)
    c0 = pts[rng.choice(n ** 3, 7, replace=False)]
    km = oracle.kmeans(n, w, c0, 4)
    # final labels: brute-force argmin against final centroids
    assert np.array_equal(km["labels"], brute_labels(pts, km["centroids"]))
    # centroids: replay the iteration with Python loops
    c = c0.copy()
    prev = None
    for _ in range(4):
        lab = brute_labels(pts, c)
        if prev is not None and np.array_equal(lab, prev):
            break
        newc = c.copy()
        for m in range(len(c)):
            mem = np.nonzero(lab == m)[0]
            sw = sum(w[p] for p in mem)
            if sw > 0:
                newc[m] = [sum(w[p] * pts[p][a] for p in mem) / sw for a in range(3)]
        c, prev = newc, lab
    assert np.allclose(km["centroids"], c, rtol=1e-13, atol=1e-13)
    # snap: nearest member of each cluster, lowest index on ties
    for m in range(len(c)):
        mem = [p for p in range(n ** 3) if km["labels"][p] == m]
        d = [sum((pts[p][a] - km["centroids"][m][a]) ** 2 for a in range(3)) for p in mem]
        assert km["idx"][m] == mem[int(np.argmin(d))]


def test_kmeans_stop_at_fixed_point_is_invisible(water8):
    """Stopping early at a fixed point gives the same result as running the
    full iteration count (reading of the loop condition of Alg. 1)."""
    phi = water8["phi"]
    w = oracle.weight(phi, phi)
    a = oracle.kmeans(water8["wl"].n, w, water8["c0"], 200)
    assert a["converged"]
    b = oracle.kmeans(water8["wl"].n, w, water8["c0"], a["iters"] + 5)
    assert np.array_equal(a["idx"], b["idx"]) and np.array_equal(a["centroids"], b["centroids"])


def test_kmeans_weight_scale_bit_identical(water8):
    """Scaling w by 2^k leaves every centroid, label and point bit-identical."""
    phi = water8["phi"]
    w = oracle.weight(phi, phi)
    a = oracle.kmeans(water8["wl"].n, w, water8["c0"], 5)
    b = oracle.kmeans(water8["wl"].n, w * 2.0 ** -40, water8["c0"], 5)
    assert np.array_equal(a["centroids"], b["centroids"])
    assert np.array_equal(a["idx"], b["idx"])


def test_kmeans_metric_scale():
    """Anisotropic spacing weighs each axis by (h_a / min h)^2: with h = (1, 2, 1)
    a point at dy = 1 is farther than one at dx = 1.9."""
    s = oracle.metric_scale((1.0, 2.0, 1.0))
    assert np.array_equal(s, [1.0, 4.0, 1.0])
    d = oracle.sqdist(np.array([[0.0, 0.0, 0.0]]), np.array([[1.9, 0, 0], [0, 1.0, 0]]), s)
    assert d[0, 0] < d[0, 1]


# --------------------------------------------------------------- fit (a7-a12)
def tiny_case(seed, n_r=40, n_phi=5, n_psi=7, n_mu=12):
    rng = np.random.default_rng(seed)
    phi = crandn(rng, n_r, n_phi)
    psi = crandn(rng, n_r, n_psi)
    idx = rng.choice(n_r, n_mu, replace=False)
    return phi, psi, idx


def test_hadamard_identity_explicit_z():
    """eq. muRownuCol: Z C^H built from explicit Z equals A . conj(B)."""
    phi, psi, idx = tiny_case(1)
    Z = oracle.explicit_z(phi, psi)
    # explicit Z by loops for an independent check of its layout
    for r in (0, 17):
        for i in range(phi.shape[1]):
            for j in range(psi.shape[1]):
                ref = phi[r, i] * np.conj(psi[r, j])
                assert abs(Z[r, i * psi.shape[1] + j] - ref) <= 4 * EPS * abs(ref)
    C = Z[idx]
    zc = Z @ C.conj().T
    A, B = oracle.gram_blocks(phi, psi, idx)
    G = oracle.hadamard(A, B)
    assert np.max(np.abs(zc - G)) <= 1e-13 * np.max(np.abs(G))


def test_cc_condition_closed_forms():
    """kappa_2(C C^H) (Sec. 2.4's matrix) in closed form.
    (i) Rows at the points are scaled unit vectors a_mu e_mu, Psi = Phi:
        A(r_mu, r_nu) = a_mu^2 delta, C C^H = diag(a_mu^4), kappa = max/min.
    (ii) Two points, Phi = Psi, rows e_1 and (cos t, sin t): C C^H =
        [[1, cos^2 t], [cos^2 t, 1]], kappa = (1 + cos^2 t) / (1 - cos^2 t).
    (iii) Two points, complex Psi != Phi with rows e_1, (i cos u, sin u):
        off-diagonal cos t * i cos u, kappa = (1 + cos t cos u) / (1 - cos t cos u)."""
    rng = np.random.default_rng(71)
    a = np.array([0.5, 1.0, 1.7, 2.0, 0.9])
    phi = crandn(rng, 40, 5)
    idx = np.array([3, 11, 19, 27, 35])
    phi[idx] = np.diag(a)
    assert abs(oracle.cc_condition(phi, phi, idx) - (a.max() / a.min()) ** 4) <= 1e-13 * (a.max() / a.min()) ** 4
    t, u = np.pi / 3, np.pi / 5
    phi = crandn(rng, 9, 2)
    psi = crandn(rng, 9, 2)
    idx = np.array([2, 6])
    phi[2], phi[6] = [1.0, 0.0], [np.cos(t), np.sin(t)]
    want = (1 + np.cos(t) ** 2) / (1 - np.cos(t) ** 2)
    assert abs(oracle.cc_condition(phi, phi, idx) - want) <= 1e-14 * want
    psi[2], psi[6] = [1.0, 0.0], [1j * np.cos(u), np.sin(u)]
    cc = np.cos(t) * np.cos(u)
    want = (1 + cc) / (1 - cc)
    assert abs(oracle.cc_condition(phi, psi, idx) - want) <= 1e-14 * want


def test_cc_condition_against_explicit_c_and_lapack():
    """kappa_2(C C^H) equals (s_max / s_min)^2 of the singular values of C
    taken from explicit Z (Sec. 2.1: C = rows of Z at the points), complex and
    Psi = Phi; for a diagonal C C^H it also equals LAPACK's 1-norm estimate
    (pocon, exact for diagonal matrices)."""
    for seed, aliased in ((72, False), (73, True)):
        phi, psi, idx = tiny_case(seed, n_r=50, n_phi=4, n_psi=5, n_mu=9)
        if aliased:
            psi = phi
        C = oracle.explicit_z(phi, psi)[idx]
        sv = np.linalg.svd(C, compute_uv=False)
        want = (sv[0] / sv[-1]) ** 2
        assert abs(oracle.cc_condition(phi, psi, idx) - want) <= 1e-9 * want
    a = np.array([3.0, 1.0, 0.25, 2.0])
    phi = np.zeros((10, 4), dtype=complex)
    idx = np.array([1, 4, 6, 9])
    phi[idx] = np.diag(a)
    M = np.diag(a ** 4)
    rcond, info = sla.lapack.dpocon(np.asfortranarray(np.linalg.cholesky(M).T), np.linalg.norm(M, 1), uplo="U")
    assert info == 0
    assert abs(oracle.cc_condition(phi, phi, idx) * rcond - 1.0) <= 1e-12


def test_fit_is_least_squares():
    """eq. theta: Theta minimises ||Z - Theta C||_F (library least squares) and
    satisfies the normal equations (Z - Theta C) C^H = 0."""
    phi, psi, idx = tiny_case(2, n_r=60)
    Z = oracle.explicit_z(phi, psi)
    C = Z[idx]
    th = oracle.fit_theta(phi, psi, idx)
    ref = sla.lstsq(C.T, Z.T)[0].T
    assert np.linalg.norm(th - ref) <= 1e-12 * np.linalg.norm(ref)
    ne = (Z - th @ C) @ C.conj().T
    assert np.linalg.norm(ne) <= 1e-12 * np.linalg.norm(Z) * np.linalg.norm(C)


def test_fit_interpolates_at_points(water8):
    """Theta(r_mu) = I: the fit reproduces Z exactly at the interpolation
    points (tolerance 10 * kappa(C C^H) * eps)."""
    phi = water8["phi"]
    w = oracle.weight(phi, phi)
    idx = oracle.kmeans(water8["wl"].n, w, water8["c0"], 30)["idx"]
    th = oracle.fit_theta(phi, phi, idx, rows=idx)
    kappa = oracle.cc_condition(phi, phi, idx)
    assert np.max(np.abs(th - np.eye(len(idx)))) <= 10 * kappa * EPS


def test_fit_full_rank_is_permutation():
    """N_mu = N_r (possible when N_r <= N_phi N_psi): every grid point is an
    interpolation point and Theta is the permutation e_r -> mu."""
    rng = np.random.default_rng(4)
    n_r = 30
    phi, psi = crandn(rng, n_r, 6), crandn(rng, n_r, 6)
    idx = rng.permutation(n_r)
    th = oracle.fit_theta(phi, psi, idx)
    P = np.zeros((n_r, n_r))
    P[idx, np.arange(n_r)] = 1.0
    assert np.max(np.abs(th - P)) <= 1e-11


def test_fit_swap_conjugates_and_aliased_is_real():
    """Z(Psi, Phi) = conj(Z(Phi, Psi)) up to a column permutation, so swapping
    the orbital sets conjugates Theta; Psi = Phi makes Theta real."""
    phi, psi, idx = tiny_case(5)
    a = oracle.fit_theta(phi, psi, idx)
    b = oracle.fit_theta(psi, phi, idx)
    assert np.linalg.norm(b - a.conj()) <= 1e-13 * np.linalg.norm(a)
    c = oracle.fit_theta(phi, phi, idx[:5])
    assert np.max(np.abs(c.imag)) <= 1e-13 * np.max(np.abs(c.real))


def test_fit_gauge_invariant():
    """Phi -> Phi U, Psi -> Psi V (unitary): Z -> Z (U x conj V) with a unitary
    Kronecker factor, which leaves the least-squares Theta unchanged."""
    rng = np.random.default_rng(6)
    phi, psi, idx = tiny_case(6, n_r=50)
    a = oracle.fit_theta(phi, psi, idx)
    b = oracle.fit_theta(phi @ haar_unitary(rng, 5), psi @ haar_unitary(rng, 7), idx)
    kappa = oracle.cc_condition(phi, psi, idx)
    assert np.linalg.norm(b - a) <= 10 * kappa * EPS * np.linalg.norm(a)


def test_fit_scale_bit_identical():
    """Scaling Phi and Psi by powers of two leaves Theta bit-identical."""
    phi, psi, idx = tiny_case(7)
    a = oracle.fit_theta(phi, psi, idx)
    b = oracle.fit_theta(phi * 2.0 ** 5, psi * 2.0 ** -9, idx)
    assert np.array_equal(a, b)


def test_fit_real_orbitals_real_theta():
    """Real orbitals (Gamma point): Theta is real and equals the least-squares
    fit computed in real arithmetic with the library solver."""
    rng = np.random.default_rng(8)
    phi = rng.standard_normal((50, 5)).astype(complex)
    psi = rng.standard_normal((50, 6)).astype(complex)
    idx = rng.choice(50, 10, replace=False)
    th = oracle.fit_theta(phi, psi, idx)
    Z = (phi.real[:, :, None] * psi.real[:, None, :]).reshape(50, -1)
    ref = np.linalg.lstsq(Z[idx].T, Z.T, rcond=None)[0].T
    assert np.max(np.abs(th.imag)) == 0.0 or np.max(np.abs(th.imag)) < 1e-14
    assert np.linalg.norm(th.real - ref) <= 1e-12 * np.linalg.norm(ref)


def test_fit_residual_formula():
    """||Z - Theta C||^2 = sum rho_phi rho_psi - Re sum conj(Z C^H) . Theta
    against the explicit residual."""
    phi, psi, idx = tiny_case(9, n_r=45)
    Z = oracle.explicit_z(phi, psi)
    th = oracle.fit_theta(phi, psi, idx)
    ref = np.linalg.norm(Z - th @ Z[idx]) ** 2
    assert abs(oracle.fit_residual(phi, psi, idx) - ref) <= 1e-11 * np.linalg.norm(Z) ** 2


def test_cluster_residual_against_explicit_projection():
    """Appendix A residual R by its definition (eqs. errorISDF, proj) on an
    explicit Z: each row minus its projection on its cluster's interpolation
    row; clusters from a real K-means run on a tiny grid."""
    rng = np.random.default_rng(31)
    n = 5
    x = rng.standard_normal((n ** 3, 7)) + 1j * rng.standard_normal((n ** 3, 7))
    y = rng.standard_normal((n ** 3, 4)) + 1j * rng.standard_normal((n ** 3, 4))
    w = oracle.weight(x, y)
    c0 = oracle.grid_points(n)[rng.choice(n ** 3, 9, replace=False)]
    km = oracle.kmeans(n, w, c0, 5)
    Z = oracle.explicit_z(x, y)
    ref = 0.0
    for r in range(n ** 3):
        zm = Z[km["idx"][km["labels"][r]]]
        proj = (Z[r] @ zm.conj()) / (zm @ zm.conj()) * zm
        ref += np.linalg.norm(Z[r] - proj) ** 2
    got = oracle.cluster_residual(x, y, km["labels"], km["idx"])
    assert abs(got - ref) <= 1e-12 * np.linalg.norm(Z) ** 2


def test_cluster_residual_bounds_and_limits():
    """R >= the least-squares residual (the cluster projection is one
    particular Theta supported on the interpolation rows); R = 0 when every
    point is its own interpolation point; R scales as 4^(2k) under
    Phi, Psi -> 2^k Phi, 2^k Psi."""
    phi, psi, idx = tiny_case(12, n_r=60)
    # clusters: every row to the interpolation point nearest in Z-row angle
    Z = oracle.explicit_z(phi, psi)
    zi = Z[idx]
    cos = np.abs(Z @ zi.conj().T) / (np.linalg.norm(Z, axis=1)[:, None] * np.linalg.norm(zi, axis=1)[None, :])
    labels = np.argmax(cos, axis=1).astype(np.int32)
    labels[idx] = np.arange(len(idx))
    R = oracle.cluster_residual(phi, psi, labels, idx)
    assert R >= oracle.fit_residual(phi, psi, idx) * (1 - 1e-12)
    everyone = np.arange(phi.shape[0])
    assert abs(oracle.cluster_residual(phi, psi, everyone, everyone)) <= 1e-13 * np.linalg.norm(Z) ** 2
    assert oracle.cluster_residual(2 * phi, 2 * psi, labels, idx) == 16 * R


def test_fit_not_pd_raises():
    """A duplicated interpolation point makes C C^H singular: reported, not
    regularised."""
    phi, psi, idx = tiny_case(10)
    idx = idx.copy()
    idx[1] = idx[0]
    with pytest.raises(np.linalg.LinAlgError):
        oracle.fit(phi, psi, idx)


# --------------------------------------------------------------- adjoint (a13-a16)
def _loss(phi, psi, idx, g):
    th = oracle.fit_theta(phi, psi, idx)
    return float(np.sum(g[:, None] * np.abs(th) ** 2))


def test_backward_central_fd():
    """Fused loss L = sum_r g_r sum_mu |Theta_rmu|^2: the gradient matches
    central finite differences (h = 1e-6) on random entries, real and
    imaginary parts."""
    rng = np.random.default_rng(11)
    n_r = 60
    phi = synth.random_orthonormal(n_r, 5, 21)
    psi = synth.random_orthonormal(n_r, 6, 22)
    idx = rng.choice(n_r, 14, replace=False)
    g = rng.uniform(0.5, 1.5, n_r)
    bw = oracle.fit_backward(phi, psi, idx, g=g)
    assert abs(bw["loss"] - _loss(phi, psi, idx, g)) <= 1e-12 * bw["loss"]
    h = 1e-6
    for which, grad in (("phi", bw["dphi"]), ("psi", bw["dpsi"])):
        X = phi if which == "phi" else psi
        for _ in range(10):
            r, c = rng.integers(n_r), rng.integers(X.shape[1])
            for unit in (1.0, 1j):
                Xp, Xm = X.copy(), X.copy()
                Xp[r, c] += unit * h
                Xm[r, c] -= unit * h
                args_p = (Xp, psi) if which == "phi" else (phi, Xp)
                args_m = (Xm, psi) if which == "phi" else (phi, Xm)
                fd = (_loss(*args_p, idx, g) - _loss(*args_m, idx, g)) / (2 * h)
                an = grad[r, c].real if unit == 1.0 else grad[r, c].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, np.max(np.abs(grad))), (which, r, c, unit, fd, an)


def test_backward_matches_torch_autograd():
    """Against reverse-mode autograd of a plain complex128 torch formula
    (LU solve, not Cholesky), with a general upstream gradient."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    n_r = 70
    phi = crandn(rng, n_r, 6)
    psi = crandn(rng, n_r, 5)
    idx = rng.choice(n_r, 16, replace=False)
    tbar = crandn(rng, n_r, 16)
    bw = oracle.fit_backward(phi, psi, idx, theta_bar=tbar)
    P = torch.tensor(phi, requires_grad=True)
    S = torch.tensor(psi, requires_grad=True)
    it = torch.tensor(idx)
    A = P @ P[it].conj().T
    B = S @ S[it].conj().T
    G = A * B.conj()
    M = G[it]
    th = torch.linalg.solve(M.transpose(0, 1), G.transpose(0, 1)).transpose(0, 1)
    # real loss whose theta-gradient is tbar: L = Re sum conj(tbar) . theta
    L = torch.real(torch.sum(torch.tensor(tbar).conj() * th))
    L.backward()
    for ours, ref in ((bw["dphi"], P.grad.numpy()), (bw["dpsi"], S.grad.numpy())):
        assert np.linalg.norm(ours - ref) <= 1e-10 * np.linalg.norm(ref)


def test_backward_gauge_invariants():
    """L is invariant under Phi -> Phi U (U unitary) and Phi -> c Phi, so
    dPhi^H Phi is Hermitian and traceless (same for Psi)."""
    rng = np.random.default_rng(13)
    n_r = 64
    phi = synth.random_orthonormal(n_r, 6, 31)
    psi = synth.random_orthonormal(n_r, 5, 32)
    idx = rng.choice(n_r, 15, replace=False)
    g = rng.uniform(0.5, 1.5, n_r)
    bw = oracle.fit_backward(phi, psi, idx, g=g)
    for X, dX in ((phi, bw["dphi"]), (psi, bw["dpsi"])):
        H = dX.conj().T @ X
        scale = np.linalg.norm(dX) * np.linalg.norm(X)
        assert np.linalg.norm(H - H.conj().T) <= 1e-11 * scale
        assert abs(np.trace(H)) <= 1e-11 * scale


def test_backward_aliased_values_equal_gradients():
    """Psi holding Phi's values: the two gradients are equal."""
    rng = np.random.default_rng(14)
    phi = synth.random_orthonormal(64, 6, 41)
    idx = rng.choice(64, 18, replace=False)
    g = rng.uniform(0.5, 1.5, 64)
    bw = oracle.fit_backward(phi, phi.copy(), idx, g=g)
    assert np.linalg.norm(bw["dphi"] - bw["dpsi"]) <= 1e-12 * np.linalg.norm(bw["dphi"])


def test_kmeans_zero_weight_cluster_keeps_centroid():
    """A cluster whose members all have zero weight has no weighted mean
    (eq. r_k divides by zero): its centroid is kept and the cluster counted."""
    n = 6
    pts = oracle.grid_points(n)
    w = np.where(pts.sum(axis=1) < 7.5, 0.0, 1.0)  # zero exactly on seed 0's Voronoi cell
    c0 = np.array([[0.0, 0.0, 0.0], [5.0, 5.0, 5.0]])
    km = oracle.kmeans(n, w, c0, 1)
    assert np.array_equal(km["centroids"][0], c0[0])
    assert km["empty"] == 1
    assert km["idx"][0] == 0
    m = pts.sum(axis=1) > 7.5
    assert np.allclose(km["centroids"][1], pts[m].mean(axis=0), rtol=1e-14)


def test_fit_matches_hand_derived_golden(golden_theta):
    """Theta = Phi . conj(Psi) when the interpolation rows are the identity
    (derivation in tests/golden/theta_identity_rows.txt)."""
    for name, c in golden_theta.items():
        th = oracle.fit_theta(c["phi"], c["psi"], c["idx"])
        assert np.max(np.abs(th - c["theta"])) <= 1e-15, name


# --------------------------------------------------- V_mu (eq. V_mu, next step)
def _plane_wave(n, h, m):
    i, j, k = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    ph = 2 * np.pi * (m[0] * i / n[0] + m[1] * j / n[1] + m[2] * k / n[2])
    gsq = sum((2 * np.pi * m[a] / (n[a] * h[a])) ** 2 for a in range(3))
    return np.exp(1j * ph).reshape(-1), gsq


def test_poisson_plane_waves_closed_form():
    """A grid plane wave e^{iG.r} is an eigenfunction: V = 4 pi / |G|^2 e^{iG.r}
    (anisotropic grid and spacings; positive and negative frequencies)."""
    n, h = (6, 5, 8), (0.7, 1.1, 0.45)
    cols, expect = [], []
    for m in [(1, 0, 0), (0, -2, 1), (2, 2, -3), (-3, 1, 4)]:
        z, gsq = _plane_wave(n, h, m)
        cols.append(z)
        expect.append(4 * np.pi / gsq * z)
    V = oracle.poisson(np.stack(cols, axis=1), n, h)
    assert np.max(np.abs(V - np.stack(expect, axis=1))) <= 1e-12


def test_poisson_background_real_and_linear():
    """Constant fields have no potential (G = 0 dropped); real fields give
    real potentials equal to the real part of the complex transform; the
    map is linear."""
    rng = np.random.default_rng(51)
    n, h = (4, 6, 5), (1.0, 0.8, 1.3)
    nr = 4 * 6 * 5
    c = np.full((nr, 1), 3.0 + 1.0j)
    assert np.max(np.abs(oracle.poisson(c, n, h))) <= 1e-13
    x = rng.standard_normal((nr, 3))
    y = rng.standard_normal((nr, 3))
    vx = oracle.poisson(x, n, h)
    assert vx.dtype == np.float64
    vxy = oracle.poisson(x + 1j * y, n, h)
    assert np.max(np.abs(vxy.real - vx)) <= 1e-12 * np.max(np.abs(vx))
    assert np.max(np.abs(vxy - vx - 1j * oracle.poisson(y, n, h))) <= 1e-12 * np.max(np.abs(vxy))


def test_exchange_is_exact_when_every_point_interpolates():
    """N_mu = N_r (every grid point an interpolation point): ISDF is exact, so
    eq. v2 with V = poisson(Theta) equals the exact exchange of eq. v computed
    from explicit pair densities (complex Phi != Psi, anisotropic grid)."""
    rng = np.random.default_rng(71)
    n, h = (3, 2, 4), (0.9, 1.2, 0.7)
    nr = 24
    phi = rng.standard_normal((nr, 5)) + 1j * rng.standard_normal((nr, 5))
    psi = rng.standard_normal((nr, 6)) + 1j * rng.standard_normal((nr, 6))
    idx = np.arange(nr)
    theta = oracle.fit_theta(phi, psi, idx)
    v = oracle.poisson(theta, n, h)
    got = oracle.exchange(phi, psi, idx, v)
    ref = oracle.exchange_direct(phi, psi, n, h)
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


def test_exchange_real_orbitals_and_linearity():
    """Real orbitals give a real exchange; the map is linear in Psi."""
    rng = np.random.default_rng(72)
    n = (4, 3, 2)
    nr = 24
    phi = rng.standard_normal((nr, 4))
    idx = rng.choice(nr, 10, replace=False)
    theta = oracle.fit_theta(phi, phi, idx).real
    v = oracle.poisson(theta, n)
    x = oracle.exchange(phi, phi, idx, v)
    assert np.max(np.abs(x.imag)) <= 1e-14 * np.max(np.abs(x.real))
    psi2 = rng.standard_normal((nr, 3)) + 1j * rng.standard_normal((nr, 3))
    y = oracle.exchange(phi, psi2, idx, v)
    assert np.allclose(oracle.exchange(phi, 2j * psi2, idx, v), 2j * y, rtol=0, atol=1e-13 * np.abs(y).max())


# ------------------------------------------------------ QRCP points (eq. QRCP)
def _orth(rng, nr, n):
    return np.linalg.qr(crandn(rng, nr, n))[0]


@pytest.mark.parametrize("aliased", [True, False])
def test_qrcp_is_greedy_by_bruteforce(aliased):
    """eq. QRCP: every pivot has the largest residual column norm of Z^T after
    projecting out the earlier pivots (checked with an orthonormal basis of
    the chosen columns, not with R), and |R_kk| does not increase."""
    rng = np.random.default_rng(80 + aliased)
    phi = _orth(rng, 400, 5)
    psi = phi if aliased else _orth(rng, 400, 4)
    o = oracle.qrcp(phi, psi, 18)
    assert o["rank"] == 18
    ex = oracle.qrcp_greedy_excess(phi, psi, o["idx"])
    assert ex.max() <= 1e-12 and ex.min() >= -1e-12
    assert np.all(np.diff(o["rdiag"]) <= 1e-15 * o["rdiag"][0])
    assert len(set(o["idx"].tolist())) == 18
    # the Gram/Cholesky property check agrees on a greedy sequence
    c = oracle.qrcp_sampled_check(phi, psi, o["idx"], o["rdiag"], np.arange(400))
    assert c["rdiag_rel"] <= 1e-12 and c["greedy_excess"] <= 1e-12


def test_qrcp_checks_catch_a_wrong_pivot():
    """The two property checks fail on planted mistakes: two pivots swapped
    (brute force), and a pivot replaced by a lower-residual row with a
    self-consistent R diagonal (Gram check)."""
    rng = np.random.default_rng(82)
    phi, psi = _orth(rng, 300, 4), _orth(rng, 300, 5)
    o = oracle.qrcp(phi, psi, 12)
    bad = o["idx"].copy()
    bad[[2, 6]] = bad[[6, 2]]
    assert oracle.qrcp_greedy_excess(phi, psi, bad).max() > 1e-3
    bad = o["idx"].copy()
    bad[4] = np.setdiff1d(np.arange(300), bad)[0]
    kpp = oracle.hadamard(*oracle.gram_blocks(phi, psi, bad, rows=bad))
    rd = np.abs(np.diag(sla.cholesky(kpp, lower=True)))
    assert oracle.qrcp_sampled_check(phi, psi, bad, rd, np.arange(300))["greedy_excess"] > 1e-3


def test_qrcp_gap_by_explicit_projection():
    """gap[k] = (s_1 - s_2) / s_1 for the two largest squared norms of the
    columns of (I - P_k) Z^T, P_k the orthogonal projector on the first k
    pivot columns (formed from a least-squares solve, not from R)."""
    rng = np.random.default_rng(83)
    phi, psi = _orth(rng, 120, 3), _orth(rng, 120, 3)
    o = oracle.qrcp(phi, psi, 6)
    zt = oracle.explicit_z(phi, psi).T
    for k in range(6):
        if k == 0:
            res = zt
        else:
            b = zt[:, o["idx"][:k]]
            coef = np.linalg.lstsq(b, zt, rcond=None)[0]
            res = zt - b @ coef
        s = np.sort((np.abs(res) ** 2).sum(axis=0))[::-1]
        assert abs(s[0] - o["rdiag"][k] ** 2) <= 1e-12 * o["rdiag"][0] ** 2
        assert abs((s[0] - s[1]) / s[0] - o["gap"][k]) <= 1e-9


@pytest.mark.parametrize("n_phi,n_psi,real,rank", [(2, 2, False, 4), (2, 3, False, 6), (3, 3, True, 6)])
def test_qrcp_rank_closed_form_and_exact_fit(n_phi, n_psi, real, rank):
    """Z has N_phi N_psi columns of rank N_phi N_psi for generic complex
    orbitals, and N(N+1)/2 for real Phi = Psi (phi_i phi_j = phi_j phi_i).
    QRCP stops at that rank (eq. QRCP: R11 non-singular, the rest zero), and
    the fit at those points reproduces Z exactly (eq. decomposition)."""
    rng = np.random.default_rng(84 + n_psi)
    nr = 200
    if real:
        phi = np.linalg.qr(rng.standard_normal((nr, n_phi)))[0].astype(np.complex128)
        psi = phi
    else:
        phi = _orth(rng, nr, n_phi)
        psi = phi if n_psi == n_phi else _orth(rng, nr, n_psi)
    o = oracle.qrcp(phi, psi, rank + 3, rtol=1e-8)
    assert o["rank"] == rank
    assert np.all(o["idx"][rank:] == -1) and np.all(o["rdiag"][rank:] == 0)
    idx = o["idx"][:rank]
    theta = oracle.fit_theta(phi, psi, idx)
    z = oracle.explicit_z(phi, psi)
    assert np.linalg.norm(theta @ z[idx] - z) <= 1e-10 * np.linalg.norm(z)


def test_qrcp_single_orbital_pair():
    """N_phi = N_psi = 1: Z^T is one row, so the first pivot is the grid point
    of largest |phi||psi| and |R_00| is that value; the rank is 1."""
    rng = np.random.default_rng(86)
    phi = crandn(rng, 97, 1)
    psi = crandn(rng, 97, 1)
    o = oracle.qrcp(phi, psi, 3)
    m = np.abs(phi[:, 0]) * np.abs(psi[:, 0])
    assert o["rank"] == 1 and o["idx"][0] == np.argmax(m)
    assert abs(o["rdiag"][0] - m.max()) <= 1e-14 * m.max()


def test_qrcp_permutation_and_gauge_equivariant():
    """Relabelling grid points relabels the pivots; a unitary mixing of the
    orbitals (Phi U, Psi V) leaves Z Z^H and hence the pivots and |R_kk|
    unchanged (Sec. 2.1: Z only enters through its row space)."""
    rng = np.random.default_rng(87)
    nr = 350
    phi, psi = _orth(rng, nr, 4), _orth(rng, nr, 5)
    o = oracle.qrcp(phi, psi, 15)
    assert o["gap"].min() > 1e-8
    perm = rng.permutation(nr)
    op = oracle.qrcp(phi[perm], psi[perm], 15)
    inv = np.argsort(perm)
    assert np.array_equal(op["idx"], inv[o["idx"]])
    og = oracle.qrcp(phi @ haar_unitary(rng, 4), psi @ haar_unitary(rng, 5), 15)
    assert np.array_equal(og["idx"], o["idx"])
    assert np.allclose(og["rdiag"], o["rdiag"], rtol=1e-12, atol=0)


def _sketch_mats(rng, n_phi, n_psi, m):
    return rng.standard_normal((n_phi, m)), rng.standard_normal((n_psi, m))


def test_qrcp_sketch_is_hadamard_of_products():
    """(Z Omega)(r, k) = (Phi g_phi[:, k])(r) conj((Psi g_psi[:, k])(r)) for the
    Khatri-Rao Omega (explicit Z against the two thin products)."""
    rng = np.random.default_rng(90)
    phi, psi = _orth(rng, 60, 4), _orth(rng, 60, 5)
    gp, gs = _sketch_mats(rng, 4, 5, 11)
    y = oracle.explicit_z(phi, psi) @ oracle.khatri_rao_sketch(gp, gs)
    y2 = (phi @ gp) * np.conj(psi @ gs)
    assert np.max(np.abs(y - y2)) <= 1e-14 * np.max(np.abs(y))


def test_qrcp_sketch_orthogonal_kronecker_is_exact():
    """With m = N_phi N_psi and g_phi[:, (a, b)] = U[:, a], g_psi[:, (a, b)] = V[:, b]
    for orthogonal U, V, Omega = U (x) V is orthogonal: the sketch keeps every
    column norm and projection of Z^T, so its pivots and |R_kk| are those of
    the exact QRCP."""
    rng = np.random.default_rng(91)
    n_phi, n_psi = 3, 4
    phi, psi = _orth(rng, 150, n_phi), _orth(rng, 150, n_psi)
    u = np.linalg.qr(rng.standard_normal((n_phi, n_phi)))[0]
    v = np.linalg.qr(rng.standard_normal((n_psi, n_psi)))[0]
    gp = np.repeat(u, n_psi, axis=1)          # column (a, b) -> U[:, a]
    gs = np.tile(v, (1, n_phi))               # column (a, b) -> V[:, b]
    om = oracle.khatri_rao_sketch(gp, gs)
    assert np.allclose(om.T @ om, np.eye(n_phi * n_psi), atol=1e-13)
    ex = oracle.qrcp(phi, psi, 10)
    sk = oracle.qrcp_sketch(phi, psi, 10, gp, gs)
    assert ex["gap"].min() > 1e-8
    assert np.array_equal(sk["idx"], ex["idx"])
    assert np.allclose(sk["rdiag"], ex["rdiag"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("aliased", [True, False])
def test_qrcp_sketch_is_greedy_on_the_sketch(aliased):
    """The sketch pivots are greedy on (Z Omega)^T (brute force), rank is
    capped by m, and they differ from the exact pivots only through Omega."""
    rng = np.random.default_rng(92 + aliased)
    phi = _orth(rng, 300, 5)
    psi = phi if aliased else _orth(rng, 300, 4)
    gp, gs = _sketch_mats(rng, 5, psi.shape[1], 14)
    sk = oracle.qrcp_sketch(phi, psi, 18, gp, gs, rtol=1e-10)
    assert sk["rank"] == 14 and np.all(sk["idx"][14:] == -1)
    ex = oracle.qrcp_greedy_excess(phi, psi, sk["idx"][:14], gp, gs)
    assert ex.max() <= 1e-12 and ex.min() >= -1e-12
