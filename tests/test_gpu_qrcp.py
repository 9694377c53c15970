"""GPU parity of isdf_qrcp (interpolation points by QR with column pivoting
of Z^T, eq. QRCP) against the FP64 oracle, which factors an explicit Z^T
with LAPACK's pivoted Householder QR.

Pivots are compared exactly up to the first step whose decision margin is
within rounding of both methods; later pivots (and full-size runs) are
checked for validity: the greedy rule by brute force on explicit Z, or at
sampled rows through the Gram matrix at any size.

Tolerance of the squared diagonal |R_kk|^2: the library accumulates it as
K_rr - sum_{j<k} |L_rj|^2 with every term at most |R_00|^2, so its rounding
error is about k eps |R_00|^2; the bar is 64 k eps |R_00|^2.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

isdf = pytest.importorskip("paper_2208_07731_amd")

EPS = np.finfo(np.float64).eps


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def first_near_tie(o, n):
    """First step whose margin s_1 - s_2 is below 1e-9 s_0 (oracle's own R)."""
    s = o["rdiag"][:n] ** 2
    near = np.nonzero(o["gap"][:n] * s <= 1e-9 * s[0])[0]
    return int(near[0]) if near.size else n


def check_against_oracle(phi, psi, r, o, n_mu, greedy_bruteforce=True):
    idx = r.idx.cpu().numpy()
    rd = r.rdiag.cpu().numpy()
    rank = r.info["rank"]
    assert rank == o["rank"]
    kstar = first_near_tie(o, rank)
    np.testing.assert_array_equal(idx[:kstar], o["idx"][:kstar])
    tol = 64 * max(rank, 1) * EPS * o["rdiag"][0] ** 2
    assert np.max(np.abs(rd[:rank] ** 2 - o["rdiag"][:rank] ** 2)) <= tol
    assert np.all(idx[rank:] == -1) and np.all(rd[rank:] == 0)
    assert len(set(idx[:rank].tolist())) == rank
    if kstar < rank and greedy_bruteforce:
        # past a near tie: the library's own order must still be greedy
        ex = oracle.qrcp_greedy_excess(phi, psi, idx[:rank])
        assert ex.max() <= 1e-9
    return kstar


def test_qrcp_water8_aliased(water8):
    """8-water box (N_r = 13824, N_e = 32, Psi = Phi), N_mu = 256."""
    phi = water8["phi"]
    n_mu = water8["wl"].n_mu
    o = oracle.qrcp(phi, phi, n_mu)
    p = dev(phi)
    r = isdf.qrcp(p, None, n_mu, grid=water8["wl"].n)
    kstar = check_against_oracle(phi, phi, r, o, n_mu)
    print(f"water8: pivots equal up to step {kstar} of {n_mu}, near ties {r.info['near_ties']}")
    # gaps agree with the oracle's margins where they are resolved
    g = r.gap.cpu().numpy()[:kstar]
    s0 = o["rdiag"][0] ** 2
    assert np.all(np.abs(g - o["gap"][:kstar]) * o["rdiag"][:kstar] ** 2 <= 1e-10 * s0)
    assert abs(r.info["r00"] - o["rdiag"][0]) <= 1e-13 * o["rdiag"][0]


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_qrcp_complex_ragged_grid(dtype):
    """Psi != Phi (complex Gram), grid 10 x 11 x 13 (a ragged last tile),
    N_phi = 7, N_psi = 9, N_mu = 50; complex64 storage is compared with the
    oracle on the same (widened) values."""
    phi = synth.random_orthonormal(1430, 7, 11).astype(dtype)
    psi = synth.random_orthonormal(1430, 9, 12).astype(dtype)
    o = oracle.qrcp(phi.astype(np.complex128), psi.astype(np.complex128), 50)
    r = isdf.qrcp(dev(phi), dev(psi), 50, grid=(10, 11, 13))
    check_against_oracle(phi.astype(np.complex128), psi.astype(np.complex128), r, o, 50)


def test_qrcp_rank_deficient_stops():
    """N_phi = N_psi = 2 complex, Psi = Phi: Z has rank 4, so asking for 9
    pivots returns 4 and fills the rest with -1 / 0."""
    phi = synth.random_orthonormal(500, 2, 13)
    o = oracle.qrcp(phi, phi, 9, rtol=1e-6)
    r = isdf.qrcp(dev(phi), None, 9, rtol=1e-6)
    assert o["rank"] == 4
    check_against_oracle(phi, phi, r, o, 9)


def test_qrcp_single_pair_and_one_pivot():
    """N_phi = N_psi = 1: the first pivot is argmax |phi||psi| and the rank
    is 1; n_mu = 1 returns that pivot alone."""
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((333, 1)) + 1j * rng.standard_normal((333, 1))
    psi = rng.standard_normal((333, 1)) + 1j * rng.standard_normal((333, 1))
    m = np.abs(phi[:, 0]) * np.abs(psi[:, 0])
    r = isdf.qrcp(dev(phi), dev(psi), 3, rtol=1e-6)
    assert r.info["rank"] == 1
    assert r.idx.cpu().tolist() == [int(np.argmax(m)), -1, -1]
    assert abs(r.rdiag[0].item() - m.max()) <= 1e-14 * m.max()
    r1 = isdf.qrcp(dev(phi), dev(psi), 1)
    assert r1.idx.cpu().tolist() == [int(np.argmax(m))] and r1.info["rank"] == 1


def test_qrcp_deterministic_and_nonfinite(water8):
    phi = water8["phi"]
    p = dev(phi)
    a = isdf.qrcp(p, None, 64)
    b = isdf.qrcp(p, None, 64)
    assert torch.equal(a.idx, b.idx) and torch.equal(a.rdiag, b.rdiag) and torch.equal(a.gap, b.gap)
    x = phi.copy()
    x[1234, 3] = np.nan
    with pytest.raises(isdf.ISDFError) as e:
        isdf.qrcp(dev(x), None, 8)
    assert e.value.code == 2


def test_qrcp_water64_sampled_properties():
    """Full-size 64-water box (N_r = 262144, N_e = 256, N_mu = 2048): the
    |R_kk| sequence equals the Cholesky diagonal of Z Z^H at the returned
    points, and the greedy rule holds at 2048 sampled grid rows."""
    d = synth.make_workload("water64")
    wl = d["wl"]
    phi = d["phi"]
    r = isdf.qrcp(dev(phi), None, wl.n_mu, grid=wl.n)
    assert r.info["rank"] == wl.n_mu
    idx = r.idx.cpu().numpy()
    rd = r.rdiag.cpu().numpy()
    assert len(set(idx.tolist())) == wl.n_mu and idx.min() >= 0
    rows = np.random.default_rng(64).choice(phi.shape[0], 2048, replace=False)
    c = oracle.qrcp_sampled_check(phi, phi, idx, rd, rows)
    print(f"water64: rdiag err {c['rdiag_rel']:.2e}, greedy excess {c['greedy_excess']:.2e}, "
          f"|R_last|/|R_00| {rd[-1] / rd[0]:.3e}, near ties {r.info['near_ties']}")
    assert c["rdiag_rel"] <= 64 * wl.n_mu * EPS
    assert c["greedy_excess"] <= 64 * wl.n_mu * EPS


def sketch_inputs(seed, n_phi, n_psi, m):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_phi, m)), rng.standard_normal((n_psi, m))


def test_qrcp_sketch_water8_aliased(water8):
    """Randomized QRCP on the 8-water box (Psi = Phi), m = N_mu + 8, against
    the oracle's pivoted QR of the explicit sketch (Z Omega)^T on the same
    random matrices."""
    phi = water8["phi"]
    n_mu = water8["wl"].n_mu
    gp, gs = sketch_inputs(101, 32, 32, n_mu + 8)
    o = oracle.qrcp_sketch(phi, phi, n_mu, gp, gs)
    p = dev(phi)
    r = isdf.qrcp(p, None, n_mu, grid=water8["wl"].n, sketch=(dev(gp), dev(gs)))
    kstar = check_against_oracle(phi, phi, r, o, n_mu, greedy_bruteforce=False)
    if kstar < r.info["rank"]:
        ex = oracle.qrcp_greedy_excess(phi, phi, r.idx.cpu().numpy()[: r.info["rank"]], gp, gs)
        assert ex.max() <= 1e-9
    print(f"water8 sketch: pivots equal up to step {kstar} of {n_mu}")


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_qrcp_sketch_complex_ragged(dtype):
    """Psi != Phi, ragged grid, m = 40 sketch rows for 30 pivots; complex64
    storage against the oracle on the widened values."""
    phi = synth.random_orthonormal(1430, 7, 21).astype(dtype)
    psi = synth.random_orthonormal(1430, 9, 22).astype(dtype)
    gp, gs = sketch_inputs(102, 7, 9, 40)
    p64, s64 = phi.astype(np.complex128), psi.astype(np.complex128)
    o = oracle.qrcp_sketch(p64, s64, 30, gp, gs)
    r = isdf.qrcp(dev(phi), dev(psi), 30, grid=(10, 11, 13), sketch=(dev(gp), dev(gs)))
    kstar = check_against_oracle(p64, s64, r, o, 30, greedy_bruteforce=False)
    if kstar < r.info["rank"]:
        assert oracle.qrcp_greedy_excess(p64, s64, r.idx.cpu().numpy()[: r.info["rank"]], gp, gs).max() <= 1e-9


def test_qrcp_sketch_rank_is_capped_by_m():
    """At most m pivots exist: asking for more returns rank m and -1 after."""
    phi = synth.random_orthonormal(500, 6, 23)
    gp, gs = sketch_inputs(103, 6, 6, 12)
    r = isdf.qrcp(dev(phi), None, 16, rtol=1e-6, sketch=(dev(gp), dev(gs)))
    assert r.info["rank"] == 12
    assert (r.idx.cpu().numpy()[12:] == -1).all()


def test_qrcp_sketch_orthogonal_kronecker_equals_exact():
    """Omega = U (x) V with orthogonal U, V (m = N_phi N_psi) keeps every
    column norm of Z^T: the randomized pivots equal the exact ones."""
    rng = np.random.default_rng(104)
    phi = synth.random_orthonormal(800, 3, 24)
    psi = synth.random_orthonormal(800, 4, 25)
    u = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    v = np.linalg.qr(rng.standard_normal((4, 4)))[0]
    gp = np.repeat(u, 4, axis=1)
    gs = np.tile(v, (1, 3))
    ex = isdf.qrcp(dev(phi), dev(psi), 10)
    sk = isdf.qrcp(dev(phi), dev(psi), 10, sketch=(dev(gp), dev(gs)))
    o = oracle.qrcp(phi, psi, 10)
    assert o["gap"].min() > 1e-8
    assert torch.equal(ex.idx, sk.idx)
    np.testing.assert_allclose(sk.rdiag.cpu().numpy(), ex.rdiag.cpu().numpy(), rtol=1e-10)


def test_qrcp_sketch_wider_than_lds():
    """m = 3500 sketch columns: the pivot's sketch row (56 KB) is read in
    place rather than staged in LDS, so m has no upper limit; Psi != Phi on
    a 12^3 grid, 30 pivots, against the oracle on the explicit sketch."""
    phi = synth.random_orthonormal(1728, 6, 31)
    psi = synth.random_orthonormal(1728, 7, 32)
    gp, gs = sketch_inputs(105, 6, 7, 3500)
    o = oracle.qrcp_sketch(phi, psi, 30, gp, gs)
    r = isdf.qrcp(dev(phi), dev(psi), 30, grid=(12, 12, 12), sketch=(dev(gp), dev(gs)))
    kstar = check_against_oracle(phi, psi, r, o, 30, greedy_bruteforce=False)
    if kstar < r.info["rank"]:
        assert oracle.qrcp_greedy_excess(phi, psi, r.idx.cpu().numpy()[: r.info["rank"]], gp, gs).max() <= 1e-9
