"""GPU parity of isdf_exchange (ISDF-compressed exchange, eq. v2) against the
FP64 oracle, alone and chained after the fit and V_mu."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

isdf = pytest.importorskip("paper_2208_07731_amd")

EPS = np.finfo(np.float64).eps


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def water8_x(water8):
    phi = water8["phi"]
    wl = water8["wl"]
    idx = oracle.kmeans(wl.n, oracle.weight(phi, phi), water8["c0"], wl.kmeans_iters)["idx"]
    th = np.ascontiguousarray(oracle.fit_theta(phi, phi, idx).real)
    h = wl.box_angstrom / 0.529177 / wl.n
    v = oracle.poisson(th, wl.n, (h, h, h))
    return dict(phi=phi, wl=wl, idx=idx.astype(np.int32), th=th, v=v, h=h,
                ref=oracle.exchange(phi, phi, idx, v))


@pytest.mark.parametrize("rblock", [None, 5000])
def test_exchange_water8_given_potentials(water8_x, rblock):
    x = water8_x
    W = isdf.exchange(dev(x["phi"]), dev(x["phi"]), dev(x["idx"]), dev(x["v"]), rblock=rblock)
    assert rel(W.cpu().numpy(), x["ref"]) <= 1e-13


def test_exchange_complex_ragged_blocks():
    rng = np.random.default_rng(81)
    n = (5, 6, 7)
    nr = 210
    big = rng.standard_normal((nr, 20)) + 1j * rng.standard_normal((nr, 20))
    phi, psi = big[:, :7], big[:, 7:16]
    idx = rng.choice(nr, 37, replace=False).astype(np.int32)
    v = oracle.poisson(oracle.fit_theta(phi, psi, idx), n)
    ref = oracle.exchange(phi, psi, idx, v)
    t = dev(big)
    W = isdf.exchange(t[:, :7], t[:, 7:16], dev(idx), dev(v), grid=n, rblock=64)
    assert rel(W.cpu().numpy(), ref) <= 1e-13
    # complex64 storage: FP64 arithmetic on the rounded inputs
    t32 = dev(big.astype(np.complex64))
    W32 = isdf.exchange(t32[:, :7], t32[:, 7:16], dev(idx), dev(v.astype(np.complex64)), grid=n)
    assert W32.dtype == torch.complex64
    assert rel(W32.cpu().numpy().astype(np.complex128), ref) <= 1e-5


def test_exchange_chain_water8(water8_x):
    """Fit, V_mu and the exchange all on the GPU against the oracle chain."""
    x = water8_x
    p, i = dev(x["phi"]), dev(x["idx"])
    theta, _, _ = isdf.fit(p, None, i)
    V = isdf.poisson(theta, x["wl"].n, (x["h"],) * 3)
    W = isdf.exchange(p, p, i, V)
    kappa = oracle.cc_condition(x["phi"], x["phi"], x["idx"])
    err = rel(W.cpu().numpy(), x["ref"])
    print(f"water8 exchange chain rel err {err:.3e} (kappa {kappa:.2e})")
    assert err <= 1e-12


def test_exchange_chain_exact_when_every_point_interpolates():
    """N_mu = N_r: the GPU chain reproduces the exact exchange of eq. v."""
    rng = np.random.default_rng(82)
    n, h = (3, 2, 4), (0.9, 1.2, 0.7)
    nr = 24
    phi = rng.standard_normal((nr, 5)) + 1j * rng.standard_normal((nr, 5))
    psi = rng.standard_normal((nr, 6)) + 1j * rng.standard_normal((nr, 6))
    idx = np.arange(nr, dtype=np.int32)
    p, q, i = dev(phi), dev(psi), dev(idx)
    theta, _, _ = isdf.fit(p, q, i, grid=n)
    V = isdf.poisson(theta, n, h)
    W = isdf.exchange(p, q, i, V, grid=n)
    assert rel(W.cpu().numpy(), oracle.exchange_direct(phi, psi, n, h)) <= 1e-9


def test_exchange_water64_sampled_rows():
    """Full-size 64-water exchange (N_r = 262144, N_e = 256, N_mu = 2048,
    r-blocks of 65536) with seeded real potentials: W at 256 sampled rows
    against the oracle (each row of W depends on its own row of Phi and V
    and on Phi_mu, Psi_mu only)."""
    import synth

    d = synth.make_workload("water64")
    wl = d["wl"]
    phi = d["phi"]
    rng = np.random.default_rng(6401)
    idx = np.sort(rng.choice(wl.n_r, wl.n_mu, replace=False)).astype(np.int32)
    v = rng.standard_normal((wl.n_r, wl.n_mu))
    rows = np.sort(rng.choice(wl.n_r, 256, replace=False))
    p = dev(phi)
    W = isdf.exchange(p, p, dev(idx), dev(v))
    got = W[torch.as_tensor(rows).cuda()].cpu().numpy()
    del W
    sub = np.concatenate([idx, rows])
    phi_sub = np.ascontiguousarray(phi[sub])
    ref = oracle.exchange(phi_sub, phi_sub, np.arange(wl.n_mu), v[sub])[wl.n_mu:]
    err = rel(got, ref)
    print(f"water64 exchange rows rel err {err:.3e}")
    assert err <= 1e-13
