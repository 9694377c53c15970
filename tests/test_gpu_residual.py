"""GPU parity of the two Z-free residuals against the FP64 oracle:
isdf_fit_residual (||Z - Theta C||^2 and ||Z||^2) and isdf_cluster_residual
(Appendix A's R for given clusters and interpolation points)."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

isdf = pytest.importorskip("paper_2208_07731_amd")


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def water8_km(water8):
    phi = water8["phi"]
    wl = water8["wl"]
    km = oracle.kmeans(wl.n, oracle.weight(phi, phi), water8["c0"], wl.kmeans_iters)
    return km


def rho2(phi, psi):
    rp = (np.abs(phi) ** 2).sum(axis=1)
    rs = (np.abs(psi) ** 2).sum(axis=1)
    return float(np.dot(rp, rs))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "fp16x3"])
def test_fit_residual_water8(water8, water8_km, prec):
    phi = water8["phi"]
    idx = water8_km["idx"].astype(np.int32)
    ref = oracle.fit_residual(phi, phi, idx)
    z2 = rho2(phi, phi)
    p, i = dev(phi), dev(idx)
    _, minv, _ = isdf.fit(p, None, i, nrows=0, prec=prec)
    res, zz = isdf.fit_residual(p, None, i, minv, prec=prec, rblock=5000)
    print(f"{prec}: residual {res:.12e} oracle {ref:.12e} (||Z||^2 {z2:.6e})")
    assert abs(zz - z2) <= 1e-13 * z2
    assert abs(res - ref) <= (1e-12 if prec == "fp64" else 1e-6) * z2


def test_fit_residual_complex_blocks():
    rng = np.random.default_rng(41)
    nr, n_phi, n_psi, n_mu = 5 * 6 * 7, 7, 9, 37
    big = rng.standard_normal((nr, 20)) + 1j * rng.standard_normal((nr, 20))
    idx = rng.choice(nr, n_mu, replace=False).astype(np.int32)
    phi, psi = big[:, :n_phi], big[:, n_phi:n_phi + n_psi]
    ref = oracle.fit_residual(phi, psi, idx)
    t = dev(big)
    _, minv, _ = isdf.fit(t[:, :n_phi], t[:, n_phi:n_phi + n_psi], dev(idx), grid=(5, 6, 7), nrows=0)
    res, zz = isdf.fit_residual(t[:, :n_phi], t[:, n_phi:n_phi + n_psi], dev(idx), minv, grid=(5, 6, 7), rblock=64)
    z2 = rho2(phi, psi)
    assert abs(zz - z2) <= 1e-13 * z2
    assert abs(res - ref) <= 1e-11 * z2


def test_residuals_vanish_when_every_point_interpolates():
    """N_mu = N_r: Theta C reproduces Z and every row is its own projection."""
    rng = np.random.default_rng(42)
    nr = 24
    x = rng.standard_normal((nr, 6)) + 1j * rng.standard_normal((nr, 6))
    idx = np.arange(nr, dtype=np.int32)
    p, i = dev(x), dev(idx)
    _, minv, _ = isdf.fit(p, None, i, grid=(nr, 1, 1), nrows=0)
    res, zz = isdf.fit_residual(p, None, i, minv, grid=(nr, 1, 1))
    assert abs(res) <= 1e-10 * zz
    R = isdf.cluster_residual(p, None, i, i, grid=(nr, 1, 1))
    assert abs(R) <= 1e-12 * zz


def test_cluster_residual_water8(water8, water8_km):
    phi = water8["phi"]
    km = water8_km
    ref = oracle.cluster_residual(phi, phi, km["labels"], km["idx"])
    got = isdf.cluster_residual(dev(phi), None, dev(km["labels"].astype(np.int32)), dev(km["idx"].astype(np.int32)))
    assert abs(got - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cluster_residual_complex_general(dtype):
    rng = np.random.default_rng(43)
    n = 6
    big = rng.standard_normal((n ** 3, 12)) + 1j * rng.standard_normal((n ** 3, 12))
    if dtype == "c64":
        big = big.astype(np.complex64)
    phi, psi = big[:, :5], big[:, 5:12]
    phi64, psi64 = phi.astype(np.complex128), psi.astype(np.complex128)
    c0 = oracle.grid_points(n)[rng.choice(n ** 3, 10, replace=False)]
    km = oracle.kmeans(n, oracle.weight(phi64, psi64), c0, 6)
    ref = oracle.cluster_residual(phi64, psi64, km["labels"], km["idx"])
    t = dev(big)
    got = isdf.cluster_residual(t[:, :5], t[:, 5:12], dev(km["labels"].astype(np.int32)),
                                dev(km["idx"].astype(np.int32)), grid=n)
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_cluster_residual_counts_invalid_labels():
    rng = np.random.default_rng(44)
    n = 4
    x = rng.standard_normal((n ** 3, 3)) + 1j * rng.standard_normal((n ** 3, 3))
    labels = np.zeros(n ** 3, dtype=np.int32)
    labels[[3, 9]] = [-1, 7]  # outside [0, n_mu) for n_mu = 2
    idx = np.array([0, 5], dtype=np.int32)
    with pytest.raises(ValueError, match="2 rows"):
        isdf.cluster_residual(dev(x), None, dev(labels), dev(idx), grid=n)
