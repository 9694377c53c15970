"""GPU parity of isdf_fit (Gram + Hadamard on MFMA, FP64 Cholesky / inverse,
Theta) against the FP64 oracle, through the C ABI."""
import time

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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def water8_fit(water8):
    phi = water8["phi"]
    wl = water8["wl"]
    w = oracle.weight(phi, phi)
    idx = oracle.kmeans(wl.n, w, water8["c0"], wl.kmeans_iters)["idx"]
    ref = oracle.fit(phi, phi, idx)
    kappa = oracle.cc_condition(phi, phi, idx)
    return dict(phi=phi, idx=idx, ref=ref, kappa=kappa, wl=wl)


# Parity bars (relative Frobenius norm against the FP64 oracle).  FP64:
# Theta within 1e-12 and gradients within 1e-11 whatever the conditioning of
# C C^H (measured errors are 1e-15 .. 1e-14 at every size); orbital
# contractions in FP32 or a split precision: Theta within 1e-6, gradients
# within 1e-5.  kappa(C C^H) is printed as a diagnostic only.
FP64_THETA = 1e-12
FP64_GRAD = 1e-11
MIXED_THETA = 1e-6
MIXED_GRAD = 1e-5


def test_fit_fp64_water8(water8_fit):
    f = water8_fit
    theta, minv, info = isdf.fit(dev(f["phi"]), None, dev(f["idx"].astype(np.int32)))
    th = theta.cpu().numpy()
    assert th.dtype == np.float64
    err = rel(th, f["ref"]["theta"].real)
    print(f"water8 fp64 theta rel err {err:.3e} (kappa {f['kappa']:.2e})")
    assert err <= FP64_THETA
    assert info["status"] == 0 and info["pivot"] == -1
    # minv against the oracle's inverse of C C^H
    M = f["ref"]["M"].real
    W = minv.cpu().numpy().reshape(M.shape)
    assert rel(W @ M, np.eye(M.shape[0])) <= 1e2 * f["kappa"] * EPS
    # interpolation property Theta(r_mu) = I
    assert np.max(np.abs(th[f["idx"]] - np.eye(len(f["idx"])))) <= 10 * f["kappa"] * EPS
    # pivots of the factorisation bound the spectrum of C C^H
    ev = np.linalg.eigvalsh(M)
    assert ev[0] * (1 - 1e-8) <= info["pivot_min"] and info["pivot_max"] <= ev[-1] * (1 + 1e-8)


def test_fit_rblocks_bitwise(water8_fit):
    """Rows are independent given minv: any partition of the rows into calls
    and internal r-blocks gives bitwise equal Theta."""
    f = water8_fit
    phi, idx = dev(f["phi"]), dev(f["idx"].astype(np.int32))
    full, minv, _ = isdf.fit(phi, None, idx)
    a, _, _ = isdf.fit(phi, None, idx, minv=minv, factor=False, row0=0, nrows=5000, rblock=1234)
    b, _, _ = isdf.fit(phi, None, idx, minv=minv, factor=False, row0=5000, nrows=full.shape[0] - 5000, rblock=777)
    assert torch.equal(torch.cat([a, b]), full)


def tiny_complex(seed, n=(5, 6, 7), n_phi=7, n_psi=9, n_mu=37, ld_pad=3):
    rng = np.random.default_rng(seed)
    nr = n[0] * n[1] * n[2]
    big = rng.standard_normal((nr, n_phi + n_psi + ld_pad)) + 1j * rng.standard_normal((nr, n_phi + n_psi + ld_pad))
    idx = rng.choice(nr, n_mu, replace=False).astype(np.int32)
    return big, idx


def test_fit_fp64_complex_ragged():
    """Psi != Phi, strided operands (shared storage), odd orbital counts, N_r
    and N_mu ragged against the 128-row / 16-column tiles."""
    big, idx = tiny_complex(5)
    t = dev(big)
    phi_t, psi_t = t[:, :7], t[:, 7:16]
    theta, _, info = isdf.fit(phi_t, psi_t, dev(idx), grid=(5, 6, 7))
    ref = oracle.fit(big[:, :7], big[:, 7:16], idx)
    kappa = oracle.cc_condition(big[:, :7], big[:, 7:16], idx)
    th = theta.cpu().numpy()
    assert th.dtype == np.complex128
    err = rel(th, ref["theta"])
    print(f"complex ragged fp64 theta rel err {err:.3e} (kappa {kappa:.2e})")
    assert err <= FP64_THETA


def test_fit_fp64_complex_swap_conjugates():
    big, idx = tiny_complex(6)
    t = dev(big)
    a, _, _ = isdf.fit(t[:, :7], t[:, 7:16], dev(idx), grid=(5, 6, 7))
    b, _, _ = isdf.fit(t[:, 7:16], t[:, :7], dev(idx), grid=(5, 6, 7))
    assert rel(b.cpu().numpy(), a.cpu().numpy().conj()) <= 1e-11


def test_fit_matches_hand_derived_golden(golden_theta):
    """Hand-derived Theta (identity interpolation rows) through the C ABI, in
    FP64 and the split precisions (whose parts represent these small integers
    exactly)."""
    for name, c in golden_theta.items():
        for prec in ("fp64", "fp32", "bf16x6", "fp16x3"):
            t = dev(np.concatenate([c["phi"], c["psi"]], axis=1))
            phi_t = t[:, :2]
            psi_t = phi_t if name == "aliased" else t[:, 2:]
            th, _, info = isdf.fit(phi_t, psi_t, dev(c["idx"]), grid=(4, 1, 1), prec=prec)
            got = th.cpu().numpy()
            ref = c["theta"].real if name == "aliased" else c["theta"]
            assert np.max(np.abs(got - ref)) <= 1e-14, (name, prec)


@pytest.fixture(scope="module")
def water64_case():
    """64-water workload (64^3 grid, N_e = 256, Psi = Phi, N_mu = 2048),
    seeded interpolation points and 256 sampled rows with their oracle
    Theta."""
    d = synth.make_workload("water64")
    wl = d["wl"]
    rng = np.random.default_rng(31)
    idx = synth.init_centroids(d["env"] ** 2, wl.n, wl.n_mu, 3031)
    idx = ((idx[:, 0] * wl.n + idx[:, 1]) * wl.n + idx[:, 2]).astype(np.int32)
    rows = np.sort(rng.choice(wl.n_r, 256, replace=False))
    ref = oracle.fit(d["phi"], d["phi"], idx, rows=rows)
    kappa = oracle.cc_condition(d["phi"], d["phi"], idx)
    return dict(d=d, wl=wl, idx=idx, rows=rows, ref=ref, kappa=kappa)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "fp16x3"])
def test_fit_water64_sampled_rows(water64_case, prec):
    """Full-size 64-water fit (the benchmark's shape, whole grid in one
    block): sampled rows of the real Theta against the oracle, FP64 to
    1e-12 and the lower orbital precisions to 1e-6."""
    c = water64_case
    theta, _, info = isdf.fit(dev(c["d"]["phi"]), None, dev(c["idx"]), prec=prec)
    got = theta[torch.as_tensor(c["rows"]).cuda()].cpu().numpy()
    err = rel(got, c["ref"]["theta"].real)
    print(f"water64 {prec} theta rel err {err:.3e} (kappa {c['kappa']:.2e})")
    assert err <= (FP64_THETA if prec == "fp64" else MIXED_THETA)
    assert info["status"] == 0


@pytest.mark.parametrize("prec", ["fp64", "bf16x6"])
def test_fit_backward_water64_gradient_rows(water64_case, prec):
    """Full-size 64-water fused-loss adjoint (the benchmark's shape and
    field g, whole grid in one block): gradient rows of Phi at the sampled
    non-interpolation points against the oracle's sub-problem."""
    c = water64_case
    d, wl = c["d"], c["wl"]
    sample = np.setdiff1d(c["rows"], c["idx"])
    phi_t = dev(d["phi"])
    idx_t = dev(c["idx"])
    g = d["g"]
    _, minv, _ = isdf.fit(phi_t, None, idx_t, nrows=0)
    dphi, _, loss, info = isdf.fit_backward(phi_t, None, idx_t, minv, g=dev(g), prec=prec)
    got = dphi[torch.as_tensor(sample).cuda()].cpu().numpy()
    del dphi
    sub = np.concatenate([c["idx"], sample])
    phi_sub = np.ascontiguousarray(d["phi"][sub])
    ref = oracle.fit_backward(phi_sub, phi_sub, np.arange(wl.n_mu), g=g[sub])
    err = rel(got, ref["dphi"][wl.n_mu:])
    tol = FP64_GRAD if prec == "fp64" else MIXED_GRAD
    print(f"water64 {prec} adjoint rows: dphi {err:.3e} (tol {tol:.1e}, {sample.size} rows)")
    assert err <= tol
    assert info["status"] == 0 and np.isfinite(loss.item()) and loss.item() > 0


@pytest.fixture(scope="module")
def water64_full_adjoint(water64_case):
    """The oracle's adjoint of the fused loss over the whole 64-water grid
    (262144 rows; about 100 GB of host memory at its peak), kept only at the
    interpolation rows and the sampled rows."""
    c = water64_case
    d = c["d"]
    rows = np.concatenate([c["idx"], np.setdiff1d(c["rows"], c["idx"])])
    print("[oracle] 64-water adjoint over the whole grid", flush=True)
    t0 = time.time()
    ref = oracle.fit_backward(d["phi"], d["phi"], c["idx"], g=d["g"])
    print(f"[oracle] done in {time.time() - t0:.1f} s", flush=True)
    out = dict(rows=rows, dphi=ref["dphi"][rows].copy(), loss=ref["loss"])
    del ref
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp16x3"])
def test_fit_backward_water64_interpolation_rows(water64_case, water64_full_adjoint, prec):
    """Full-size 64-water fused-loss adjoint against the oracle's adjoint over
    the whole grid: the gradient at all 2048 interpolation points, which
    carries Mbar = -Theta^H S (the split-K H = G^T diag(g) G over all 262144
    rows at the split factor this shape selects) and the scatter of
    Abar^H Phi, and at the sampled other rows; the loss."""
    c, ref = water64_case, water64_full_adjoint
    d, wl = c["d"], c["wl"]
    phi_t, idx_t = dev(d["phi"]), dev(c["idx"])
    _, minv, _ = isdf.fit(phi_t, None, idx_t, nrows=0, prec=prec)
    dphi, _, loss, info = isdf.fit_backward(phi_t, None, idx_t, minv, g=dev(d["g"]), prec=prec)
    got = dphi[torch.as_tensor(ref["rows"]).cuda()].cpu().numpy()
    del dphi
    e_idx = rel(got[: wl.n_mu], ref["dphi"][: wl.n_mu])
    e_all = rel(got, ref["dphi"])
    e_loss = abs(loss.item() - ref["loss"]) / ref["loss"]
    tol = FP64_GRAD if prec == "fp64" else MIXED_GRAD
    print(f"water64 {prec} adjoint: interpolation rows {e_idx:.3e}, with sampled rows {e_all:.3e}, "
          f"loss {e_loss:.3e} (kappa {c['kappa']:.2e})")
    assert e_idx <= tol and e_all <= tol and e_loss <= tol
    assert info["status"] == 0


@pytest.fixture(scope="module")
def sio2_case():
    """SiO2-like workload (72^3 grid, N_phi = 192, N_psi = 384 sharing the
    first 192 columns, N_mu = 3072, complex), seeded interpolation points and
    256 sampled rows with their oracle Theta."""
    d = synth.make_workload("sio2")
    wl = d["wl"]
    rng = np.random.default_rng(30)
    idx = synth.init_centroids(d["env"] ** 2, wl.n, wl.n_mu, 3030)
    idx = ((idx[:, 0] * wl.n + idx[:, 1]) * wl.n + idx[:, 2]).astype(np.int32)
    rows = np.sort(rng.choice(wl.n_r, 256, replace=False))
    ref = oracle.fit(d["phi"], d["psi"], idx, rows=rows)
    kappa = oracle.cc_condition(d["phi"], d["psi"], idx)
    return dict(d=d, wl=wl, idx=idx, rows=rows, ref=ref, kappa=kappa)


def test_fit_sio2_shape_sampled_rows(sio2_case):
    """Full-size SiO2 fit in FP64, r-blocks of 65536: sampled rows of Theta
    against the oracle."""
    c = sio2_case
    psi_t = dev(c["d"]["psi"])
    phi_t = psi_t[:, : c["wl"].n_phi]
    theta, _, info = isdf.fit(phi_t, psi_t, dev(c["idx"]), rblock=65536)
    got = theta[torch.as_tensor(c["rows"]).cuda()].cpu().numpy()
    err = rel(got, c["ref"]["theta"])
    print(f"sio2 fp64 theta rel err {err:.3e} (kappa {c['kappa']:.2e})")
    assert err <= FP64_THETA


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6", "fp16x3"])
def test_fit_backward_sio2_gradient_rows(sio2_case, prec):
    """Full-size SiO2 adjoint (Psi != Phi, complex G, n' = 6144), fused loss
    with the workload's field g, r-blocks of 65536: the gradient rows of Phi
    and Psi at the sampled non-interpolation points against the oracle on the
    sub-problem of the interpolation rows plus those rows (the rows are local
    given Phi_mu and Psi_mu).  Orbital contractions in `prec` (FP64 solve):
    1e-5 relative for the lower precisions."""
    c = sio2_case
    d, wl = c["d"], c["wl"]
    sample = np.setdiff1d(c["rows"], c["idx"])
    psi_t = dev(d["psi"])
    phi_t = psi_t[:, : wl.n_phi]
    idx_t = dev(c["idx"])
    g = d["g"]
    _, minv, _ = isdf.fit(phi_t, psi_t, idx_t, nrows=0)
    dphi, dpsi, loss, info = isdf.fit_backward(phi_t, psi_t, idx_t, minv, g=dev(g), rblock=65536, prec=prec)
    sel = torch.as_tensor(sample).cuda()
    got_phi, got_psi = dphi[sel].cpu().numpy(), dpsi[sel].cpu().numpy()
    del dphi, dpsi
    sub = np.concatenate([c["idx"], sample])
    phi_sub = np.ascontiguousarray(d["phi"][sub])
    psi_sub = np.ascontiguousarray(d["psi"][sub])
    ref = oracle.fit_backward(phi_sub, psi_sub, np.arange(wl.n_mu), g=g[sub])
    tol = FP64_GRAD if prec == "fp64" else MIXED_GRAD
    e_phi = rel(got_phi, ref["dphi"][wl.n_mu:])
    e_psi = rel(got_psi, ref["dpsi"][wl.n_mu:])
    print(f"sio2 {prec} adjoint rows: dphi {e_phi:.3e}, dpsi {e_psi:.3e} (tol {tol:.1e}, {sample.size} rows)")
    assert e_phi <= tol and e_psi <= tol
    assert info["status"] == 0 and np.isfinite(loss.item()) and loss.item() > 0


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "fp16x3"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fit_sio2_mixed_precision_sampled_rows(sio2_case, prec, dtype):
    """Full-size SiO2 fit with the orbital contractions in FP32 or a split
    precision and the factorisation and solve in FP64.  The error is measured
    against (i) the oracle on the c128 data and, for c64 storage, (ii) the
    oracle on the c64 data upcast (arithmetic error alone).  The target is
    1e-6 relative for every precision."""
    c = sio2_case
    d, wl = c["d"], c["wl"]
    psi = d["psi"] if dtype == "c128" else d["psi"].astype(np.complex64)
    psi_t = dev(psi)
    phi_t = psi_t[:, : wl.n_phi]
    theta, _, info = isdf.fit(phi_t, psi_t, dev(c["idx"]), rblock=65536, prec=prec)
    got = theta[torch.as_tensor(c["rows"]).cuda()].cpu().numpy().astype(np.complex128)
    err_i = rel(got, c["ref"]["theta"])
    if dtype == "c128":
        err = err_i
        print(f"sio2 {prec} c128 theta rel err {err:.3e} (kappa {c['kappa']:.2e})")
    else:
        up = psi.astype(np.complex128)
        ref2 = oracle.fit(up[:, : wl.n_phi], up, c["idx"], rows=c["rows"])
        err = rel(got, ref2["theta"])
        print(f"sio2 {prec} c64 theta rel err {err:.3e} vs upcast oracle, {err_i:.3e} vs c128 oracle")
    assert err <= MIXED_THETA


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fit_fp32_gram_water8(water8_fit, dtype):
    """FP32 MFMA Gram blocks, FP64 solve: error against the FP64 oracle on the
    c128 data (and, for c64 storage, on the c64 data upcast)."""
    f = water8_fit
    phi = f["phi"] if dtype == "c128" else f["phi"].astype(np.complex64)
    theta, _, info = isdf.fit(dev(phi), None, dev(f["idx"].astype(np.int32)), prec="fp32")
    th = theta.cpu().numpy().astype(np.float64)
    ref = f["ref"]["theta"].real if dtype == "c128" else \
        oracle.fit_theta(phi.astype(np.complex128), phi.astype(np.complex128), f["idx"]).real
    err = rel(th, ref)
    print(f"water8 fp32 {dtype} theta rel err {err:.3e}")
    assert err <= MIXED_THETA


def test_fit_duplicate_and_out_of_range_idx():
    big, idx = tiny_complex(7)
    t = dev(big)
    bad = idx.copy()
    bad[3] = bad[1]
    _, _, info = isdf.fit(t[:, :7], t[:, 7:16], dev(bad), grid=(5, 6, 7), check=False)
    assert info["status"] == 4 and info["bad_idx"] == 3
    bad = idx.copy()
    bad[2] = 10 ** 6
    _, _, info = isdf.fit(t[:, :7], t[:, 7:16], dev(bad), grid=(5, 6, 7), check=False)
    assert info["status"] == 4 and info["bad_idx"] == 2


def test_fit_not_positive_definite():
    """Orbitals vanishing at an interpolation point make C C^H exactly
    singular: reported as not positive definite, with the pivot."""
    big, idx = tiny_complex(8)
    big[idx[0], :] = 0.0
    t = dev(big)
    _, _, info = isdf.fit(t[:, :7], None, dev(idx), grid=(5, 6, 7), check=False)
    assert info["status"] == 1 and info["pivot"] == 0


@pytest.mark.parametrize("n_mu,aliased", [(37, True), (100, True), (200, False), (130, True), (97, False)])
def test_minv_ragged_orders(n_mu, aliased):
    """(C C^H)^-1 for orders that are not multiples of the 64-wide diagonal
    blocks or of the doubling levels of the triangular inverse."""
    rng = np.random.default_rng(n_mu)
    nr = 9 * 9 * 9
    phi = rng.standard_normal((nr, 24)) + 1j * rng.standard_normal((nr, 24))
    psi = phi if aliased else rng.standard_normal((nr, 20)) + 1j * rng.standard_normal((nr, 20))
    idx = rng.choice(nr, n_mu, replace=False).astype(np.int32)
    pt = dev(phi)
    st = pt if aliased else dev(psi)
    theta, minv, info = isdf.fit(pt, None if aliased else st, dev(idx))
    ref = oracle.fit(phi, psi, idx)
    kappa = oracle.cc_condition(phi, psi, idx)
    assert info["status"] == 0
    th = theta.cpu().numpy()
    want = ref["theta"].real if aliased else ref["theta"]
    err = rel(th, want)
    print(f"minv order {n_mu} aliased {aliased}: theta rel err {err:.3e} (kappa {kappa:.2e})")
    assert err <= FP64_THETA
    n1 = n_mu if aliased else 2 * n_mu
    W = minv.cpu().numpy().reshape(n1, n1)
    M = ref["M"]
    if not aliased:  # real 2x2-block form of the complex matrix
        Me = np.zeros((n1, n1))
        Me[0::2, 0::2] = M.real
        Me[0::2, 1::2] = M.imag
        Me[1::2, 0::2] = -M.imag
        Me[1::2, 1::2] = M.real
        M = Me
    assert np.linalg.norm(W @ M.real - np.eye(n1)) <= 1e2 * kappa * EPS * np.sqrt(n1)


@pytest.mark.parametrize("prec", ["bf16x6", "fp16x3"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fit_split_precision_water8(water8_fit, prec, dtype):
    """Split-precision Gram blocks on 16-bit matrix cores, FP64 factorisation
    and solve: Theta within 1e-6 of the FP64 oracle (c64 storage: of the
    oracle on the upcast data)."""
    f = water8_fit
    phi = f["phi"] if dtype == "c128" else f["phi"].astype(np.complex64)
    theta, _, info = isdf.fit(dev(phi), None, dev(f["idx"].astype(np.int32)), prec=prec)
    th = theta.cpu().numpy().astype(np.float64)
    ref = f["ref"]["theta"].real if dtype == "c128" else \
        oracle.fit_theta(phi.astype(np.complex128), phi.astype(np.complex128), f["idx"]).real
    err = rel(th, ref)
    print(f"{prec} {dtype} theta rel err {err:.3e}")
    assert err <= MIXED_THETA


@pytest.mark.parametrize("prec", ["bf16x6", "fp16x3", "fp32"])
def test_fit_split_precision_complex_ragged(prec):
    big, idx = tiny_complex(15)
    t = dev(big)
    theta, _, _ = isdf.fit(t[:, :7], t[:, 7:16], dev(idx), grid=(5, 6, 7), prec=prec)
    ref = oracle.fit(big[:, :7], big[:, 7:16], idx)
    kappa = oracle.cc_condition(big[:, :7], big[:, 7:16], idx)
    err = rel(theta.cpu().numpy(), ref["theta"])
    print(f"{prec} complex theta rel err {err:.3e} (kappa {kappa:.1e})")
    assert err <= MIXED_THETA


@pytest.mark.parametrize("prec", ["bf16x6", "fp16x3"])
def test_split_precision_aliased_odd_slices(prec):
    """Phi = Psi through the one-operand-pair split kernels with K extents of
    an odd number of 32-deep slices, so the last LDS stage holds one slice:
    the Gram (2 N_e = 80 -> 96), Abar Phi_mu (2 N_mu = 140 -> 160) and the
    products over grid rows in r-blocks of 130, 130 and 40 rows (160 and 64).
    Theta and the fused-loss gradient against the oracle."""
    rng = np.random.default_rng(23)
    nr, n_e, n_mu = 300, 40, 70
    phi = rng.standard_normal((nr, n_e)) + 1j * rng.standard_normal((nr, n_e))
    idx = np.sort(rng.choice(nr, n_mu, replace=False)).astype(np.int32)
    g = rng.uniform(0.5, 1.5, nr)
    pt, it = dev(phi), dev(idx)
    theta, minv, _ = isdf.fit(pt, None, it, grid=(nr, 1, 1), prec=prec, rblock=130)
    ref = oracle.fit(phi, phi, idx)
    e_t = rel(theta.cpu().numpy(), ref["theta"].real)
    dphi, _, loss, info = isdf.fit_backward(pt, None, it, minv, g=dev(g), grid=(nr, 1, 1), prec=prec, rblock=130)
    rb = oracle.fit_backward(phi, phi, idx, g=g)
    e_g = rel(dphi.cpu().numpy(), rb["dphi"])
    print(f"{prec} aliased odd slices: theta {e_t:.3e}, dphi {e_g:.3e}")
    assert e_t <= MIXED_THETA and e_g <= MIXED_GRAD
    assert info["status"] == 0


@pytest.mark.parametrize("prec", ["bf16x6", "fp16x3"])
def test_zc_split_precision(prec):
    """Z C^H rows from isdf_zc against the oracle's A . conj(B)."""
    import ctypes as C
    from paper_2208_07731_amd import _lib as L
    rng = np.random.default_rng(16)
    nr, n_phi, n_psi, n_mu = 300, 40, 33, 70
    phi = rng.standard_normal((nr, n_phi)) + 1j * rng.standard_normal((nr, n_phi))
    psi = rng.standard_normal((nr, n_psi)) + 1j * rng.standard_normal((nr, n_psi))
    idx = rng.choice(nr, n_mu, replace=False).astype(np.int32)
    lib = L.load()
    pt, st, it = dev(phi), dev(psi), dev(idx)
    G = torch.empty(nr, 2 * n_mu, dtype=torch.float64, device="cuda")
    p = L.PRECS[prec]
    ws = torch.empty(lib.isdf_zc_workspace(n_mu, n_phi, n_psi, 0, p, nr), dtype=torch.uint8, device="cuda")
    g = L.make_grid((nr, 1, 1))
    code = lib.isdf_zc(C.byref(g), 0, pt.data_ptr(), n_phi, n_phi, st.data_ptr(), n_psi, n_psi, it.data_ptr(), n_mu,
                       p, 0, nr, G.data_ptr(), 2 * n_mu, ws.data_ptr(), ws.numel(),
                       torch.cuda.current_stream().cuda_stream)
    assert code == 0
    torch.cuda.synchronize()
    A, B = oracle.gram_blocks(phi, psi, idx)
    ref = oracle.hadamard(A, B)
    got = G.cpu().numpy().view(np.complex128)
    assert rel(got, ref) <= MIXED_THETA
