"""isdf_kmeans_noalloc (K-means with its scratch in a static device array,
for callers that cannot allocate) against isdf_kmeans with a workspace,
through the C ABI: bitwise equal outputs on two calls in a row, the second
with a smaller problem, so that the second reads a scratch the first left
dirty."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

isdf = pytest.importorskip("paper_2208_07731_amd")
from paper_2208_07731_amd import _lib as L  # noqa: E402


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def case(seed, n, n_orb, n_mu):
    rng = np.random.default_rng(seed)
    nr = n[0] * n[1] * n[2]
    phi = rng.standard_normal((nr, n_orb)) + 1j * rng.standard_normal((nr, n_orb))
    c0 = oracle.grid_points(n)[rng.choice(nr, n_mu, replace=False)]
    return phi, c0


def run(lib, noalloc, phi_t, n, n_mu, c0_t, rounds):
    nr = phi_t.shape[0]
    g = L.make_grid(n)
    idx = torch.full((n_mu,), -7, dtype=torch.int32, device="cuda")
    cent = torch.full((n_mu, 3), -7.0, dtype=torch.float64, device="cuda")
    labels = torch.full((nr,), -7, dtype=torch.int32, device="cuda")
    w = torch.full((nr,), -7.0, dtype=torch.float64, device="cuda")
    obj = torch.full((rounds + 1,), -7.0, dtype=torch.float64, device="cuda")
    info = torch.zeros(C.sizeof(L.KmeansInfo), dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    ld, ne = phi_t.stride(0), phi_t.shape[1]
    args = (C.byref(g), L.C128, phi_t.data_ptr(), ld, ne, phi_t.data_ptr(), ld, ne, 0, 0, n_mu, c0_t.data_ptr(),
            rounds, 1e-6, idx.data_ptr(), cent.data_ptr(), labels.data_ptr(), w.data_ptr(), obj.data_ptr(),
            info.data_ptr())
    if noalloc:
        code = lib.isdf_kmeans_noalloc(*args, s)
    else:
        ws = torch.empty(lib.isdf_kmeans_workspace(C.byref(g), n_mu, rounds), dtype=torch.uint8, device="cuda")
        code = lib.isdf_kmeans(*args, ws.data_ptr(), ws.numel(), s)
    assert code == L.OK
    torch.cuda.synchronize()
    return dict(idx=idx, cent=cent, labels=labels, w=w, obj=obj, info=info)


def test_noalloc_kmeans_matches_workspace_form_twice():
    lib = L.load()
    cases = [((20, 18, 22), 24, 300, 12), ((9, 10, 11), 7, 37, 5)]  # the second is smaller
    for k, (n, n_orb, n_mu, rounds) in enumerate(cases):
        phi, c0 = case(40 + k, n, n_orb, n_mu)
        phi_t, c0_t = dev(phi), dev(c0)
        a = run(lib, True, phi_t, n, n_mu, c0_t, rounds)
        b = run(lib, False, phi_t, n, n_mu, c0_t, rounds)
        for key in a:
            assert torch.equal(a[key], b[key]), (k, key)
        inf = L.KmeansInfo.from_buffer_copy(bytes(a["info"].cpu().numpy()))
        assert inf.status == L.OK and inf.iters >= 1
        # and the oracle's points (Alg. 1 with the same seeds)
        km = oracle.kmeans(n, oracle.weight(phi, None), c0, rounds)
        assert np.array_equal(a["idx"].cpu().numpy(), km["idx"])

