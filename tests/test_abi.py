"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/isdf.h, and rejects bad arguments on the host before
enqueueing anything."""
import ctypes as C
import os
import re

import pytest

from paper_2208_07731_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "isdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(isdf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ("isdf_kmeans", "isdf_fit", "isdf_fit_backward", "isdf_kmeans_workspace", "isdf_fit_workspace",
              "isdf_fit_backward_workspace", "isdf_fit_minv_elems", "isdf_version", "isdf_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for n in header_functions():
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, n


def test_strerror_and_version():
    lib = L.load()
    assert b"gfx950" in lib.isdf_version()
    for code in (L.OK, L.E_ARG, L.E_WORKSPACE, L.E_HIP, L.E_UNSUPPORTED, L.E_SCRATCH, L.E_NOT_PD, L.E_NONFINITE,
                 L.W_EMPTY_CLUSTER, L.E_BAD_IDX):
        assert L.strerror(code) != "unknown status"
    assert L.strerror(12345) == "unknown status"


def test_workspace_queries():
    lib = L.load()
    g = L.make_grid(24)
    a = lib.isdf_kmeans_workspace(C.byref(g), 256, 30)
    b = lib.isdf_kmeans_workspace(C.byref(g), 256, 60)
    assert 0 < a < b
    assert lib.isdf_kmeans_workspace(C.byref(g), 0, 30) == 0
    f1 = lib.isdf_fit_workspace(C.byref(g), 256, 32, 32, 1, 0, 1000)
    f2 = lib.isdf_fit_workspace(C.byref(g), 256, 32, 32, 1, 0, 2000)
    assert 0 < f1 < f2
    assert lib.isdf_fit_minv_elems(256, 1) == 256 * 256
    assert lib.isdf_fit_minv_elems(256, 0) == 512 * 512
    assert lib.isdf_fit_backward_workspace(C.byref(g), 256, 32, 32, 1, 0, 1000) > 0


FAKE = 0x1000  # never dereferenced: every call below must fail its host checks


@pytest.mark.parametrize("case", ["n_mu0", "n_mu_big", "null_c0", "neg_iter", "bad_ld", "bad_kind", "flags",
                                  "no_ws", "bad_grid"])
def test_kmeans_rejects_bad_arguments(case):
    lib = L.load()
    g = L.make_grid(8)
    kw = dict(dt=L.C128, phi=FAKE, ld=4, n=4, kind=0, flags=0, n_mu=5, c0=FAKE, iters=3, idx=FAKE, info=FAKE,
              ws=FAKE, wsb=1 << 30)
    if case == "n_mu0":
        kw["n_mu"] = 0
    elif case == "n_mu_big":
        kw["n_mu"] = 513
    elif case == "null_c0":
        kw["c0"] = None
    elif case == "neg_iter":
        kw["iters"] = -1
    elif case == "bad_ld":
        kw["ld"] = 3
    elif case == "bad_kind":
        kw["kind"] = 9
    elif case == "flags":
        kw["flags"] = 6
    elif case == "no_ws":
        kw["wsb"] = 16
    elif case == "bad_grid":
        g.n[1] = 0
    code = lib.isdf_kmeans(C.byref(g), kw["dt"], kw["phi"], kw["ld"], kw["n"], kw["phi"], kw["ld"], kw["n"],
                           kw["kind"], kw["flags"], kw["n_mu"], kw["c0"], kw["iters"], 1e-6, kw["idx"], None, None,
                           None, None, kw["info"], kw["ws"], kw["wsb"], None)
    assert code == (L.E_WORKSPACE if case == "no_ws" else L.E_ARG)


@pytest.mark.parametrize("case", ["n_mu0", "null_c0", "bad_kind", "no_labels", "no_w", "no_centroids",
                                  "beyond_scratch"])
def test_kmeans_noalloc_rejects_on_the_host(case):
    """The allocation-free K-means checks its arguments, and that its scratch
    (4 MiB) holds the request, before touching the device."""
    lib = L.load()
    g = L.make_grid(8)
    kw = dict(kind=0, n_mu=5, c0=FAKE, cent=FAKE, labels=FAKE, w=FAKE, iters=3)
    if case == "n_mu0":
        kw["n_mu"] = 0
    elif case == "null_c0":
        kw["c0"] = None
    elif case == "bad_kind":
        kw["kind"] = 9
    elif case == "no_labels":
        kw["labels"] = None
    elif case == "no_w":
        kw["w"] = None
    elif case == "no_centroids":
        kw["cent"] = None
    elif case == "beyond_scratch":
        g = L.make_grid(64)
        kw["n_mu"] = 200000  # 4.8 MB of per-cluster bounding boxes alone
    code = lib.isdf_kmeans_noalloc(C.byref(g), L.C128, FAKE, 4, 4, FAKE, 4, 4, kw["kind"], 0, kw["n_mu"], kw["c0"],
                                   kw["iters"], 1e-6, FAKE, kw["cent"], kw["labels"], kw["w"], None, FAKE, None)
    assert code == (L.E_SCRATCH if case == "beyond_scratch" else L.E_ARG)


@pytest.mark.parametrize("case", ["rows", "ld_theta", "prec_dtype", "null_minv", "flags", "no_ws", "bad_prec"])
def test_fit_rejects_bad_arguments(case):
    lib = L.load()
    g = L.make_grid(8)
    kw = dict(dt=L.C128, prec=0, minv=FAKE, flags=1, row0=0, nrows=512, ldt=5, wsb=1 << 30)
    if case == "rows":
        kw["row0"] = 10
    elif case == "ld_theta":
        kw["ldt"] = 4
    elif case == "prec_dtype":
        kw["dt"] = L.C64
    elif case == "null_minv":
        kw["minv"] = None
    elif case == "flags":
        kw["flags"] = 2
    elif case == "no_ws":
        kw["wsb"] = 16
    elif case == "bad_prec":
        kw["prec"] = 7
    code = lib.isdf_fit(C.byref(g), kw["dt"], FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, kw["prec"], kw["minv"], kw["flags"],
                        kw["row0"], kw["nrows"], FAKE, kw["ldt"], 512, FAKE, FAKE, kw["wsb"], None)
    expect = {"no_ws": L.E_WORKSPACE}.get(case, L.E_ARG)
    assert code == expect


def test_residual_entry_points_reject_bad_arguments():
    lib = L.load()
    g = L.make_grid(8)
    assert lib.isdf_cluster_residual_workspace() > 0
    assert lib.isdf_fit_residual_workspace(C.byref(g), 5, 4, 4, 1, 0, 512) > 0
    # cluster residual: missing labels, bad dtype, short workspace
    assert lib.isdf_cluster_residual(C.byref(g), L.C128, FAKE, 4, 4, FAKE, 4, 4, None, FAKE, 5, FAKE, FAKE, 1 << 20,
                                     None) == L.E_ARG
    assert lib.isdf_cluster_residual(C.byref(g), 7, FAKE, 4, 4, FAKE, 4, 4, FAKE, FAKE, 5, FAKE, FAKE, 1 << 20,
                                     None) == L.E_ARG
    assert lib.isdf_cluster_residual(C.byref(g), L.C128, FAKE, 4, 4, FAKE, 4, 4, FAKE, FAKE, 5, FAKE, FAKE, 8,
                                     None) == L.E_WORKSPACE
    # fit residual: no minv, FP64 on c64 storage, short workspace
    assert lib.isdf_fit_residual(C.byref(g), L.C128, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, 0, None, 512, FAKE, FAKE, FAKE,
                                 1 << 30, None) == L.E_ARG
    assert lib.isdf_fit_residual(C.byref(g), L.C64, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, 0, FAKE, 512, FAKE, FAKE, FAKE,
                                 1 << 30, None) == L.E_ARG
    assert lib.isdf_fit_residual(C.byref(g), L.C128, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, 0, FAKE, 512, FAKE, FAKE, FAKE,
                                 16, None) == L.E_WORKSPACE


def test_poisson_rejects_bad_arguments():
    lib = L.load()
    g = L.make_grid(8)
    assert lib.isdf_poisson_workspace(C.byref(g), 10, 0) > 0
    bad = L.make_grid((8, 11, 8))  # prime factor 11
    assert lib.isdf_poisson_workspace(C.byref(bad), 10, 0) == 0
    assert lib.isdf_poisson(C.byref(bad), L.C128, FAKE, 10, 10, 0, FAKE, 10, FAKE, 1 << 30, None) == L.E_UNSUPPORTED
    big = L.make_grid((8, 8, 288))  # axis above 256 points
    assert lib.isdf_poisson(C.byref(big), L.C128, FAKE, 10, 10, 0, FAKE, 10, FAKE, 1 << 30, None) == L.E_UNSUPPORTED
    assert lib.isdf_poisson(C.byref(g), L.C128, FAKE, 9, 10, 0, FAKE, 10, FAKE, 1 << 30, None) == L.E_ARG
    assert lib.isdf_poisson(C.byref(g), L.C128, FAKE, 10, 10, 0, FAKE, 10, FAKE, 8, None) == L.E_WORKSPACE
    g0 = L.make_grid(8, (1.0, 0.0, 1.0))
    assert lib.isdf_poisson(C.byref(g0), L.C128, FAKE, 10, 10, 0, FAKE, 10, FAKE, 1 << 30, None) == L.E_ARG


def test_qrcp_rejects_bad_arguments():
    lib = L.load()
    g = L.make_grid(8)
    wa = lib.isdf_qrcp_workspace(C.byref(g), 10, 1)
    wc = lib.isdf_qrcp_workspace(C.byref(g), 10, 0)
    assert 0 < wa < wc and wa >= 9 * 512 * 8 and wc >= 9 * 512 * 16
    assert lib.isdf_qrcp_workspace(C.byref(g), 0, 1) == 0

    def call(**over):
        kw = dict(dt=L.C128, phi=FAKE, ld=4, n=4, psi=FAKE, ldp=4, np_=4, n_mu=10, rtol=1e-7, ntr=1e-9,
                  idx=FAKE, rd=FAKE, gap=None, info=FAKE, ws=FAKE, wsb=1 << 30)
        kw.update(over)
        return lib.isdf_qrcp(C.byref(g), kw["dt"], kw["phi"], kw["ld"], kw["n"], kw["psi"], kw["ldp"], kw["np_"],
                             kw["n_mu"], kw["rtol"], kw["ntr"], kw["idx"], kw["rd"], kw["gap"], kw["info"], kw["ws"],
                             kw["wsb"], None)

    assert call(n_mu=0) == L.E_ARG
    assert call(n_mu=513) == L.E_ARG
    assert call(idx=None) == L.E_ARG
    assert call(rd=None) == L.E_ARG
    assert call(info=None) == L.E_ARG
    assert call(ld=3) == L.E_ARG
    assert call(dt=5) == L.E_ARG
    assert call(rtol=1.0) == L.E_ARG
    assert call(rtol=-1.0) == L.E_ARG
    assert call(ntr=float("nan")) == L.E_ARG
    assert call(wsb=wa - 1) == L.E_WORKSPACE
    assert call(psi=FAKE + 64, wsb=wc - 1) == L.E_WORKSPACE  # Psi != Phi needs the complex workspace
    assert call(n=3000, ld=3000, psi=FAKE + 64, np_=3000, ldp=3000) == L.E_UNSUPPORTED


def test_saved_gram_entry_points_reject_bad_arguments():
    lib = L.load()
    g = L.make_grid(8)
    full = lib.isdf_fit_backward_workspace(C.byref(g), 5, 4, 4, 1, 0, 512)
    saved = lib.isdf_fit_backward_gram_workspace(C.byref(g), 5, 4, 4, 1, 0, 512)
    assert 0 < saved < full  # no r-block copies of G and A
    # isdf_zc_ab: A missing
    assert lib.isdf_zc_ab(C.byref(g), L.C128, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, 0, 0, 512, FAKE, 5, None, None,
                          FAKE, 1 << 30, None) == L.E_ARG
    # Psi != Phi: B missing
    assert lib.isdf_zc_ab(C.byref(g), L.C128, FAKE, 4, 4, FAKE + 64, 4, 4, FAKE, 5, 0, 0, 512, FAKE, 10, FAKE, None,
                          FAKE, 1 << 30, None) == L.E_ARG

    def bwd(G=FAKE, A=FAKE, B=None, wsb=1 << 30, psi=FAKE):
        return lib.isdf_fit_backward_gram(C.byref(g), L.C128, FAKE, 4, 4, psi, 4, 4, FAKE, 5, 0, FAKE, None, 0, FAKE,
                                          FAKE, 4, FAKE + 4096, 4, None, 512, G, A, B, FAKE, FAKE, wsb, None)

    assert bwd(G=None) == L.E_ARG
    assert bwd(A=None) == L.E_ARG
    assert bwd(psi=FAKE + 64) == L.E_ARG  # general case needs B
    assert bwd(wsb=saved - 1) == L.E_WORKSPACE


def test_qrcp_sketch_rejects_bad_arguments():
    lib = L.load()
    g = L.make_grid(8)
    w = lib.isdf_qrcp_sketch_workspace(C.byref(g), 10, 4, 4, 12)
    assert w >= 512 * 12 * 16 and lib.isdf_qrcp_sketch_workspace(C.byref(g), 10, 4, 4, 0) == 0

    def call(**over):
        kw = dict(gp=FAKE, gs=FAKE, m=12, n_mu=10, wsb=1 << 30)
        kw.update(over)
        return lib.isdf_qrcp_sketch(C.byref(g), L.C128, FAKE, 4, 4, FAKE, 4, 4, kw["gp"], kw["gs"], kw["m"],
                                    kw["n_mu"], 1e-7, 1e-9, FAKE, FAKE, None, FAKE, FAKE, kw["wsb"], None)

    assert call(gp=None) == L.E_ARG
    assert call(gs=None) == L.E_ARG
    assert call(m=0) == L.E_ARG
    assert call(n_mu=600) == L.E_ARG
    # no upper limit on m: the step kernel reads the pivot's sketch row in place
    assert lib.isdf_qrcp_sketch_workspace(C.byref(g), 10, 4, 4, 5000) > 512 * 5000 * 16
    assert call(wsb=w - 1) == L.E_WORKSPACE


@pytest.mark.parametrize("bad", [-1, 2, 7, 1 << 20])
def test_out_of_range_enumerations_are_rejected(bad):
    """dtype and precision arrive as int32; values outside isdf_dtype /
    isdf_prec are rejected on the host (workspace queries return 0)."""
    lib = L.load()
    g = L.make_grid(8)
    badp = bad + 2 if bad == 2 else bad  # 2 is a valid precision (BF16x6)
    assert lib.isdf_fit_workspace(C.byref(g), 5, 4, 4, 1, badp, 512) == 0
    assert lib.isdf_fit_residual_workspace(C.byref(g), 5, 4, 4, 1, badp, 512) == 0
    assert lib.isdf_zc_workspace(5, 4, 4, 1, badp, 512) == 0
    assert lib.isdf_fit_backward_workspace(C.byref(g), 5, 4, 4, 1, badp, 512) == 0
    assert lib.isdf_fit_backward_gram_workspace(C.byref(g), 5, 4, 4, 1, badp, 512) == 0
    for dt, prec in ((bad, 0), (L.C128, badp)):
        assert lib.isdf_fit(C.byref(g), dt, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, prec, FAKE, 1, 0, 512, FAKE, 5, 512,
                            FAKE, FAKE, 1 << 30, None) == L.E_ARG
        assert lib.isdf_zc(C.byref(g), dt, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, prec, 0, 512, FAKE, 5, FAKE, 1 << 30,
                           None) == L.E_ARG
        assert lib.isdf_fit_backward(C.byref(g), dt, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, prec, FAKE, None, 0, FAKE,
                                     FAKE, 4, FAKE + 4096, 4, None, 512, FAKE, FAKE, 1 << 30, None) == L.E_ARG
        assert lib.isdf_fit_residual(C.byref(g), dt, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, prec, FAKE, 512, FAKE, FAKE,
                                     FAKE, 1 << 30, None) == L.E_ARG
    assert lib.isdf_kmeans(C.byref(g), bad, FAKE, 4, 4, FAKE, 4, 4, 0, 0, 5, FAKE, 3, 1e-6, FAKE, None, None, None,
                           None, FAKE, FAKE, 1 << 30, None) == L.E_ARG
    assert lib.isdf_apply_minv(5, 1, FAKE, FAKE, 5, 512, bad, FAKE, 5, None) == L.E_ARG
    assert lib.isdf_poisson(C.byref(g), bad, FAKE, 10, 10, 0, FAKE, 10, FAKE, 1 << 30, None) == L.E_ARG
    assert lib.isdf_exchange(C.byref(g), bad, FAKE, 4, 4, FAKE, 4, 4, FAKE, 5, FAKE, 5, 0, FAKE, 4, 512, FAKE,
                             1 << 30, None) == L.E_ARG
    assert lib.isdf_qrcp(C.byref(g), bad, FAKE, 4, 4, FAKE, 4, 4, 10, 1e-7, 1e-9, FAKE, FAKE, None, FAKE, FAKE,
                         1 << 30, None) == L.E_ARG
    assert lib.isdf_qrcp_sketch(C.byref(g), bad, FAKE, 4, 4, FAKE, 4, 4, FAKE, FAKE, 12, 10, 1e-7, 1e-9, FAKE, FAKE,
                                None, FAKE, FAKE, 1 << 30, None) == L.E_ARG
    assert lib.isdf_cluster_residual(C.byref(g), bad, FAKE, 4, 4, FAKE, 4, 4, FAKE, FAKE, 5, FAKE, FAKE, 1 << 20,
                                     None) == L.E_ARG


def test_one_hip_runtime_in_the_process():
    """Loading the library after torch maps a single HIP runtime: the one
    torch ships (same soname), not a second copy from /opt/rocm, so the
    streams and device memory torch hands over belong to the runtime the
    library's launches go through.  Checked in a fresh interpreter."""
    import subprocess
    import sys

    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2208_07731_amd import _lib as L\n"
        "L.load()\n"
        "paths = set()\n"
        "for line in open('/proc/self/maps'):\n"
        "    f = line.split()\n"
        "    if len(f) >= 6 and 'libamdhip64' in f[5]:\n"
        "        paths.add(f[5])\n"
        "print(len(paths), sorted(paths))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    n = int(out.stdout.split()[0])
    assert n == 1, out.stdout
