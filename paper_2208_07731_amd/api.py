"""Python binding of libisdf: argument marshalling around the C ABI.

Every step of the ISDF path runs in the library's HIP kernels; this module
only checks tensors, allocates outputs / workspace through PyTorch, passes
raw device pointers and the current stream, and turns status codes into
exceptions.  Names follow the C calls: kmeans, fit, fit_backward.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import warnings

import torch

from . import _lib as L


class ISDFError(RuntimeError):
    def __init__(self, code: int, where: str, extra: str = ""):
        self.code = int(code)
        super().__init__(f"{where}: {L.strerror(code)} (status {code}){extra}")


def _stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check(code: int, where: str):
    if code != L.OK:
        raise ISDFError(code, where)


def _orbital(x: torch.Tensor, name: str):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype not in (torch.complex128, torch.complex64) or x.dim() != 2:
        raise TypeError(f"{name} must be a 2-D complex128/complex64 tensor (N_r, n)")
    if x.stride(1) != 1 or x.stride(0) < x.shape[1]:
        raise ValueError(f"{name} needs unit column stride and row stride >= columns")
    dt = L.C128 if x.dtype == torch.complex128 else L.C64
    return dt, x.data_ptr(), x.stride(0), x.shape[1]


def _same(a: torch.Tensor, b: torch.Tensor) -> bool:
    return a.data_ptr() == b.data_ptr() and a.stride() == b.stride() and a.shape == b.shape and a.dtype == b.dtype


def _read_struct(buf: torch.Tensor, cls):
    raw = bytes(buf.cpu().numpy().tobytes())
    return cls.from_buffer_copy(raw)


def _grid(grid, n_r: int, h, geometry: bool = True):
    if grid is None and not geometry:
        grid = (n_r, 1, 1)  # the fit uses only the number of grid rows
    if grid is None:
        n = round(n_r ** (1.0 / 3.0))
        if n ** 3 != n_r:
            raise ValueError("grid=(n0, n1, n2) is required for non-cubic grids")
        grid = (n, n, n)
    g = L.make_grid(grid, h)
    if g.n[0] * g.n[1] * g.n[2] != n_r:
        raise ValueError("grid does not match the number of orbital rows")
    return g


@dataclasses.dataclass
class KMeansResult:
    idx: torch.Tensor        # int32 [n_mu]
    centroids: torch.Tensor  # float64 [n_mu, 3]
    labels: torch.Tensor     # int32 [N_r]
    w: torch.Tensor          # float64 [N_r]
    objective: torch.Tensor  # float64 [max_iter + 1], -1 where no classification ran
    info: dict


def kmeans(phi: torch.Tensor | None, psi: torch.Tensor | None, n_mu: int, c0, max_iter: int, *,
           grid=None, h=(1.0, 1.0, 1.0), weight: str = "ssm", w: torch.Tensor | None = None,
           near_tie_rel: float = 1e-6, check: bool = True) -> KMeansResult:
    """Weighted K-means on the grid (isdf_kmeans).  With `w` given, the weight
    pass is skipped and phi/psi may be None."""
    lib = L.load()
    dev = (phi if phi is not None else w).device
    flags = 0
    if w is not None:
        if w.dtype != torch.float64 or not w.is_contiguous() or not w.is_cuda:
            raise TypeError("w must be a contiguous float64 CUDA tensor")
        n_r = w.numel()
        flags |= L.KM_WEIGHT_GIVEN
        dt, pp, lp, npf, ps, lps, nps = L.C128, None, 0, 0, None, 0, 0
        wout = w
    else:
        if psi is None:
            psi = phi
        dt, pp, lp, npf = _orbital(phi, "phi")
        dt2, ps, lps, nps = _orbital(psi, "psi")
        if dt2 != dt:
            raise TypeError("phi and psi must have the same dtype")
        n_r = phi.shape[0]
        if psi.shape[0] != n_r:
            raise ValueError("phi and psi must have the same number of rows")
        wout = torch.empty(n_r, dtype=torch.float64, device=dev)
    g = _grid(grid, n_r, h)
    c0 = torch.as_tensor(c0, dtype=torch.float64).to(dev).contiguous()
    if c0.shape != (n_mu, 3):
        raise ValueError("c0 must have shape (n_mu, 3)")
    idx = torch.empty(n_mu, dtype=torch.int32, device=dev)
    cent = torch.empty(n_mu, 3, dtype=torch.float64, device=dev)
    labels = torch.empty(n_r, dtype=torch.int32, device=dev)
    obj = torch.empty(max_iter + 1, dtype=torch.float64, device=dev)
    info = torch.zeros(C.sizeof(L.KmeansInfo), dtype=torch.uint8, device=dev)
    wsb = lib.isdf_kmeans_workspace(C.byref(g), n_mu, max_iter)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    code = lib.isdf_kmeans(C.byref(g), dt, pp, lp, npf, ps, lps, nps, L.WEIGHTS[weight], flags, n_mu,
                           c0.data_ptr(), max_iter, near_tie_rel, idx.data_ptr(), cent.data_ptr(),
                           labels.data_ptr(), wout.data_ptr(), obj.data_ptr(), info.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream_handle())
    _check(code, "isdf_kmeans")
    torch.cuda.current_stream().synchronize()
    inf = _read_struct(info, L.KmeansInfo)
    d = {f: getattr(inf, f) for f, _ in L.KmeansInfo._fields_}
    if check:
        if inf.status == L.W_EMPTY_CLUSTER:
            warnings.warn(f"isdf_kmeans: {inf.empty_final} cluster(s) ended empty (idx = -1)")
        elif inf.status != L.OK:
            raise ISDFError(inf.status, "isdf_kmeans")
    return KMeansResult(idx, cent, labels, wout, obj, d)


@dataclasses.dataclass
class QRCPResult:
    idx: torch.Tensor    # int32 [n_mu], -1 from the rank on
    rdiag: torch.Tensor  # float64 [n_mu], |R_kk|
    gap: torch.Tensor    # float64 [n_mu], decision margin of each pivot
    info: dict


def qrcp(phi: torch.Tensor, psi: torch.Tensor | None, n_mu: int, *, rtol: float = 1e-7,
         near_tie_rel: float = 1e-9, grid=None, sketch=None) -> QRCPResult:
    """Interpolation points by QR with column pivoting of Z^T (isdf_qrcp,
    eq. QRCP), Z never formed.  psi None or psi is phi: the aliased path.
    sketch=(g_phi, g_psi), float64 device tensors [N_phi][m] and [N_psi][m]:
    the randomized QRCP of the Khatri-Rao sketch (isdf_qrcp_sketch)."""
    lib = L.load()
    if psi is None:
        psi = phi
    dt, pp, lp, npf = _orbital(phi, "phi")
    dt2, ps, lps, nps = _orbital(psi, "psi")
    if dt2 != dt or psi.shape[0] != phi.shape[0] or psi.device != phi.device:
        raise TypeError("phi and psi must share dtype, row count and device")
    n_r = phi.shape[0]
    g = _grid(grid, n_r, (1.0, 1.0, 1.0), geometry=False)
    dev = phi.device
    idx = torch.empty(n_mu, dtype=torch.int32, device=dev)
    rdiag = torch.empty(n_mu, dtype=torch.float64, device=dev)
    gap = torch.empty(n_mu, dtype=torch.float64, device=dev)
    info = torch.zeros(C.sizeof(L.QrcpInfo), dtype=torch.uint8, device=dev)
    if sketch is None:
        wsb = lib.isdf_qrcp_workspace(C.byref(g), n_mu, int(_same(phi, psi)))
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        code = lib.isdf_qrcp(C.byref(g), dt, pp, lp, npf, ps, lps, nps, n_mu, rtol, near_tie_rel, idx.data_ptr(),
                             rdiag.data_ptr(), gap.data_ptr(), info.data_ptr(), ws.data_ptr(), ws.numel(),
                             _stream_handle())
        _check(code, "isdf_qrcp")
    else:
        gp, gs = sketch
        m = gp.shape[1]
        for t, n in ((gp, npf), (gs, nps)):
            if t.dtype != torch.float64 or t.device != dev or not t.is_contiguous() or t.shape != (n, m):
                raise TypeError("sketch matrices must be contiguous float64 (N_phi, m) and (N_psi, m) on the "
                                "orbitals' device")
        wsb = lib.isdf_qrcp_sketch_workspace(C.byref(g), n_mu, npf, nps, m)
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        code = lib.isdf_qrcp_sketch(C.byref(g), dt, pp, lp, npf, ps, lps, nps, gp.data_ptr(), gs.data_ptr(), m, n_mu,
                                    rtol, near_tie_rel, idx.data_ptr(), rdiag.data_ptr(), gap.data_ptr(),
                                    info.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle())
        _check(code, "isdf_qrcp_sketch")
    torch.cuda.current_stream().synchronize()
    inf = _read_struct(info, L.QrcpInfo)
    if inf.status != L.OK:
        raise ISDFError(inf.status, "isdf_qrcp")
    return QRCPResult(idx, rdiag, gap, {f: getattr(inf, f) for f, _ in L.QrcpInfo._fields_})


def _prec(prec: str) -> int:
    if prec not in L.PRECS:
        raise ValueError(f"prec must be one of {list(L.PRECS)}")
    return L.PRECS[prec]


def _fit_common(phi, psi, idx):
    if psi is None:
        psi = phi
    dt, pp, lp, npf = _orbital(phi, "phi")
    dt2, ps, lps, nps = _orbital(psi, "psi")
    if dt2 != dt or psi.shape[0] != phi.shape[0] or psi.device != phi.device:
        raise ValueError("phi and psi must match in dtype, rows and device")
    if idx.dtype != torch.int32 or not idx.is_contiguous() or idx.device != phi.device:
        raise TypeError("idx must be a contiguous int32 tensor on the orbitals' device")
    aliased = _same(phi, psi)
    return psi, dt, pp, lp, npf, ps, lps, nps, aliased


def fit(phi: torch.Tensor, psi: torch.Tensor | None, idx: torch.Tensor, *, prec: str = "fp64",
        minv: torch.Tensor | None = None, factor: bool = True, row0: int = 0, nrows: int | None = None,
        rblock: int | None = None, grid=None, check: bool = True):
    """Interpolation vectors Theta for rows [row0, row0 + nrows) (isdf_fit).

    Returns (theta, minv, info).  theta is real (float64 / float32) when psi is
    phi, complex otherwise.  minv holds (C C^H)^-1 for reuse (factor=False).
    """
    lib = L.load()
    psi, dt, pp, lp, npf, ps, lps, nps, aliased = _fit_common(phi, psi, idx)
    n_r, n_mu = phi.shape[0], idx.numel()
    g = _grid(grid, n_r, (1.0, 1.0, 1.0), geometry=False)
    nrows = n_r - row0 if nrows is None else nrows
    rblock = max(1, min(nrows, 1 << 17)) if rblock is None else rblock
    p = _prec(prec)
    dev = phi.device
    n_minv = lib.isdf_fit_minv_elems(n_mu, int(aliased))
    if minv is None:
        minv = torch.empty(n_minv, dtype=torch.float64, device=dev)
        factor = True
    if minv.numel() < n_minv or minv.dtype != torch.float64:
        raise ValueError("minv too small or not float64")
    real_t = torch.float64 if dt == L.C128 else torch.float32
    cplx_t = torch.complex128 if dt == L.C128 else torch.complex64
    theta = torch.empty(nrows, n_mu, dtype=real_t if aliased else cplx_t, device=dev)
    info = torch.zeros(C.sizeof(L.FitInfo), dtype=torch.uint8, device=dev)
    wsb = lib.isdf_fit_workspace(C.byref(g), n_mu, npf, nps, int(aliased), p, rblock)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    code = lib.isdf_fit(C.byref(g), dt, pp, lp, npf, ps, lps, nps, idx.data_ptr(), n_mu, p, minv.data_ptr(),
                        L.FIT_FACTOR if factor else 0, row0, nrows, theta.data_ptr(), n_mu, rblock,
                        info.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle())
    _check(code, "isdf_fit")
    torch.cuda.current_stream().synchronize()
    inf = _read_struct(info, L.FitInfo)
    d = {f: getattr(inf, f) for f, _ in L.FitInfo._fields_}
    if check and inf.status != L.OK:
        raise ISDFError(inf.status, "isdf_fit", f" pivot={inf.pivot} bad_idx={inf.bad_idx}")
    return theta, minv, d


def fit_backward(phi: torch.Tensor, psi: torch.Tensor | None, idx: torch.Tensor, minv: torch.Tensor, *,
                 theta_bar: torch.Tensor | None = None, g: torch.Tensor | None = None, prec: str = "fp64",
                 rblock: int | None = None, grid=None, check: bool = True):
    """Gradients (dphi, dpsi, loss, info) of the fit (isdf_fit_backward).

    theta_bar: upstream gradient of Theta; or g: field of the fused loss
    L = sum_r g_r sum_mu |Theta_r,mu|^2 (then loss is its value)."""
    lib = L.load()
    psi, dt, pp, lp, npf, ps, lps, nps, aliased = _fit_common(phi, psi, idx)
    n_r, n_mu = phi.shape[0], idx.numel()
    gr = _grid(grid, n_r, (1.0, 1.0, 1.0), geometry=False)
    rblock = min(n_r, 1 << 17) if rblock is None else rblock
    p = _prec(prec)
    dev = phi.device
    if (theta_bar is None) == (g is None):
        raise ValueError("give exactly one of theta_bar and g")
    tb_ptr, tb_ld, g_ptr = None, 0, None
    if theta_bar is not None:
        want = (torch.float64 if dt == L.C128 else torch.float32) if aliased else \
            (torch.complex128 if dt == L.C128 else torch.complex64)
        if theta_bar.dtype != want or theta_bar.shape != (n_r, n_mu) or theta_bar.stride(1) != 1:
            raise TypeError(f"theta_bar must be {want} of shape (N_r, n_mu) with unit column stride")
        tb_ptr, tb_ld = theta_bar.data_ptr(), theta_bar.stride(0)
    else:
        if g.dtype != torch.float64 or g.numel() != n_r or not g.is_contiguous():
            raise TypeError("g must be a contiguous float64 tensor of N_r entries")
        g_ptr = g.data_ptr()
    dphi = torch.empty(n_r, npf, dtype=phi.dtype, device=dev)
    dpsi = dphi if aliased else torch.empty(n_r, nps, dtype=psi.dtype, device=dev)
    loss = torch.zeros((), dtype=torch.float64, device=dev)
    info = torch.zeros(C.sizeof(L.FitInfo), dtype=torch.uint8, device=dev)
    wsb = lib.isdf_fit_backward_workspace(C.byref(gr), n_mu, npf, nps, int(aliased), p, rblock)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    code = lib.isdf_fit_backward(C.byref(gr), dt, pp, lp, npf, ps, lps, nps, idx.data_ptr(), n_mu, p,
                                 minv.data_ptr(), tb_ptr, tb_ld, g_ptr, dphi.data_ptr(), npf, dpsi.data_ptr(),
                                 nps, loss.data_ptr(), rblock, info.data_ptr(), ws.data_ptr(), ws.numel(),
                                 _stream_handle())
    _check(code, "isdf_fit_backward")
    torch.cuda.current_stream().synchronize()
    inf = _read_struct(info, L.FitInfo)
    d = {f: getattr(inf, f) for f, _ in L.FitInfo._fields_}
    if check and inf.status != L.OK:
        raise ISDFError(inf.status, "isdf_fit_backward")
    if aliased:
        dpsi = dphi.clone()
    return dphi, dpsi, loss, d


def fit_residual(phi: torch.Tensor, psi: torch.Tensor | None, idx: torch.Tensor, minv: torch.Tensor, *,
                 prec: str = "fp64", rblock: int | None = None, grid=None) -> tuple[float, float]:
    """(||Z - Theta C||_F^2, ||Z||_F^2) for the fit of minv (isdf_fit_residual)."""
    lib = L.load()
    psi, dt, pp, lp, npf, ps, lps, nps, aliased = _fit_common(phi, psi, idx)
    n_r, n_mu = phi.shape[0], idx.numel()
    g = _grid(grid, n_r, (1.0, 1.0, 1.0), geometry=False)
    rblock = min(n_r, 1 << 17) if rblock is None else rblock
    p = _prec(prec)
    dev = phi.device
    if minv.dtype != torch.float64 or minv.numel() < lib.isdf_fit_minv_elems(n_mu, int(aliased)):
        raise ValueError("minv too small or not float64")
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    info = torch.zeros(C.sizeof(L.FitInfo), dtype=torch.uint8, device=dev)
    wsb = lib.isdf_fit_residual_workspace(C.byref(g), n_mu, npf, nps, int(aliased), p, rblock)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    code = lib.isdf_fit_residual(C.byref(g), dt, pp, lp, npf, ps, lps, nps, idx.data_ptr(), n_mu, p,
                                 minv.data_ptr(), rblock, out.data_ptr(), info.data_ptr(), ws.data_ptr(), ws.numel(),
                                 _stream_handle())
    _check(code, "isdf_fit_residual")
    torch.cuda.current_stream().synchronize()
    inf = _read_struct(info, L.FitInfo)
    if inf.status != L.OK:
        raise ISDFError(inf.status, "isdf_fit_residual")
    r = out.cpu().tolist()
    return r[0], r[1]


def cluster_residual(phi: torch.Tensor, psi: torch.Tensor | None, labels: torch.Tensor, idx: torch.Tensor, *,
                     grid=None) -> float:
    """Appendix A cluster residual R for K-means labels and interpolation
    points (isdf_cluster_residual); raises if any row had an invalid label."""
    lib = L.load()
    psi, dt, pp, lp, npf, ps, lps, nps, aliased = _fit_common(phi, psi, idx)
    n_r, n_mu = phi.shape[0], idx.numel()
    if labels.dtype != torch.int32 or not labels.is_contiguous() or labels.numel() != n_r:
        raise TypeError("labels must be a contiguous int32 tensor of N_r entries")
    g = _grid(grid, n_r, (1.0, 1.0, 1.0), geometry=False)
    out = torch.zeros(2, dtype=torch.float64, device=phi.device)
    ws = torch.empty(lib.isdf_cluster_residual_workspace(), dtype=torch.uint8, device=phi.device)
    code = lib.isdf_cluster_residual(C.byref(g), dt, pp, lp, npf, ps, lps, nps, labels.data_ptr(), idx.data_ptr(),
                                     n_mu, out.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle())
    _check(code, "isdf_cluster_residual")
    r = out.cpu().tolist()
    if r[1] != 0:
        raise ValueError(f"{int(r[1])} rows have a label outside [0, n_mu) or an invalid interpolation point")
    return r[0]


def poisson(theta: torch.Tensor, grid, h=(1.0, 1.0, 1.0)) -> torch.Tensor:
    """V_mu = int zeta_mu(r') / |r - r'| dr' for every column of Theta
    (isdf_poisson): theta [N_r][N_mu] real or complex, double or single, on
    the periodic grid `grid` (n or (n0, n1, n2)) with spacings h (Bohr)."""
    lib = L.load()
    if theta.dim() != 2 or theta.stride(1) != 1 or not theta.is_cuda:
        raise TypeError("theta must be a 2-D CUDA tensor with unit column stride")
    kinds = {torch.float64: (L.C128, 0), torch.float32: (L.C64, 0), torch.complex128: (L.C128, 1),
             torch.complex64: (L.C64, 1)}
    if theta.dtype not in kinds:
        raise TypeError("theta must be float64, float32, complex128 or complex64")
    dt, cplx = kinds[theta.dtype]
    n_r, n_mu = theta.shape
    g = L.make_grid(grid, h)
    if g.n[0] * g.n[1] * g.n[2] != n_r:
        raise ValueError("grid does not match the rows of theta")
    V = torch.empty(n_r, n_mu, dtype=theta.dtype, device=theta.device)
    wsb = lib.isdf_poisson_workspace(C.byref(g), n_mu, cplx)
    if wsb == 0:
        raise ISDFError(L.E_UNSUPPORTED, "isdf_poisson_workspace")
    ws = torch.empty(wsb, dtype=torch.uint8, device=theta.device)
    code = lib.isdf_poisson(C.byref(g), dt, theta.data_ptr(), theta.stride(0), n_mu, cplx, V.data_ptr(), n_mu,
                            ws.data_ptr(), ws.numel(), _stream_handle())
    _check(code, "isdf_poisson")
    return V


def exchange(phi: torch.Tensor, psi: torch.Tensor, idx: torch.Tensor, V: torch.Tensor, *,
             rblock: int | None = None, grid=None) -> torch.Tensor:
    """ISDF-compressed exchange W = V_X psi (isdf_exchange, eq. v2) from the
    potentials V of the fit's Theta (as returned by `poisson`)."""
    lib = L.load()
    psi, dt, pp, lp, npf, ps, lps, nps, _ = _fit_common(phi, psi, idx)
    n_r, n_mu = phi.shape[0], idx.numel()
    if V.shape != (n_r, n_mu) or V.stride(1) != 1 or V.device != phi.device:
        raise TypeError("V must be (N_r, n_mu) with unit column stride on the orbitals' device")
    want_real = torch.float64 if dt == L.C128 else torch.float32
    want_cplx = torch.complex128 if dt == L.C128 else torch.complex64
    if V.dtype not in (want_real, want_cplx):
        raise TypeError(f"V must be {want_real} or {want_cplx}")
    g = _grid(grid, n_r, (1.0, 1.0, 1.0), geometry=False)
    rblock = min(n_r, 1 << 16) if rblock is None else rblock
    W = torch.empty(n_r, nps, dtype=want_cplx, device=phi.device)
    wsb = lib.isdf_exchange_workspace(C.byref(g), n_mu, npf, nps, rblock)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=phi.device)
    code = lib.isdf_exchange(C.byref(g), dt, pp, lp, npf, ps, lps, nps, idx.data_ptr(), n_mu, V.data_ptr(),
                             V.stride(0), int(V.is_complex()), W.data_ptr(), nps, rblock, ws.data_ptr(), ws.numel(),
                             _stream_handle())
    _check(code, "isdf_exchange")
    return W
