"""A whole ISDF step enqueued on one stream with preallocated buffers.

    step = ISDFStep(phi, psi, n_mu, c0, max_iter, g=g, prec="fp64")
    step.enqueue()          # K-means -> (C C^H)^-1 -> Z C^H -> Theta -> adjoint
    step.check()            # synchronises, raises on a device-side status

With block_rows < N_r the forward runs Z C^H and Theta block by block
(block_rows rows at a time); keep_theta=False then keeps only the current
block of Theta (the streamed form for grids whose Theta does not fit).

With the adjoint, each block's forward also keeps the Gram blocks
A = Phi Phi_mu^H (and B = Psi Psi_mu^H) beside Z C^H (isdf_zc_ab), and the
adjoint of that block runs right after its Theta from them
(isdf_fit_backward_rows, blocks in grid order, the last one applying the
interpolation-row terms), so no Gram product is computed twice and only one
block of G, A, B and Theta is ever held; save_gram=False instead runs the
whole adjoint after the forward, recomputing its Gram products in r-blocks
of `rblock` rows (isdf_fit_backward).

Nothing is allocated and nothing synchronises inside enqueue(): every
output, workspace and info struct is created in the constructor, and the
calls go straight to the C ABI on the current stream.  This is the form a
serving loop or a benchmark uses; the functions of `api` are the convenient
one-shot form.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .api import ISDFError, _orbital, _read_struct, _same


class ISDFStep:
    def __init__(self, phi: torch.Tensor, psi: torch.Tensor | None, n_mu: int, c0, max_iter: int, *,
                 g: torch.Tensor | None = None, prec: str = "fp64", grid=None, h=(1.0, 1.0, 1.0),
                 rblock: int | None = None, backward: bool = True, near_tie_rel: float = 1e-6,
                 block_rows: int | None = None, keep_theta: bool = True, save_gram: bool | None = None):
        self.lib = L.load()
        psi = phi if psi is None else psi
        self.phi, self.psi = phi, psi
        self.dt, self.pp, self.lp, self.npf = _orbital(phi, "phi")
        _, self.ps, self.lps, self.nps = _orbital(psi, "psi")
        self.aliased = _same(phi, psi)
        dev = phi.device
        n_r = phi.shape[0]
        if grid is None:
            n = round(n_r ** (1 / 3))
            grid = (n, n, n)
        self.grid = L.make_grid(grid, h)
        self.n_r, self.n_mu, self.max_iter, self.near = n_r, n_mu, max_iter, near_tie_rel
        self.prec = L.PRECS[prec]
        self.rblock = min(n_r, 1 << 17) if rblock is None else rblock
        self.backward = backward
        f64, i32, u8 = torch.float64, torch.int32, torch.uint8
        self.c0 = torch.as_tensor(c0, dtype=f64).to(dev).contiguous()
        self.idx = torch.empty(n_mu, dtype=i32, device=dev)
        self.cent = torch.empty(n_mu, 3, dtype=f64, device=dev)
        self.labels = torch.empty(n_r, dtype=i32, device=dev)
        self.w = torch.empty(n_r, dtype=f64, device=dev)
        self.km_info = torch.zeros(C.sizeof(L.KmeansInfo), dtype=u8, device=dev)
        self.km_ws = torch.empty(self.lib.isdf_kmeans_workspace(C.byref(self.grid), n_mu, max_iter), dtype=u8,
                                 device=dev)
        self.n1 = n_mu if self.aliased else 2 * n_mu
        self.minv = torch.empty(self.lib.isdf_fit_minv_elems(n_mu, int(self.aliased)), dtype=f64, device=dev)
        self.fit_info = torch.zeros(C.sizeof(L.FitInfo), dtype=u8, device=dev)
        self.fit_ws = torch.empty(self.lib.isdf_fit_workspace(C.byref(self.grid), n_mu, self.npf, self.nps,
                                                              int(self.aliased), self.prec, 1), dtype=u8, device=dev)
        # the factorisation runs on a second stream, beside Z C^H (they only
        # meet at the first solve); default priority like every other stream
        self.side = torch.cuda.Stream(device=dev)
        self.ev_km = torch.cuda.Event()
        self.ev_factor = torch.cuda.Event()
        self.block_rows = n_r if block_rows is None else min(int(block_rows), n_r)
        self.blocks = [(r, min(self.block_rows, n_r - r)) for r in range(0, n_r, self.block_rows)]
        self.keep_theta = keep_theta or len(self.blocks) == 1
        self.zc_ws = torch.empty(self.lib.isdf_zc_workspace(n_mu, self.npf, self.nps, int(self.aliased), self.prec,
                                                            self.block_rows), dtype=u8, device=dev)
        self.G = torch.empty(self.block_rows, self.n1, dtype=f64, device=dev)
        real_t = f64 if self.dt == L.C128 else torch.float32
        cplx_t = torch.complex128 if self.dt == L.C128 else torch.complex64
        self.theta = torch.empty(n_r if self.keep_theta else self.block_rows, n_mu,
                                 dtype=real_t if self.aliased else cplx_t, device=dev)
        if save_gram is None:
            save_gram = backward
        if save_gram and not backward:
            raise ValueError("save_gram needs the adjoint")
        self.save_gram = save_gram
        self.A = self.B = None
        if save_gram:
            self.A = torch.empty(self.block_rows, 2 * n_mu, dtype=f64, device=dev)
            self.B = None if self.aliased else torch.empty(self.block_rows, 2 * n_mu, dtype=f64, device=dev)
        if backward:
            if g is None:
                raise ValueError("the adjoint needs the loss field g")
            self.g = g.to(dev, f64).contiguous()
            self.dphi = torch.empty(n_r, self.npf, dtype=phi.dtype, device=dev)
            self.dpsi = self.dphi if self.aliased else torch.empty(n_r, self.nps, dtype=psi.dtype, device=dev)
            self.loss = torch.zeros((), dtype=f64, device=dev)
            self.bwd_info = torch.zeros(C.sizeof(L.FitInfo), dtype=u8, device=dev)
            if save_gram:
                wsb = self.lib.isdf_fit_backward_gram_workspace(C.byref(self.grid), n_mu, self.npf, self.nps,
                                                                int(self.aliased), self.prec, self.block_rows)
            else:
                wsb = self.lib.isdf_fit_backward_workspace(C.byref(self.grid), n_mu, self.npf, self.nps,
                                                           int(self.aliased), self.prec, self.rblock)
            self.bwd_ws = torch.empty(wsb, dtype=u8, device=dev)

    @staticmethod
    def _ptr(t):
        return None if t is None else t.data_ptr()

    def _call(self, code, where):
        if code != L.OK:
            raise ISDFError(code, where)

    def enqueue(self, block_events=None, phase_events=None, factor_events=None):
        """Enqueue the step on the current stream (the factorisation of C C^H
        forks onto a second stream right after K-means and joins back before
        the first solve).  block_events (one 4-tuple of events per row block)
        bracket each block's Z C^H, Theta and (kept Gram blocks) adjoint
        launches (with kept Gram blocks the adjoint runs block by block between
        the third and fourth event; otherwise those two coincide);
        phase_events (5 events) are recorded before K-means, after K-means,
        after the fork, after the last block, and after the adjoint that
        follows the blocks when the Gram blocks are recomputed (else right
        after the fourth); factor_events (2) bracket the factorisation on its
        own stream."""
        main = torch.cuda.current_stream()
        lib, s = self.lib, main.cuda_stream
        gp = C.byref(self.grid)
        ph = phase_events or [None] * 5

        def mark(i):
            if ph[i] is not None:
                ph[i].record()

        mark(0)
        self._call(lib.isdf_kmeans(gp, self.dt, self.pp, self.lp, self.npf, self.ps, self.lps, self.nps, 0, 0,
                                   self.n_mu, self.c0.data_ptr(), self.max_iter, self.near, self.idx.data_ptr(),
                                   self.cent.data_ptr(), self.labels.data_ptr(), self.w.data_ptr(), None,
                                   self.km_info.data_ptr(), self.km_ws.data_ptr(), self.km_ws.numel(), s),
                   "isdf_kmeans")
        mark(1)
        self.ev_km.record(main)
        self.side.wait_event(self.ev_km)
        if factor_events:
            factor_events[0].record(self.side)
        self._call(lib.isdf_fit(gp, self.dt, self.pp, self.lp, self.npf, self.ps, self.lps, self.nps,
                                self.idx.data_ptr(), self.n_mu, self.prec, self.minv.data_ptr(), L.FIT_FACTOR, 0, 0,
                                None, self.n_mu, 1, self.fit_info.data_ptr(), self.fit_ws.data_ptr(),
                                self.fit_ws.numel(), self.side.cuda_stream), "isdf_fit")
        if factor_events:
            factor_events[1].record(self.side)
        self.ev_factor.record(self.side)
        mark(2)
        esz = self.theta.element_size()
        for b, (r0, nrows) in enumerate(self.blocks):
            be = block_events[b] if block_events else None
            if be:
                be[0].record()
            if self.save_gram:
                self._call(lib.isdf_zc_ab(gp, self.dt, self.pp, self.lp, self.npf, self.ps, self.lps, self.nps,
                                          self.idx.data_ptr(), self.n_mu, self.prec, r0, nrows, self.G.data_ptr(),
                                          self.n1, self.A.data_ptr(), self._ptr(self.B), self.zc_ws.data_ptr(),
                                          self.zc_ws.numel(), s), "isdf_zc_ab")
            else:
                self._call(lib.isdf_zc(gp, self.dt, self.pp, self.lp, self.npf, self.ps, self.lps, self.nps,
                                       self.idx.data_ptr(), self.n_mu, self.prec, r0, nrows, self.G.data_ptr(),
                                       self.n1, self.zc_ws.data_ptr(), self.zc_ws.numel(), s), "isdf_zc")
            if be:
                be[1].record()
            if b == 0:
                main.wait_event(self.ev_factor)
            th = self.theta.data_ptr() + (r0 * self.n_mu * esz if self.keep_theta else 0)
            self._call(lib.isdf_apply_minv(self.n_mu, int(self.aliased), self.minv.data_ptr(), self.G.data_ptr(),
                                           self.n1, nrows, self.dt, th, self.n_mu, s), "isdf_apply_minv")
            if be:
                be[2].record()
            if self.backward and self.save_gram:
                # this block's share of the adjoint, from the Gram blocks just kept
                flags = (L.BWD_FIRST if b == 0 else 0) | (L.BWD_LAST if b == len(self.blocks) - 1 else 0)
                self._call(lib.isdf_fit_backward_rows(
                    gp, self.dt, self.pp, self.lp, self.npf, self.ps, self.lps, self.nps, self.idx.data_ptr(),
                    self.n_mu, self.prec, self.minv.data_ptr(), None, 0, self.g.data_ptr(), self.dphi.data_ptr(),
                    self.npf, self.dpsi.data_ptr(), self.nps, self.loss.data_ptr(), r0, nrows, self.block_rows,
                    self.G.data_ptr(), self.A.data_ptr(), self._ptr(self.B), flags, self.bwd_info.data_ptr(),
                    self.bwd_ws.data_ptr(), self.bwd_ws.numel(), s), "isdf_fit_backward_rows")
            if be:
                be[3].record()
        mark(3)
        if self.backward and not self.save_gram:
            self._call(lib.isdf_fit_backward(gp, self.dt, self.pp, self.lp, self.npf, self.ps, self.lps, self.nps,
                                             self.idx.data_ptr(), self.n_mu, self.prec, self.minv.data_ptr(), None,
                                             0, self.g.data_ptr(), self.dphi.data_ptr(), self.npf,
                                             self.dpsi.data_ptr(), self.nps, self.loss.data_ptr(), self.rblock,
                                             self.bwd_info.data_ptr(), self.bwd_ws.data_ptr(), self.bwd_ws.numel(),
                                             s), "isdf_fit_backward")
        mark(4)

    def check(self) -> dict:
        """Synchronise and return the device-side infos; raise on errors."""
        torch.cuda.current_stream().synchronize()
        out = {"kmeans": _read_struct(self.km_info, L.KmeansInfo), "fit": _read_struct(self.fit_info, L.FitInfo)}
        if self.backward:
            out["backward"] = _read_struct(self.bwd_info, L.FitInfo)
        km = out["kmeans"]
        if km.status not in (L.OK, L.W_EMPTY_CLUSTER):
            raise ISDFError(km.status, "isdf_kmeans")
        for k in ("fit", "backward"):
            if k in out and out[k].status != L.OK:
                raise ISDFError(out[k].status, f"isdf_{k}")
        return {k: {f: getattr(v, f) for f, _ in type(v)._fields_} for k, v in out.items()}
