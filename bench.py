#!/usr/bin/env python
"""ISDF benchmark on one MI355X: K-means + fit + adjoint of the 512-water workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload water512]
                    [--prec fp16x3] [--mixed fp64] [--side-steps 1] [--no-cpu-baseline]

One step = the whole hot path on inputs resident in HBM: SSM weight and
K-means (up to the workload's round count), factorisation and inverse of
C C^H (on a second stream, concurrent with Z C^H), then block by block
Z C^H (Gram products kept), Theta = Z C^H (C C^H)^-1 and that block's share
of the adjoint with the fused loss L = sum_r g_r sum_mu |Theta_r,mu|^2, and
finally the adjoint's terms at the interpolation rows.  The headline step
runs the orbital contractions in --prec (the 512-water workload is the
mixed-precision one: split FP16, FP64 factorisation and solve); each
precision of --mixed (FP64 by default) is timed beside it over --side-steps
steps, with its Theta error against the headline's.  Prints one JSON line;
phase times come from HIP events on the stream each phase runs on (the
factorisation overlaps Z C^H, so the phases add up to more than the step).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3}  # TFLOP/s, MI355X dense MFMA
HBM_PEAK = 8000.0  # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of what defines the solve GEMM: the kernel template (gemm.h) and
    the lines of fitlib.h that instantiate the FP64 tile configuration."""
    csrc = os.path.join(ROOT, "paper_2208_07731_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "gemm.h"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "fitlib.h")) as fh:
        for line in fh:
            if "launch_gemm<double, " in line:
                h.update(line.encode())
    return h.hexdigest()[:16]


def read_traffic(workload: str):
    """HBM traffic of the solve GEMM from the committed PMC summary, only if
    it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pmc_dgemm_apply_minv_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


MFMA_PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x6": 2500.0, "fp16x3": 2500.0}  # TFLOP/s, dense
ISSUED = {"fp64": 1, "fp32": 1, "bf16x6": 6, "fp16x3": 3}  # MFMA products per algorithmic product


def phase_rates(wl, prec: str, phases: dict, rounds: int, saved_gram: bool = False, km: dict | None = None) -> dict:
    """Algorithmic work of each phase, its rate and its fraction of the
    roofline that bounds it.

    kmeans : HBM bytes = weight pass (orbitals read once, w written) plus, per
             round, w read and, once, the labels written.
    factor : FLOPs of M = C C^H (real form) + Cholesky, triangular inverse and
             W = Y^T Y of the real n1 x n1 matrix (n1^3 / 3 each).
    zc     : 8 N_r N_mu (N_phi [+ N_psi]); split precisions issue 6x / 3x
             as many 16-bit MFMA products, against the 16-bit peak.
    solve  : 2 N_r n1^2 (FP64).
    adjoint: Gram recompute 8 N_r N_mu N (not when the forward kept the
             Gram blocks), orbital products Abar F and Abar^T X 16 N_r N_mu N,
             and the fused-loss products H = G^T g G over the lower half
             (N_r n1^2; in the split precision when the orbital products are)
             and S = G M^-2 (2 N_r n1^2, FP64).
    """
    n_e = wl.n_phi + (0 if wl.aliased else wl.n_psi)
    esize = 16
    n1 = wl.n_mu if wl.aliased else 2 * wl.n_mu
    out = {}
    km_bytes = wl.n_r * n_e * esize + 8 * wl.n_r + rounds * 8 * wl.n_r + 4 * wl.n_r
    ms = phases["kmeans"]
    gbs = km_bytes / (ms * 1e-3) / 1e9
    out["kmeans"] = {"ms": ms, "bound": "hbm", "bytes": km_bytes, "GB/s": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK, 4), "rounds": rounds,
                     "brute_force_pairs": (rounds + 1) * wl.n_r * wl.n_mu}
    if km is not None:  # what the pruned classification actually evaluated
        out["kmeans"]["evaluated_pairs"] = km.get("pairs_evaluated")
        out["kmeans"]["bound_tests"] = km.get("bound_tests")
    work = {
        "factor": (8.0 * wl.n_mu ** 2 * n_e + float(n1) ** 3, "fp64", 1),
        "zc": (8.0 * wl.n_r * wl.n_mu * n_e, prec, ISSUED[prec]),
        "solve": (2.0 * wl.n_r * n1 * n1, "fp64", 1),
    }
    for name, (flops, pk, issued) in work.items():
        ms = phases[name]
        tf = flops / (ms * 1e-3) / 1e12
        out[name] = {"ms": ms, "bound": "mfma", "flops": flops, "TFLOP/s": round(tf, 2), "peak": MFMA_PEAK[pk],
                     "frac": round(tf * issued / MFMA_PEAK[pk], 4)}
        if issued != 1:
            out[name]["issued_per_flop"] = issued
    # adjoint: the FP64 product with the inverse (S = G M^-2, 2 N_r n1^2),
    # H = G^T g G (N_r n1^2: FP64, or the split precision with split orbital
    # contractions) and the orbital products in the orbital precision; frac =
    # time the parts would take at their peaks over the measured time
    split = prec in ("bf16x6", "fp16x3")
    f64 = (2.0 if split else 3.0) * wl.n_r * n1 * n1
    orb = (16.0 if saved_gram else 24.0) * wl.n_r * wl.n_mu * n_e + (1.0 * wl.n_r * n1 * n1 if split else 0.0)
    ms = phases["adjoint"]
    t_peak = f64 / (MFMA_PEAK["fp64"] * 1e12) + orb * ISSUED[prec] / (MFMA_PEAK[prec] * 1e12)
    out["adjoint"] = {"ms": ms, "bound": "mfma", "flops": f64 + orb, "fp64_flops": f64, "orbital_flops": orb,
                      "orbital_prec": prec, "TFLOP/s": round((f64 + orb) / (ms * 1e-3) / 1e12, 2),
                      "frac": round(t_peak / (ms * 1e-3), 4)}
    return out


def poisson_leg(st, wl, steps, exchange=False) -> dict:
    """V_mu for every column of the step's Theta (isdf_poisson), HIP-event
    timed; algorithmic bytes: Theta read once and V written once, plus the
    four intermediate passes over the complex work array (real Theta packs
    two columns per complex signal)."""
    import torch

    from paper_2208_07731_amd import api

    h = wl.box_angstrom / 0.529177 / wl.n
    th = st.theta
    api.poisson(th, wl.n, (h, h, h))
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        v = api.poisson(th, wl.n, (h, h, h))
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    cols = th.shape[1] if th.is_complex() else (th.shape[1] + 1) // 2
    work = th.shape[0] * cols * 16
    io = th.numel() * th.element_size()
    nbytes = 2 * io + 8 * work  # 5 passes: Theta in, V out, 4 x (W in + W out) in between
    out = {"ms": round(ms, 3), "bound": "hbm", "bytes": nbytes, "GB/s": round(nbytes / ms / 1e6, 1),
           "frac": round(nbytes / ms / 1e6 / HBM_PEAK, 4), "columns": th.shape[1],
           "note": "includes the per-call workspace allocation by the Python wrapper"}
    if exchange:
        # exchange of eq. v2 on the step's own orbitals: Gram 8 N_r N_mu N_phi
        # plus the product with Psi_mu 8 N_r N_mu N_psi, FP64
        api.exchange(st.phi, st.psi, st.idx, v)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            w = api.exchange(st.phi, st.psi, st.idx, v)
        b.record()
        torch.cuda.synchronize()
        ms_x = a.elapsed_time(b) / steps
        flops = 8.0 * th.shape[0] * wl.n_mu * (wl.n_phi + wl.n_psi)
        out["exchange"] = {"ms": round(ms_x, 3), "bound": "mfma", "flops": flops,
                           "TFLOP/s": round(flops / ms_x / 1e9, 2), "peak": MFMA_PEAK["fp64"],
                           "frac": round(flops / ms_x / 1e9 / MFMA_PEAK["fp64"], 4)}
        del w
    del v
    return out


def qrcp_leg(phi, psi, wl, km_idx, km_ms, steps, sketch_rows=-1) -> dict:
    """Interpolation points by QRCP of Z^T (isdf_qrcp, eq. QRCP), the paper's
    baseline for K-means: HIP-event time of the whole selection, its
    algorithmic HBM bytes (each of the N_mu - 1 column steps reads the
    orbitals and the first k columns of L and writes column k and the
    residual diagonal), and the FP64 fit's least-squares residual at the QRCP
    points beside the K-means points'; then the randomized QRCP of a
    Khatri-Rao sketch of Z^T with sketch_rows rows (N_mu + 8 when negative,
    skipped when 0; isdf_qrcp_sketch), timed and fitted the same way."""
    import math

    import numpy as np
    import torch

    from paper_2208_07731_amd import api

    psi_arg = None if wl.aliased else psi
    api.qrcp(phi, psi_arg, wl.n_mu, grid=wl.n)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        r = api.qrcp(phi, psi_arg, wl.n_mu, grid=wl.n)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    esz = phi.element_size()
    cw = 8 if wl.aliased else 16
    orb = wl.n_r * (wl.n_phi + (0 if wl.aliased else wl.n_psi)) * esz
    nk = wl.n_mu - 1
    lread = wl.n_r * cw * nk * (nk - 1) / 2.0
    nbytes = nk * (orb + wl.n_r * (cw + 16)) + lread
    out = {"ms": round(ms, 2), "bound": "hbm", "bytes": nbytes, "GB/s": round(nbytes / ms / 1e6, 1),
           "frac": round(nbytes / ms / 1e6 / HBM_PEAK, 4), "rank": r.info["rank"],
           "near_ties": r.info["near_ties"], "r_last_over_r00": float(r.rdiag[-1] / r.rdiag[0]),
           "kmeans_ms": km_ms, "qrcp_over_kmeans_time": round(ms / km_ms, 1) if km_ms else None}
    # randomized QRCP (Khatri-Rao sketch with m rows, seeded normal)
    m = wl.n_mu + 8 if sketch_rows < 0 else sketch_rows
    if m == 0:
        rs = None
    else:
        rs = _qrcp_sketch_timed(phi, psi_arg, wl, m, steps, r, out)
    for name, idx in (("qrcp", r.idx), ("qrcp_sketch", rs.idx if rs is not None else None), ("kmeans", km_idx)):
        if idx is None:
            continue
        idx = idx[idx >= 0].contiguous()
        _, minv, info = api.fit(phi, psi_arg, idx, nrows=0)
        res, zz = api.fit_residual(phi, psi_arg, idx, minv, rblock=wl.rblock or None)
        out[f"{name}_ls_rel_residual"] = math.sqrt(max(res, 0.0) / zz)
        out[f"{name}_cc_pivot_ratio"] = info["pivot_max"] / info["pivot_min"] if info["pivot_min"] > 0 else None
        del minv
    torch.cuda.empty_cache()
    log(f"[bench] qrcp: {out}")
    return out


def _qrcp_sketch_timed(phi, psi_arg, wl, m, steps, r, out):
    """Warm-up plus `steps` timed calls of the randomized QRCP with m sketch
    rows; records the time and the overlap with the exact pivots in out."""
    import numpy as np
    import torch

    from paper_2208_07731_amd import api

    rng = np.random.default_rng(1000 * wl.cfg + 6)
    gp = torch.as_tensor(rng.standard_normal((wl.n_phi, m))).cuda()
    gs = torch.as_tensor(rng.standard_normal((wl.n_psi, m))).cuda()
    api.qrcp(phi, psi_arg, wl.n_mu, grid=wl.n, sketch=(gp, gs))
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        rs = api.qrcp(phi, psi_arg, wl.n_mu, grid=wl.n, sketch=(gp, gs))
    b.record()
    torch.cuda.synchronize()
    ms_s = a.elapsed_time(b) / steps
    out["sketch"] = {"m": m, "ms": round(ms_s, 2), "rank": rs.info["rank"],
                     "pivots_shared_with_exact": int(np.intersect1d(rs.idx.cpu().numpy(),
                                                                    r.idx.cpu().numpy()).size)}
    return rs


def weight_study(phi, psi, wl, d, kinds) -> dict:
    """K-means with each weight function (eq. weight function for PSM, eq.
    weight function 2 for alpha = 1..4), then the FP64 fit: the relative
    least-squares residual ||Z - Theta C|| / ||Z|| and Appendix A's cluster
    residual R / ||Z||^2 for each (the paper's SSM-vs-PSM comparison, on these
    synthetic orbitals).  Empty clusters are dropped before the fit."""
    import math

    import torch

    from paper_2208_07731_amd import api

    out = {}
    for kind in kinds:
        t0 = time.perf_counter()
        r = api.kmeans(phi, None if wl.aliased else psi, wl.n_mu, d["c0"], wl.kmeans_iters, grid=wl.n, weight=kind)
        live = r.idx >= 0
        lut = torch.cumsum(live.to(torch.int32), 0, dtype=torch.int32) - 1
        idx = r.idx[live].contiguous()
        labels = lut[r.labels.long()].to(torch.int32).contiguous()
        _, minv, info = api.fit(phi, None if wl.aliased else psi, idx, nrows=0)
        res, zz = api.fit_residual(phi, None if wl.aliased else psi, idx, minv, rblock=wl.rblock or None)
        R = api.cluster_residual(phi, None if wl.aliased else psi, labels, idx)
        out[kind] = {"n_mu": int(idx.numel()), "kmeans_rounds": r.info["iters"],
                     "ls_rel_residual": math.sqrt(max(res, 0.0) / zz), "cluster_residual_rel": R / zz,
                     "cc_pivot_ratio": info["pivot_max"] / info["pivot_min"] if info["pivot_min"] > 0 else None,
                     "seconds": round(time.perf_counter() - t0, 2)}
        log(f"[bench] weight {kind}: {out[kind]}")
        del minv
        torch.cuda.empty_cache()
    return out


def _host_description() -> dict:
    """CPU model and the thread settings the oracle's numpy/scipy ran with."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    return {"cpu_model": model, "nproc": os.cpu_count(), "threads_env": {k: v for k, v in env.items() if v}}


def cpu_baseline(d, idx, iters_run: int) -> dict:
    """The FP64 oracle on a bounded sample of the same workload, scaled to
    one full step (ms).

    Grids up to 64^3: weight at full size, two K-means rounds at full size
    (scaled to the rounds the GPU ran), and the fit and fused-loss adjoint on
    two sub-problems made of the interpolation rows plus 1024 / 3072 other
    grid rows, whose per-row slope is scaled to N_r.

    Larger grids (512-water): weight on the first 1/32 of the rows, one
    classification and update of 1/32 of the grid points against all
    centroids (scaled to the grid and to the rounds the GPU ran), the fit on
    256 and 1024 rows beside the interpolation rows (oracle.fit with
    `rows`: fixed part + per-row slope), and the adjoint once on the
    sub-problem of the interpolation rows plus 256 others, whose time less
    the fit's fixed part is scaled per row."""
    import numpy as np

    import oracle

    wl = d["wl"]
    phi, g = d["phi"], d["g"]
    pts = oracle.grid_points(wl.n)
    s = oracle.metric_scale()
    c = d["c0"]
    rng = np.random.default_rng(7)
    others = np.setdiff1d(np.arange(wl.n_r), idx)
    cores = len(os.sched_getaffinity(0))
    if wl.n_r <= 64 ** 3:
        t0 = time.perf_counter()
        w = oracle.weight(phi, None)
        t_w = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(2):
            lab, _, _ = oracle.assign(pts, c, s)
            c, _ = oracle.update(pts, w, lab, c)
        t_round = (time.perf_counter() - t0) / 2
        t_fit, t_bwd = [], []
        sizes = (1024, 3072)
        for extra in sizes:
            rows = np.concatenate([idx, rng.choice(others, extra, replace=False)])
            sub = np.ascontiguousarray(phi[rows])
            loc = np.arange(len(idx))
            t0 = time.perf_counter()
            oracle.fit(sub, sub, loc)
            t_fit.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            oracle.fit_backward(sub, sub, loc, g=g[rows])
            t_bwd.append(time.perf_counter() - t0)
        slope_f = (t_fit[1] - t_fit[0]) / (sizes[1] - sizes[0])
        slope_b = (t_bwd[1] - t_bwd[0]) / (sizes[1] - sizes[0])
        fix_f = t_fit[0] - slope_f * (len(idx) + sizes[0])
        fix_b = t_bwd[0] - slope_b * (len(idx) + sizes[0])
        sample = (f"numpy/scipy FP64 oracle on {cores} host threads: weight at full size, 2 of "
                  f"{iters_run + 1} K-means rounds at full size, fit and fused adjoint on sub-problems of "
                  f"N_mu+1024 and N_mu+3072 grid rows, extrapolated linearly in rows and rounds")
    else:
        frac = 32
        nw = wl.n_r // frac
        t0 = time.perf_counter()
        w = oracle.weight(np.ascontiguousarray(phi[:nw]), None)
        t_w = (time.perf_counter() - t0) * frac
        pk = rng.choice(wl.n_r, wl.n_r // frac, replace=False)
        wk = rng.uniform(0.5, 1.5, pk.size)  # weights only enter the update's sums
        t0 = time.perf_counter()
        lab, _, _ = oracle.assign(pts[pk], c, s)
        oracle.update(pts[pk], wk, lab, c)
        t_round = (time.perf_counter() - t0) * frac
        loc = np.arange(len(idx))
        t_fit = []
        sizes = (256, 1024)
        for extra in sizes:
            rows = rng.choice(others, extra, replace=False)
            t0 = time.perf_counter()
            oracle.fit(phi, phi, idx, rows=rows)
            t_fit.append(time.perf_counter() - t0)
        slope_f = (t_fit[1] - t_fit[0]) / (sizes[1] - sizes[0])
        fix_f = max(t_fit[0] - slope_f * sizes[0], 0.0)
        rows = np.concatenate([idx, rng.choice(others, 256, replace=False)])
        sub = np.ascontiguousarray(phi[rows])
        t0 = time.perf_counter()
        oracle.fit_backward(sub, sub, loc, g=g[rows])
        t_b = time.perf_counter() - t0
        fix_b = fix_f
        slope_b = max(t_b - fix_b, 0.0) / rows.size
        t_bwd = [t_b]
        sample = (f"numpy/scipy FP64 oracle on {cores} host threads: weight on 1/{frac} of the rows, one "
                  f"classification + update of 1/{frac} of the points against all {len(idx)} centroids, "
                  f"scaled to the grid and to {iters_run + 1} rounds; fit on 256 and 1024 rows beside the "
                  f"interpolation rows (fixed part + per-row slope); fused adjoint on the sub-problem of "
                  f"N_mu+256 rows, less the fit's fixed part, scaled per row; all extrapolated to N_r")
    total = t_w + t_round * (iters_run + 1) + (fix_f + slope_f * wl.n_r) + (fix_b + slope_b * wl.n_r)
    return {
        "value": round(total * 1e3, 1), "unit": "ms", "cores": cores, "kind": "oracle",
        "host": _host_description(), "sample": sample,
        "phases_s": {"weight": round(t_w, 3), "kmeans_round": round(t_round, 3),
                     "fit_rows_slope_us": round(slope_f * 1e6, 2), "bwd_rows_slope_us": round(slope_b * 1e6, 2),
                     "fit_sample_s": [round(t, 2) for t in t_fit], "bwd_sample_s": [round(t, 2) for t in t_bwd]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="water512")
    ap.add_argument("--prec", default="fp16x3",
                    help="orbital-contraction precision of the timed step (fp64, fp32, bf16x6, fp16x3)")
    ap.add_argument("--mixed", default="fp64",
                    help="comma-separated precisions timed beside --prec ('' to skip)")
    ap.add_argument("--side-steps", type=int, default=1, help="timed steps of each --mixed precision")
    ap.add_argument("--side-warmup", type=int, default=0, help="warm-up steps of each --mixed precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="time the step as replays of one captured HIP graph (phases still from eager steps)")
    ap.add_argument("--poisson", action="store_true",
                    help="also time V_mu (isdf_poisson) on the step's Theta")
    ap.add_argument("--exchange", action="store_true",
                    help="with --poisson: also time the ISDF-compressed exchange (isdf_exchange)")
    ap.add_argument("--qrcp", action="store_true",
                    help="also select the points by QRCP of Z^T (isdf_qrcp) and compare with K-means")
    ap.add_argument("--qrcp-sketch-rows", type=int, default=-1,
                    help="with --qrcp: rows m of the randomized QRCP's sketch (default N_mu + 8; 0 skips it)")
    ap.add_argument("--weight-study", default="",
                    help="comma-separated weight functions (ssm,psm,sm,scm,sqm) to compare by fit residuals")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the ISDF path here has no "
              f"multi-GPU mode.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2208_07731_amd.pipeline import ISDFStep

    torch.cuda.set_device(0)
    t0 = time.time()
    wl = synth.WORKLOADS[args.workload]
    d = synth.make_workload(args.workload, log=log)
    psi = torch.as_tensor(d["psi"]).cuda()
    phi = psi if wl.aliased else psi[:, : wl.n_phi]
    log(f"[bench] workload {wl.name}: N_r={wl.n_r} N_e={wl.n_phi} N_mu={wl.n_mu} ({time.time() - t0:.1f}s)")
    g = torch.as_tensor(d["g"]).cuda()
    if args.no_cpu_baseline:
        d["phi"] = d["psi"] = None  # the host copy is only needed by the oracle
    # grids whose Z C^H / Theta do not fit run the step in row blocks
    block_rows = wl.rblock or None
    torch.cuda.synchronize()
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst

    def run_graph(st, steps):
        """The step captured once as a HIP graph and replayed `steps` times."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            st.enqueue()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            st.enqueue()
        graph.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            graph.replay()
        b.record()
        torch.cuda.synchronize()
        st.check()
        return a.elapsed_time(b) / steps

    def run(prec, steps, warmup):
        slow = wl.n_r > (1 << 20)  # steps of seconds: progress lines while the GPU works
        st = ISDFStep(phi, None if wl.aliased else psi, wl.n_mu, d["c0"], wl.kmeans_iters, g=g, prec=prec,
                      block_rows=block_rows, keep_theta=block_rows is None)
        for w in range(warmup):
            st.enqueue()
            if slow:
                torch.cuda.synchronize()
                log(f"[bench] {prec}: warm-up step {w + 1} of {warmup} done")
        if warmup:
            st.check()
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        nb = len(st.blocks)
        blocks = [[(ev(), ev(), ev(), ev()) for _ in range(nb)] for _ in range(steps)]
        phases = [[ev() for _ in range(5)] for _ in range(steps)]
        factor = [(ev(), ev()) for _ in range(steps)]
        done = [ev() for _ in range(steps)]
        torch.cuda.synchronize()
        start, stop = ev(), ev()
        start.record()
        for k in range(steps):
            st.enqueue(block_events=blocks[k], phase_events=phases[k], factor_events=factor[k])
            done[k].record()
            if slow and k > 0:
                # one step stays queued while the host waits for the one before
                # it, so the GPU never idles; this only paces the progress lines
                done[k - 1].synchronize()
                log(f"[bench] {prec}: timed step {k} of {steps} done")
        stop.record()
        torch.cuda.synchronize()
        info = st.check()
        total = start.elapsed_time(stop) / steps
        zc_ms = sum(a.elapsed_time(b) for bl in blocks for a, b, _, _ in bl) / steps
        solve_ms = sum(b.elapsed_time(c) for bl in blocks for _, b, c, _ in bl) / steps
        adj_blk = sum(c.elapsed_time(e) for bl in blocks for _, _, c, e in bl) / steps
        el = lambda i: sum(p[i].elapsed_time(p[i + 1]) for p in phases) / steps  # noqa: E731
        factor_ms = sum(a.elapsed_time(b) for a, b in factor) / steps
        ph = {"kmeans": round(el(0), 3), "factor": round(factor_ms, 3), "zc": round(zc_ms, 3),
              "solve": round(solve_ms, 3), "adjoint": round(adj_blk + el(3), 3)}
        if args.graph:
            ph["eager_step"] = round(total, 3)
            total = run_graph(st, steps)
        return st, total, solve_ms / nb, ph, info

    log(f"[bench] {args.prec}: warmup {args.warmup}, timing {args.steps} steps")
    st, ms, solve_ms, phases, info = run(args.prec, args.steps, args.warmup)
    log(f"[bench] {args.prec}: {ms:.2f} ms/step, phases {phases}")
    n1 = wl.n_mu if wl.aliased else 2 * wl.n_mu
    nb = len(st.blocks)
    flops = 2.0 * (wl.n_r / nb) * n1 * n1  # per launch (row blocks of equal size)
    achieved = flops / (solve_ms * 1e-3) / 1e12
    traffic = read_traffic(wl.name)
    dtype = {"fp64": "f64", "fp32": "f32+f64", "bf16x6": "bf16x6+f64", "fp16x3": "f16x3+f64"}[args.prec]
    out = {
        "metric": "ISDF time (K-means+fit+bwd), % MFMA/HBM peak, mixed vs FP64 at 1e-6 rel err",
        "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.n}^3 grid (N_r={wl.n_r}), N_e={wl.n_phi}, N_mu={wl.n_mu}, "
                               f"{'Phi=Psi' if wl.aliased else 'Phi!=Psi'}, K-means {wl.kmeans_iters} rounds, "
                               f"fit + fused-loss adjoint, orbital contractions {args.prec}, FP64 C C^H solve"
                               + (f", streamed in blocks of {st.block_rows} rows" if nb > 1 else "")
                               + (" (Gram blocks kept for the adjoint)" if st.save_gram else ""),
                   "gram_prec": args.prec},
        "phases_ms": phases,
        "phases": phase_rates(wl, args.prec, phases, info["kmeans"]["iters"], st.save_gram, info["kmeans"]),
        "kmeans": {"rounds": info["kmeans"]["iters"], "converged": info["kmeans"]["converged"]},
        "roofline": {"bound": "mfma", "kernel": "FP64 GEMM Theta = (Z C^H)(C C^H)^-1 (one r-block per launch)",
                     "achieved": round(achieved, 2), "peak": PEAK["fp64"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK["fp64"], 4), "traffic": traffic,
                     "flops_per_launch": flops, "ms_per_launch": round(solve_ms, 3)},
    }
    if args.poisson:
        out["poisson"] = poisson_leg(st, wl, args.steps, args.exchange)
    if args.qrcp:
        out["qrcp"] = qrcp_leg(phi, psi, wl, st.idx.clone(), phases["kmeans"], 1,
                               sketch_rows=args.qrcp_sketch_rows)
    if args.mixed:
        theta_h = st.theta.clone()  # (the last block when streamed)
        del st
        torch.cuda.empty_cache()
        out["mixed"] = {}
        for prec in [p for p in args.mixed.split(",") if p]:
            log(f"[bench] {prec}: warmup {args.side_warmup}, timing {args.side_steps} steps")
            st2, ms2, _, ph2, _ = run(prec, args.side_steps, args.side_warmup)
            log(f"[bench] {prec}: {ms2:.2f} ms/step, phases {ph2}")
            th2 = st2.theta.to(theta_h.dtype)
            ref = th2 if prec == "fp64" else theta_h
            err = float(torch.linalg.norm(theta_h - th2) / torch.linalg.norm(ref))
            out["mixed"][prec] = {"steps": args.side_steps, "warmup": args.side_warmup, "ms_per_step": round(ms2, 3),
                                  "phases_ms": ph2, "zc": phase_rates(wl, prec, ph2, out["kmeans"]["rounds"])["zc"],
                                  "theta_rel_err_vs_timed_step": err,
                                  "timed_step_speedup": round(ms2 / ms, 3)}
            del st2, th2
            torch.cuda.empty_cache()
        del theta_h
    if args.weight_study:
        out["weight_study"] = weight_study(phi, psi, wl, d, [k for k in args.weight_study.split(",") if k])
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on a bounded sample)")
        c0 = np.asarray(d["c0"], dtype=np.int64)  # seeds are distinct grid points
        idx = (c0[:, 0] * wl.n + c0[:, 1]) * wl.n + c0[:, 2]
        out["cpu_baseline"] = cpu_baseline(d, idx, out["kmeans"]["rounds"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
