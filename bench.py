"""Throughput of the VUP/IPSA hot path on one MI355X.

One step = the whole path over one batch of synthetic input, all resident in
HBM before timing starts:
    model evaluation on the grid -> uniform bin edges -> model matrix (bins,
    bin map, compressed-by-bin sort) -> propagation of all K pdfs (FP32
    densities) -> exact-f moments -> IPSA variance / entropy.
Workload: 2-D grid 1024 x 1024 on [-3,3]^2, f = sin x + 0.5 cos 2y + xy/4,
B = 256 bins, K = 65536 isotropic Gaussians (means on the 256 x 256 midpoint
subgrid, sigma ~ U[0.05, 0.5], seed 11246002), truncated at 4 sigma.

value = cell-distribution updates per second = U / step time, with U the
exact number of (cell, distribution) pairs inside the truncation windows.

Also reported (same workload, same run): propagation alone at each density
precision, and forward + backward (propagate + IPSA + adjoint sweep), each
with its error against the FP64 oracle on a seeded sample of distributions;
the IPSA probability matrix, field lines and marginal over locations on the
step's P with their HBM rooflines; the IPSA example of Sec. 5.3 at its five
measurement uncertainties; the timing experiment of Sec. 4.1 (the whole
pipeline for L = 1 ... 1000 pdfs on 10^6 cells, wall clock); the Bayes
inversion of 64 distributions; the banded MFMA form on a tensor-product
family of the same grid size (shared sigma) with its MFMA roofline;
the roofline of the longest sweep kernel of the step (and of the other one)
from HIP events; and the CPU oracle's own throughput on a bounded sample.

Profiling helpers (rocprofv3 wraps the program; see profiles/):
  --kernels-once              one propagation and one moments launch on the
                              workload, then a plain 256 MiB copy (the
                              calibration dispatch for the byte counters)
  --summarize-traffic F W     FETCH_SIZE / WRITE_SIZE counter CSVs of two
                              --kernels-once runs -> profiles/traffic_grid1024.*
  --summarize-stats CSV OUT   rocprofv3 kernel_stats.csv -> markdown table
  --summarize-pmc OUT U CSV.. counter CSVs of --pmc passes over one
                              --kernels-once workload (U updates, as it
                              prints) -> markdown table of per-kernel counters
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 FP32 lanes per clock x 2.4 GHz, non-packed VALU issue.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
# algorithmic arithmetic per cell-distribution update, from the definitions:
#   propagation: density (row factor x fastest-axis factor) and its add into
#   the bin: 2 operations;
#   exact-f moments on the matrix cores: per cell and distribution the two
#   multiply-adds of the bilinear forms sum g (f - a) and sum g (f - a)^2
#   (4 flops at FP64 quality; the kernel forms them exactly from 33-bit and
#   27-bit fixed-point operands as 2 x 17 int8 digit products), the row
#   factors and shifts being per row and per tile.
OPS_PER_UPDATE = {"propagate": 2}
MOMENTS_FLOPS_PER_UPDATE = 4
MOMENTS_INT8_MACS_PER_UPDATE = 34
MFMA_FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
MFMA_INT8_PEAK_TOPS = 5000.0   # MI355X dense int8 matrix peak
KERNELS = {"propagate": "k_propagate_runs (run form) / k_propagate<FP32> (cell form)",
           "moments": "k_mt_tiles + k_mt_prep + k_mt_main (v_mfma_i32_16x16x64_i8 digit "
                      "products) + k_mt_final"}


def traffic_bytes(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a plain copy of
    known size), or None when that summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_grid1024.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    entry = rec.get("kernels", {}).get(kernel)
    if entry is None or entry.get("source_sha256") != source_sha256(kernel):
        return None
    return entry["hbm_bytes_per_launch"]


# sources each measured kernel is built from (its launch and its input layout)
KERNEL_SOURCES = {
    "propagate": ("k_sweep.hip", "k_grid.hip", "vup_device.hpp", "vup_internal.hpp"),
    "moments": ("k_mtiles.hip", "k_grid.hip", "vup_device.hpp", "vup_internal.hpp"),
    "ipsa": ("k_fields.hip", "vup_fields.hpp", "vup_device.hpp"),
}


def source_sha256(kernel="propagate"):
    """Digest of the kernel sources a kernel's counters depend on."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1908_11246_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernels_once(name="grid1024"):
    """One launch of each sweep kernel on a workload (propagation at every
    density precision the workload is measured at, moments, IPSA, adjoint),
    then a plain 256 MiB copy: the calibration dispatch of the byte counters."""
    import torch
    import paper_1908_11246_amd as vup
    import workloads
    wl = workloads.CONFIGS[name]()
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mu = torch.from_numpy(wl.mu).cuda()
    sigma = torch.from_numpy(wl.sigma).cuda()
    w = None if wl.weight is None else torch.from_numpy(wl.weight).cuda()
    win = vup.windows(g, mu, sigma)
    U = int(torch.prod((win[..., 1] - win[..., 0] + 1).clamp(min=0).to(torch.int64),
                       dim=-1).sum().item())
    print(f"kernels-once {name}: U = {U} cell-distribution updates per sweep", flush=True)
    f = vup.eval_grid(g, wl.model, wl.theta)
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, wl.B), want_bin=False)
    P, _ = vup.propagate(mm, mu, sigma, w, "fp32", want_Z=False)
    vup.moments(mm, mu, sigma, w)
    mh, _, _ = vup.ipsa(mm, P)
    if name != "grid1024":
        for prec in PRECISIONS[name][1:]:
            vup.propagate(mm, mu, sigma, w, prec, want_Z=False)
        one = torch.ones(wl.K, dtype=torch.float64, device="cuda")
        vup.ipsa_backward(mm, mu, sigma, w, P, mh, one, one)
    else:
        # the banded form on the tensor-product family of the same grid
        # (256 x 256 locations, shared sigma = 0.25)
        m = workloads.subgrid_midpoints(wl.lo[0], wl.hi[0], 256)
        s = np.full(256, 0.25)
        for prec in ("fp32", "bf16", "bf16x2"):
            vup.propagate_separable(mm, m, m, s, s, want_Z=False, precision=prec)
    torch.cuda.synchronize()
    src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)  # last dispatch: the calibration copy
    torch.cuda.synchronize()
    print(f"kernels-once {name} done", flush=True)


# density precisions each configuration is measured at (the first is FP32,
# the reference the others are compared with)
PRECISIONS = {"grid1024": ("fp32", "bf16", "bf16x2", "fp8e4m3"),
              "grid128_3d": ("fp32", "bf16", "bf16x2"),
              "grid48_4d": ("fp32", "fp8e4m3")}


CALIB_BYTES = 256 << 20
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
# LDS rates of the run loop's operations, per CU and clock, at the vendor
# clock: integer atomic adds to random addresses (measured on this part with a
# microbenchmark: 6.4 lanes per clock per CU) and the LDS bandwidth (128 bytes
# per clock per CU)
LDS_ATOMIC_PEAK = 6.4 * 256 * 2.4e9
LDS_BYTES_PEAK = 128 * 256 * 2.4e9


def runs_in_windows(runidx, rows, pitch, win):
    """Runs of equal bin that the 2-D windows hold, summed over the windows:
    per window row r, runidx[r][hi] - runidx[r][lo] + 1 (runidx: each cell's
    run within its row, [rows][pitch]; win: [K][2][2] inclusive bounds, empty
    windows (hi < lo) count 0), by prefix sums over the rows."""
    ri = (np.asarray(runidx).astype(np.int64) & 0xFFFF).reshape(rows, pitch)
    pre = np.zeros((rows + 1, pitch), dtype=np.int64)
    np.cumsum(ri, axis=0, out=pre[1:])
    r0, r1 = win[:, 0, 0].astype(np.int64), win[:, 0, 1].astype(np.int64)
    c0, c1 = win[:, 1, 0].astype(np.int64), win[:, 1, 1].astype(np.int64)
    ok = (r1 >= r0) & (c1 >= c0)
    r0, r1, c0, c1 = (np.where(ok, v, 0) for v in (r0, r1, c0, c1))
    cnt = (pre[r1 + 1, c1] - pre[r0, c1]) - (pre[r1 + 1, c0] - pre[r0, c0]) + (r1 - r0 + 1)
    return int(np.where(ok, cnt, 0).sum())


def _time_on(stream, fn, reps, batch=1):
    """Mean ms per fn() call, HIP events on the launch stream around `batch`
    back-to-back calls (so that short kernels are not timed with host gaps),
    averaged over reps."""
    import torch
    fn()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record(stream)
        for _ in range(batch):
            fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b) / batch)
    return float(np.mean(ts))


def _c_call(vup, name, *args):
    """A prepared C-ABI call (argument marshalling done once) that raises on error."""
    f = getattr(vup.lib(), name)

    def call():
        rc = f(*args)
        if rc != 0:
            raise RuntimeError(f"{name}: {vup.lib().vup_last_error().decode()}")
    return call


def ipsa_views(vup, mm, P, mu, sigma, stream, reps):
    """The IPSA probability matrix, field lines and marginal on the step's P
    (Sec. 5.2), and the Bayes inversion (Sec. 3) for 64 of the distributions:
    time and HBM roofline of each (algorithmic bytes per launch: what the
    kernel must read and write once)."""
    import torch
    K, B = P.shape
    e = mm.edges.cpu().numpy()
    rng_f = float(e[-1] - e[0])
    n_dy = 2 * B
    dy_lo, dy_w = -rng_f, 2 * rng_f / n_dy
    lv = (0.025, 0.5, 0.975)
    y = vup.eval_points("sincos2", mu[:, 0, :])
    Q, lost = vup.ipsa_matrix(mm, P, y, dy_lo, dy_w, n_dy)
    fl = vup.ipsa_fields(mm, P, y, lv)
    ws = torch.empty(max(vup.marginal_workspace_bytes(K, n_dy), 1), dtype=torch.uint8,
                     device=P.device)
    chunks_bytes = vup.marginal_workspace_bytes(K, n_dy)
    g_out = torch.empty(n_dy, dtype=torch.float64, device=P.device)
    y2 = torch.empty_like(y)
    v = lambda t: ctypes.c_void_p(t.data_ptr())
    sp = ctypes.c_void_p(stream.cuda_stream)
    mref = ctypes.byref(mm.mm)
    model = vup.make_model("sincos2")
    mu0 = mu[:, 0, :]
    lvc = (ctypes.c_double * len(lv))(*lv)
    P2 = torch.empty_like(P)
    dists = vup._dists(mu, sigma, None, 4.0)
    cases = {
        "eval_points": (_c_call(vup, "vup_eval_points", ctypes.byref(model), 2, K, v(mu0),
                                mu0.stride(0), v(y2), sp), K * (16 + 8), "k_eval_points"),
        "ipsa_matrix": (_c_call(vup, "vup_ipsa_matrix", mref, K, v(P), v(y), dy_lo, dy_w, n_dy,
                                v(Q), v(lost), sp),
                        K * B * 4 + K * 8 + K * n_dy * 4 + K * 8, "k_ipsa_matrix"),
        "ipsa_fields": (_c_call(vup, "vup_ipsa_fields", mref, K, v(P), v(y), len(lv), lvc,
                                v(fl["y_mode"]), v(fl["p_max"]), v(fl["quant"]), v(fl["dev"]),
                                v(fl["delta2"]), sp),
                        K * B * 4 + K * 8 + K * (4 + len(lv)) * 8, "k_ipsa_fields"),
        "marginalize_Q": (_c_call(vup, "vup_marginalize", K, n_dy, v(Q), None, v(ws),
                                  ws.numel(), v(g_out), sp),
                          K * n_dy * 4 + 2 * chunks_bytes + n_dy * 8,
                          "k_marg_partial + k_marg_combine"),
    }
    # Bayes inversion (Sec. 3) for 64 distributions spread over K: 64 x N FP32
    # posteriors plus per-bin posterior means
    n_sel = 64
    sel = torch.arange(0, K, K // n_sel, dtype=torch.int64, device=P.device)[:n_sel].contiguous()
    N = int(mm.mm.N)
    post = torch.empty((n_sel, N), dtype=torch.float32, device=P.device)
    pmean = torch.empty((n_sel, B, 2), dtype=torch.float64, device=P.device)
    Zc = torch.empty((K, 1), dtype=torch.float64, device=P.device)
    vup.lib().vup_propagate(mref, ctypes.byref(dists), 0, v(P2), v(Zc), sp)
    cases["posterior_64"] = (_c_call(vup, "vup_posterior", mref, ctypes.byref(dists), n_sel, v(sel),
                                     v(P2), v(Zc), v(post), v(pmean), sp),
                             n_sel * N * 4 + N * 2 + n_sel * B * 2 * 8,
                             "k_posterior + k_posterior_mean")
    out = {"n_dy": n_dy, "levels": list(lv), "timing": "HIP events around 20 back-to-back "
           "C-ABI calls on the launch stream, mean of reps"}
    for name, (fn, nbytes, kern) in cases.items():
        ms = _time_on(stream, fn, reps, batch=20)
        ach = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "roofline": {"bound": "hbm", "achieved": ach,
                                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                             "frac": ach / HBM_PEAK_GBS,
                                             "algorithmic_bytes": nbytes, "kernel": kern}}
    return out


MFMA_FP32_PEAK_TFLOPS = 157.3
MFMA_BF16_PEAK_TFLOPS = 2500.0  # dense


def separable_run(vup, workloads, stream, reps, keep=None):
    """The banded MFMA form on a tensor-product family at full scale: 1024^2
    grid on [-3,3]^2, sincos model, B = 256, 256 x 256 locations on the
    midpoint subgrid with one shared sigma = 0.25 per axis (4-sigma windows).
    Timed with HIP events around the whole separable call (factors, prefix
    sums, the run scatter and the MFMA contraction); the MFMA roofline counts
    the banded contraction's algorithmic flops 2 B M_y sum_mx |window_x(mx)|
    against that whole time, so its fraction is a lower bound for the
    contraction kernel. The same for the BF16 and split-BF16 contractions
    (against the dense BF16 MFMA peak); `keep` receives 64 sampled rows of
    each precision's P for the error against the oracle."""
    import torch
    n, lo, hi, B, M, sg = (1024, 1024), (-3.0, -3.0), (3.0, 3.0), 256, 256, 0.25
    g = vup.make_grid(n, lo, hi)
    f = vup.eval_grid(g, "sincos2")
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, B), want_bin=False)
    m = workloads.subgrid_midpoints(lo[0], hi[0], M)
    s = np.full(M, sg)
    P, Z, ws = vup.propagate_separable(mm, m, m, s, s, want_Z=False)
    # windows per axis from the library, U = sum over the family of |wx| |wy|
    mu1 = torch.zeros((M, 1, 2), dtype=torch.float64, device="cuda")
    mu1[:, 0, 0] = torch.from_numpy(m).cuda()
    mu1[:, 0, 1] = torch.from_numpy(m).cuda()
    win = vup.windows(g, mu1, torch.full_like(mu1, sg))
    wlen = (win[:, 0, :, 1] - win[:, 0, :, 0] + 1).clamp(min=0).to(torch.float64)
    wx, wy = wlen[:, 0], wlen[:, 1]
    U = float(wx.sum().item() * wy.sum().item())
    flops = 2.0 * B * M * float(wx.sum().item())
    out = {"workload": "1024^2 grid on [-3,3]^2, sincos model, B=256, 256x256 locations on "
                       "the midpoint subgrid, shared sigma=0.25, 4-sigma windows",
           "updates": U}
    rows = workloads.sample_indices(M * M, 64, 9)
    for prec, peak, kern in (("fp32", MFMA_FP32_PEAK_TFLOPS, "k_sep_gemm"),
                             ("bf16", MFMA_BF16_PEAK_TFLOPS, "k_sep_gemm_bf16<2, false>"),
                             ("bf16x2", MFMA_BF16_PEAK_TFLOPS, "k_sep_gemm_bf16<2, true> "
                              "(three BF16 products per term)")):
        ms = _time_on(stream, lambda: vup.propagate_separable(mm, m, m, s, s, ws=ws, want_Z=False,
                                                              precision=prec), reps)
        P, _, _ = vup.propagate_separable(mm, m, m, s, s, ws=ws, want_Z=False, precision=prec)
        torch.cuda.synchronize()
        if keep is not None:
            keep[prec] = P.cpu().numpy()[rows]
        ach = flops / (ms * 1e-3) / 1e12
        entry = {"ms": ms, "updates_per_s": U / (ms * 1e-3),
                 "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                              "frac": ach / peak, "algorithmic_flops": flops,
                              "kernel": f"vup_propagate_separable ({kern} + set-up, whole call)"}}
        if prec == "fp32":
            out.update(entry)
        else:
            out[prec] = entry
    if keep is not None:
        keep["rows"] = rows
        keep["m"] = m
    return out


def _errors_vs_fp64(orc, wl, b, e, Ps, mh_v, ks):
    """Errors of each precision's P (and of the IPSA quantities computed from
    it on the GPU) against the FP64 oracle on the sampled distributions ks;
    Ps[prec] and mh_v[prec] hold the GPU's rows ks only."""
    sub = wl.subset(ks)
    Po, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, sub.mu, sub.sigma, sub.weight)
    mo, vo, ho = orc.ipsa(Po, e)
    out = {"metric": f"max over {len(ks)} sampled distributions: column L1 of P, |d mean_hist|, "
                     "|d var_hist| / var_hist, |d entropy| (nats), against the FP64 oracle"}
    for prec, P in Ps.items():
        Pg = P.astype(np.float64)
        mg, vg, hg = mh_v[prec]
        out[prec] = {"P_L1": float(np.abs(Pg - Po).sum(axis=1).max()),
                     "mean_hist": float(np.abs(mg - mo).max()),
                     "var_hist_rel": float((np.abs(vg - vo) / vo).max()),
                     "entropy": float(np.abs(hg - ho).max())}
    return out


def config_runs(vup, workloads, name, stream, reps, keep):
    """A 3-D or 4-D configuration: propagation at each density precision the
    configuration names, and forward + backward (propagate + IPSA + adjoint
    sweep, with the mixture-weight gradient where there are mixtures), each
    with U / time and its fraction of the separable-form roofline
    R(d) = (VALU lane-op peak) / d. The columns and IPSA quantities of 64
    sampled distributions go to `keep` for the error against the FP64 oracle
    (computed in the CPU-oracle leg)."""
    import torch
    wl = workloads.CONFIGS[name]()
    D = wl.ndim
    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mu = torch.from_numpy(wl.mu).cuda()
    sg = torch.from_numpy(wl.sigma).cuda()
    w = None if wl.weight is None else torch.from_numpy(wl.weight).cuda()
    win = vup.windows(g, mu, sg)
    U = int(torch.prod((win[..., 1] - win[..., 0] + 1).clamp(min=0).to(torch.int64),
                       dim=-1).sum().item())
    f = vup.eval_grid(g, wl.model, wl.theta)
    mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, wl.B), want_bin=False)
    out = {"workload": f"{name}: {'x'.join(map(str, wl.n))} grid, {wl.model} model, B={wl.B}, "
                       f"K={wl.K}" + (f" {wl.C}-component mixtures" if wl.C > 1 else ""),
           "updates": U, "sweep_form": mm.sweep}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            ev[0].record(stream)
            r = fn()
            ev[1].record(stream)
            ev[1].synchronize()
            ts.append(ev[0].elapsed_time(ev[1]))
        return float(np.mean(ts)), r

    Ps, stats = {}, {}
    for prec in PRECISIONS[name]:
        ms, (P, _) = timed(lambda: vup.propagate(mm, mu, sg, w, prec, want_Z=False))
        Ps[prec] = P.cpu().numpy()
        stats[prec] = tuple(t.cpu().numpy() for t in vup.ipsa(mm, P))
        ups = U / (ms * 1e-3)
        out[f"propagate_{prec}"] = {"ms": ms, "updates_per_s": ups,
                                    "frac_of_R(d)": ups * D / VALU_PEAK_OPS}
    P32 = torch.from_numpy(Ps["fp32"]).cuda()
    one = torch.ones(wl.K, dtype=torch.float64, device="cuda")

    def fwd_bwd():
        P, _ = vup.propagate(mm, mu, sg, w, "fp32", want_Z=False)
        mh, _, _ = vup.ipsa(mm, P)
        return vup.ipsa_backward(mm, mu, sg, w, P, mh, one, one)

    ms, _ = timed(fwd_bwd)
    mh, _, _ = vup.ipsa(mm, P32)
    ms_b, _ = timed(lambda: vup.ipsa_backward(mm, mu, sg, w, P32, mh, one, one))
    # forward d lane-ops per update, adjoint 3d + 2 (three FMAs per axis and
    # the weight lookup-and-add), so the pair is bounded by peak / (4d + 2)
    ups = U / (ms * 1e-3)
    out["fwd_bwd_fp32"] = {"ms": ms, "backward_ms": ms_b, "updates_per_s": ups,
                           "frac_of_peak/(4d+2)": ups * (4 * D + 2) / VALU_PEAK_OPS,
                           "note": "U counted once; forward and adjoint each sweep U"
                                   + ("; gradients wrt mu, sigma and the mixture weights"
                                      if wl.C > 1 else "")}
    ks = workloads.sample_indices(wl.K, 64, 21)
    keep[name] = (wl, ks, {p: P[ks] for p, P in Ps.items()},
                  {p: tuple(a[ks] for a in v) for p, v in stats.items()})
    return out


def timing_study_runs(vup, workloads, reps):
    """The timing experiment of Sec. 4.1 as a synthetic run: for L pdfs on
    N = 10^6 cells, the whole VUP pipeline (model evaluation, bin edges, model
    matrix with its sweep-form choice, propagation of all L pdfs), wall clock
    with the device synchronised on both sides, best of `reps`. The paper's
    figures (other hardware, context only) are L = 1: 0.43 s and L = 1000:
    4.39 s on a Quadro P4000, excluding GPU initialisation."""
    import torch
    res = {}
    for L in (1, 10, 100, 1000):
        wl = workloads.timing_study(L)
        g = vup.make_grid(wl.n, wl.lo, wl.hi)
        mu = torch.from_numpy(wl.mu).cuda()
        sg = torch.from_numpy(wl.sigma).cuda()

        def run():
            f = vup.eval_grid(g, wl.model)
            mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, wl.B), want_bin=False)
            P, _ = vup.propagate(mm, mu, sg, None, "fp32", wl.n_sigma, want_Z=False)
            return P

        run()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        U = wl.N * L
        res[str(L)] = {"ms": best * 1e3, "updates": U, "updates_per_s": U / best}
    res["growth_L1_to_L1000"] = res["1000"]["ms"] / res["1"]["ms"]
    return res


def ipsa_example_runs(vup, workloads, stream, reps):
    """The IPSA example of Sec. 5.3 (N = 10^6 grid over (x, alpha), K = 1000
    locations, B = 1000) at each measurement uncertainty: model matrix once,
    then propagation, y(l), the IPSA matrix (2000 Delta-y cells) and the field
    lines, timed together with HIP events."""
    import torch
    res = {}
    for s_l in workloads.IPSA_EXAMPLE_SIGMAS:
        wl = workloads.ipsa_example(s_l)
        g = vup.make_grid(wl.n, wl.lo, wl.hi)
        f = vup.eval_grid(g, wl.model)
        mm = vup.build_model_matrix(g, f, vup.uniform_edges(f, wl.B), want_bin=False)
        mu = torch.from_numpy(wl.mu).to("cuda")
        sg = torch.from_numpy(wl.sigma).to("cuda")
        win = vup.windows(g, mu, sg, wl.n_sigma)
        U = int(torch.prod((win[..., 1] - win[..., 0] + 1).to(torch.int64), dim=-1).sum().item())
        e = mm.edges.cpu().numpy()
        rng_f = float(e[-1] - e[0])

        def run():
            P, _ = vup.propagate(mm, mu, sg, None, "fp32", wl.n_sigma, want_Z=False)
            y = vup.eval_points("ipsa2", mu[:, 0, :])
            vup.ipsa_matrix(mm, P, y, -rng_f, rng_f / 1000, 2000)
            vup.ipsa_fields(mm, P, y, (0.025, 0.5, 0.975))

        ms = _time_on(stream, run, reps)
        # the alpha factor is shared by all locations: the same propagation in
        # the banded MFMA form (M_x = 1000 locations, M_y = 1), and the
        # general propagation alone for comparison
        mux = wl.mu[:, 0, 0].copy()
        sgx = wl.sigma[:, 0, 0].copy()
        _, _, ws = vup.propagate_separable(mm, mux, [0.0], sgx, [0.25], wl.n_sigma, want_Z=False)
        ms_sep = _time_on(stream, lambda: vup.propagate_separable(mm, mux, [0.0], sgx, [0.25],
                                                                   wl.n_sigma, ws=ws,
                                                                   want_Z=False), reps)
        ms_prop = _time_on(stream, lambda: vup.propagate(mm, mu, sg, None, "fp32", wl.n_sigma,
                                                          want_Z=False), reps)
        res[str(s_l)] = {"ms": ms, "updates": U, "updates_per_s": U / (ms * 1e-3),
                         "sweep_form": mm.sweep, "propagate_ms": ms_prop,
                         "propagate_separable_ms": ms_sep}
    return res
# kernel-name fragments of the sweep kernels in rocprofv3 output
TRACE_NAMES = {"propagate": "k_propagate_runs", "moments": "k_mt_main", "ipsa": "k_ipsa<"}


def _counter_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def summarize_traffic(fetch_csv, write_csv):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the sweep kernels, scaled
    by the ratio of the known byte count of the calibration copy (the last
    dispatch) to what the same counter reports for it."""
    out = {"workload": "grid1024", "calibration_bytes": CALIB_BYTES, "kernels": {}}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _counter_rows(path) if r["Counter_Name"] == counter]
        by_dispatch = {}
        for r in rows:
            d = int(r["Dispatch_Id"])
            by_dispatch.setdefault(d, [r["Kernel_Name"], 0.0])
            by_dispatch[d][1] += float(r["Counter_Value"])
        last = max(by_dispatch)
        calib_kib = by_dispatch[last][1]
        scale = CALIB_BYTES / (calib_kib * 1024.0)
        out[f"{counter.lower()}_calibration"] = {"kernel": by_dispatch[last][0][:120],
                                                 "counter_kib": calib_kib, "scale": scale}
        for key, frag in TRACE_NAMES.items():
            vals = [v for name, v in by_dispatch.values() if frag in name]
            if vals:
                per.setdefault(key, {})[counter] = vals[0] * 1024.0 * scale
    for key, v in per.items():
        if "FETCH_SIZE" in v and "WRITE_SIZE" in v:
            out["kernels"][key] = {"fetch_bytes": v["FETCH_SIZE"], "write_bytes": v["WRITE_SIZE"],
                                   "hbm_bytes_per_launch": v["FETCH_SIZE"] + v["WRITE_SIZE"],
                                   "source_sha256": source_sha256(key)}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "traffic_grid1024.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


# counter-derived fractions: GRBM_GUI_ACTIVE counts busy cycles on each of the
# 8 XCDs (rocprofv3 sums the instances); a CU issues at most one wave64 VALU
# instruction per cycle (four SIMDs, 16 lanes, four cycles each), so
#   VALU issue   = SQ_INSTS_VALU / (256 CUs x cycles)
#   VALU busy    = 4 SQ_ACTIVE_INST_VALU (quad-cycles) / (1024 SIMDs x cycles)
#   LDS conflict = SQ_LDS_BANK_CONFLICT / (256 CUs x cycles)
#   MFMA busy    = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x cycles)
N_XCD, N_CU, N_SIMD = 8, 256, 1024
SWEEP_FRAGMENTS = ("k_propagate", "k_moments", "k_backward", "k_mt_main")


def summarize_pmc(out_path, updates, csv_paths):
    """Per-dispatch hardware counters of rocprofv3 --pmc passes over one
    --kernels-once run each (same dispatch order in every pass), merged into a
    markdown table with the fractions above and, for the sweep kernels (each
    sweeps every update once), VALU and LDS lane-instructions per update."""
    disp = {}
    for i, path in enumerate(csv_paths):
        for r in _counter_rows(path):
            d = int(r["Dispatch_Id"])
            e = disp.setdefault(d, {"name": r["Kernel_Name"], "p": {}})
            key = (r["Counter_Name"], i)  # summed over the instances (XCDs) of one pass
            e["p"][key] = e["p"].get(key, 0.0) + float(r["Counter_Value"])
    for e in disp.values():
        # a counter taken in several passes (GRBM_GUI_ACTIVE) is averaged over them
        acc = {}
        for (cname, _), v in e["p"].items():
            acc.setdefault(cname, []).append(v)
        e["c"] = {cname: sum(v) / len(v) for cname, v in acc.items()}
    lines = ["| kernel | cycles / XCD | waves | VALU instr | VALU issue | VALU busy | "
             "LDS instr | LDS bank-conflict | MFMA busy | VALU lane-instr / update | "
             "LDS lane-instr / update |", "|---" * 11 + "|"]

    def f(v, fmt):
        return "—" if v is None else format(v, fmt)
    for d in sorted(disp):
        name, c = disp[d]["name"], disp[d]["c"]
        if not name.startswith(("vup::", "void vup::")) or c.get("SQ_WAVES", 1.0) < 256:
            continue
        short = name[5:] if name.startswith("void ") else name
        short = short.replace("(anonymous namespace)::", "").split("(")[0]
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / N_XCD or None
        get = c.get
        valu_issue = get("SQ_INSTS_VALU") / (N_CU * cyc) if cyc and "SQ_INSTS_VALU" in c else None
        valu_busy = (4 * get("SQ_ACTIVE_INST_VALU") / (N_SIMD * cyc)
                     if cyc and "SQ_ACTIVE_INST_VALU" in c else None)
        conf = (get("SQ_LDS_BANK_CONFLICT") / (N_CU * cyc)
                if cyc and "SQ_LDS_BANK_CONFLICT" in c else None)
        mfma = (get("SQ_VALU_MFMA_BUSY_CYCLES") / (N_SIMD * cyc)
                if cyc and "SQ_VALU_MFMA_BUSY_CYCLES" in c else None)
        sweep = any(t in short for t in SWEEP_FRAGMENTS) and updates
        vpu = 64 * get("SQ_INSTS_VALU") / updates if sweep and "SQ_INSTS_VALU" in c else None
        lpu = 64 * get("SQ_INSTS_LDS") / updates if sweep and "SQ_INSTS_LDS" in c else None
        lines.append(f"| `{short[:60]}` | {f(cyc, '.4g')} | {f(get('SQ_WAVES'), '.0f')} | "
                     f"{f(get('SQ_INSTS_VALU'), '.4g')} | {f(valu_issue, '.3f')} | "
                     f"{f(valu_busy, '.3f')} | {f(get('SQ_INSTS_LDS'), '.4g')} | {f(conf, '.3f')} | "
                     f"{f(mfma, '.3f')} | {f(vpu, '.2f')} | {f(lpu, '.2f')} |")
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1908_11246_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    text = "\n".join(lines) + f"\n\nKernel sources (csrc/, sorted) sha256: {h.hexdigest()}\n"
    with open(out_path, "w") as fh:
        fh.write(text)
    print(text)


def summarize_stats(csv_path, out_path):
    rows = _counter_rows(csv_path)
    lines = ["| kernel | calls | avg (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"][5:] if r["Name"].startswith("void ") else r["Name"]
        lines.append(f"| `{name[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f}% |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--kernels-once":
        return kernels_once(*sys.argv[2:3])
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-traffic":
        return summarize_traffic(sys.argv[2], sys.argv[3])
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-stats":
        return summarize_stats(sys.argv[2], sys.argv[3])
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-pmc":
        return summarize_pmc(sys.argv[2], float(sys.argv[3]), sys.argv[4:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the propagation shards over distributions with no "
              "communication, and runs on more than one GPU are not supported.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1908_11246_amd as vup
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda"
    wl = workloads.grid1024()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"[bench] workload {wl.name} n={wl.n} B={wl.B} K={wl.K}")

    g = vup.make_grid(wl.n, wl.lo, wl.hi)
    mu = torch.from_numpy(wl.mu).to(dev)
    sigma = torch.from_numpy(wl.sigma).to(dev)
    U = int(torch.prod((vup.windows(g, mu, sigma)[..., 1] - vup.windows(g, mu, sigma)[..., 0] + 1)
                       .to(torch.int64), dim=-1).sum().item())
    log(f"[bench] U = {U:.4e} cell-distribution updates per step")

    stream = torch.cuda.current_stream()
    parts = ["eval_grid", "edges", "model_matrix", "propagate", "moments", "ipsa"]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(parts) + 1)]

    # The FP32 sweep form is a property of the model matrix, identical in every
    # step: resolve it once (one stream sync, outside the timed steps) and set
    # it on each rebuilt matrix without a sync.
    f0 = vup.eval_grid(g, wl.model, wl.theta)
    mm0 = vup.build_model_matrix(g, f0, vup.uniform_edges(f0, wl.B), want_bin=False)
    form = mm0.sweep
    log(f"[bench] FP32 sweep form: {form}")
    # the tiled moments' workspace (per-pdf records and totals), allocated once
    mws = vup.moments_workspace(mm0, mu, sigma)

    def step(timed=False):
        mark = (lambda i: ev[i].record(stream)) if timed else (lambda i: None)
        mark(0)
        f = vup.eval_grid(g, wl.model, wl.theta)
        mark(1)
        e = vup.uniform_edges(f, wl.B)
        mark(2)
        mm = vup.build_model_matrix(g, f, e, want_bin=False, resolve_sweep=False)
        mm.set_sweep_mode(form)
        mark(3)
        P, _ = vup.propagate(mm, mu, sigma, None, "fp32", want_Z=False)
        mark(4)
        mean, var, _ = vup.moments(mm, mu, sigma, workspace=mws)
        mark(5)
        mh, vh, ent = vup.ipsa(mm, P)
        mark(6)
        return mm, P

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    part_ms = {k: [] for k in parts}
    for _ in range(args.steps):
        step(timed=True)
        ev[-1].synchronize()
        for i, k in enumerate(parts):
            part_ms[k].append(ev[i].elapsed_time(ev[i + 1]))
    part_ms = {k: float(np.mean(v)) for k, v in part_ms.items()}
    # headline: steps back to back, no per-step host sync
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ms_step = (t3 - t2) * 1e3 / args.steps
    value = U / (ms_step * 1e-3)
    log(f"[bench] step {ms_step:.3f} ms; parts (HIP events) " +
        ", ".join(f"{k} {v:.3f}" for k, v in part_ms.items()))
    # roofline of the longest sweep kernel of the step, and of the other one
    rooflines = {}
    t = part_ms["propagate"] * 1e-3
    ach = OPS_PER_UPDATE["propagate"] * U / t
    rooflines["propagate"] = {"bound": "alu", "achieved": ach / 1e12,
                              "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s",
                              "frac": ach / VALU_PEAK_OPS, "traffic": traffic_bytes("propagate"),
                              "kernel": KERNELS["propagate"], "kernel_ms": part_ms["propagate"],
                              "ops_per_update": OPS_PER_UPDATE["propagate"]}
    if form == "runs" and len(wl.n) == 2:
        # the run loop's own bound: per run of equal bin inside a window one
        # random LDS atomic and two 8-byte prefix-sum reads
        win = vup.windows(g, mu, sigma)[:, 0].cpu().numpy()
        R = runs_in_windows(mm0.runidx.cpu().numpy(), int(mm0.mm.rows), int(mm0.mm.pitch), win)
        rooflines["propagate"]["lds"] = {
            "runs_per_launch": R,
            "atomics_per_s": R / t, "atomic_peak_per_s": LDS_ATOMIC_PEAK,
            "atomic_frac": R / t / LDS_ATOMIC_PEAK,
            "read_bytes_per_s": 16 * R / t, "read_peak_bytes_per_s": LDS_BYTES_PEAK,
            "read_frac": 16 * R / t / LDS_BYTES_PEAK,
            "peaks": "random-address ds_add_u32 rate measured on this part (6.4 lanes/clk/CU) "
                     "and LDS bandwidth (128 B/clk/CU), at 2.4 GHz"}
        log(f"[bench] run loop: {R:.3e} runs, LDS atomics "
            f"{rooflines['propagate']['lds']['atomic_frac']:.2f} and prefix-sum reads "
            f"{rooflines['propagate']['lds']['read_frac']:.2f} of their peaks")
    # moments: the algorithmic flops of the two FP64-quality bilinear forms
    # over the whole moments call (its four kernels), against the dense FP64
    # matrix peak; beside it the int8 digit products executed, against the
    # dense int8 peak
    t = part_ms["moments"] * 1e-3
    ach = MOMENTS_FLOPS_PER_UPDATE * U / t / 1e12
    ach8 = 2 * MOMENTS_INT8_MACS_PER_UPDATE * U / t / 1e12
    rooflines["moments"] = {"bound": "mfma", "achieved": ach, "peak": MFMA_FP64_PEAK_TFLOPS,
                            "unit": "TFLOP/s", "frac": ach / MFMA_FP64_PEAK_TFLOPS,
                            "traffic": traffic_bytes("moments"), "kernel": KERNELS["moments"],
                            "kernel_ms": part_ms["moments"],
                            "flops_per_update": MOMENTS_FLOPS_PER_UPDATE,
                            "int8_ops": {"achieved": ach8, "peak": MFMA_INT8_PEAK_TOPS,
                                         "unit": "TOP/s", "frac": ach8 / MFMA_INT8_PEAK_TOPS,
                                         "macs_per_update": MOMENTS_INT8_MACS_PER_UPDATE}}
    # the IPSA column statistics stream P once: HBM bound, K*B*4 bytes read
    # plus mean, variance and entropy (3*K*8 bytes) written
    ipsa_bytes = wl.K * wl.B * 4 + 3 * wl.K * 8
    ach = ipsa_bytes / (part_ms["ipsa"] * 1e-3) / 1e9
    rooflines["ipsa"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": traffic_bytes("ipsa"),
                         "kernel": "k_ipsa", "kernel_ms": part_ms["ipsa"],
                         "algorithmic_bytes": ipsa_bytes}
    dominant = max(("propagate", "moments"), key=lambda k: part_ms[k])

    result = {
        "metric": "cell\u00b7distribution updates/sec (FP32 vs BF16 vs fwd+bwd) at stated error",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "grid1024: 2-D 1024x1024, sincos model, B=256, K=65536 "
                               "Gaussians, sigma~U[0.05,0.5], 4-sigma truncation; value = "
                               "FP32 full VUP+IPSA step (BF16 and fwd+bwd in variants, "
                               "errors in error_vs_fp64_oracle)",
                   "grid": list(wl.n), "B": wl.B, "K": wl.K, "updates_per_step": U},
        "roofline": rooflines[dominant],
        "rooflines": rooflines,
        "step_parts_ms": part_ms,
        "sweep_form": form,
    }

    # ---- variants on the same workload -------------------------------------
    ev = ev[:2]
    kept = {}
    if not args.no_variants:
        mm, _ = step()
        torch.cuda.synchronize()
        variants = {}
        Ps = {}
        stats = {}
        for prec in PRECISIONS["grid1024"]:
            vup.propagate(mm, mu, sigma, None, prec, want_Z=False)
            torch.cuda.synchronize()
            times = []
            for _ in range(max(3, args.steps // 2)):
                ev[0].record(stream)
                P, _ = vup.propagate(mm, mu, sigma, None, prec, want_Z=False)
                ev[1].record(stream)
                ev[1].synchronize()
                times.append(ev[0].elapsed_time(ev[1]))
            Ps[prec] = P
            stats[prec] = tuple(t.cpu().numpy() for t in vup.ipsa(mm, P))
            t = float(np.mean(times)) * 1e-3
            variants[f"propagate_{prec}"] = {"updates_per_s": U / t, "ms": 1e3 * t}
        # forward + backward: propagate + IPSA + adjoint sweep
        gv = torch.ones(wl.K, dtype=torch.float64, device=dev)
        ge = torch.ones(wl.K, dtype=torch.float64, device=dev)
        times = []
        for i in range(max(3, args.steps // 2) + 1):
            ev[0].record(stream)
            P, _ = vup.propagate(mm, mu, sigma, None, "fp32", want_Z=False)
            mh, vh, ent = vup.ipsa(mm, P)
            gm, gs, _ = vup.ipsa_backward(mm, mu, sigma, None, P, mh, gv, ge)
            ev[1].record(stream)
            ev[1].synchronize()
            if i:
                times.append(ev[0].elapsed_time(ev[1]))
        t = float(np.mean(times)) * 1e-3
        variants["fwd_bwd_fp32"] = {"updates_per_s": U / t, "ms": 1e3 * t,
                                    "note": "U counted once; forward and adjoint each sweep U"}
        result["variants"] = variants
        result["ipsa_views"] = ipsa_views(vup, mm, Ps["fp32"], mu, sigma, stream,
                                          max(3, args.steps // 2))
        sep_keep = {}
        sep = separable_run(vup, workloads, stream, max(3, args.steps // 2), sep_keep)
        variants["propagate_separable"] = sep
        log(f"[bench] separable (banded MFMA) FP32 {sep['ms']:.3f} ms, "
            f"{sep['updates_per_s']:.3e} updates/s, MFMA frac {sep['roofline']['frac']:.3f}; "
            f"BF16 {sep['bf16']['ms']:.3f} ms, split BF16 {sep['bf16x2']['ms']:.3f} ms")
        result["ipsa_example"] = ipsa_example_runs(vup, workloads, stream,
                                                   max(3, args.steps // 2))
        log("[bench] IPSA views " + ", ".join(
            f"{k} {v['ms']:.3f} ms" for k, v in result["ipsa_views"].items()
            if isinstance(v, dict)))
        for name in ("grid128_3d", "grid48_4d"):
            variants[name] = config_runs(vup, workloads, name, stream, max(3, args.steps // 2),
                                         kept)
            log(f"[bench] {name}: " + ", ".join(
                f"{k} {v['ms']:.3f} ms" for k, v in variants[name].items()
                if isinstance(v, dict) and "ms" in v))
        result["timing_study"] = timing_study_runs(vup, workloads, 3)
        log("[bench] Sec. 4.1 timing study (whole pipeline, wall clock) " + ", ".join(
            f"L={k}: {v['ms']:.3f} ms" for k, v in result["timing_study"].items()
            if isinstance(v, dict)) +
            f"; growth L=1 -> 1000: x{result['timing_study']['growth_L1_to_L1000']:.2f}")
        log("[bench] Sec. 5.3 example " + ", ".join(
            f"sigma_l={k}: {v['ms']:.3f} ms" for k, v in result["ipsa_example"].items()))
    else:
        Ps = None

    # ---- CPU oracle baseline + sampled error --------------------------------
    if not args.no_cpu_baseline:
        import oracle as orc
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        f = orc.eval_grid(wl.n, wl.lo, wl.hi, wl.model, wl.theta)
        e = orc.uniform_edges(f, wl.B)
        b = orc.bins(f, e)
        # calibrate on a small sample, then size the timed sample to the target
        ks = workloads.sample_indices(wl.K, 128, 7)
        sub = wl.subset(ks)
        t0 = time.perf_counter()
        orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, sub.mu, sub.sigma, nthreads=nthreads)
        tc = time.perf_counter() - t0
        nks = int(min(wl.K, max(128, 128 * args.cpu_seconds / max(tc, 1e-3))))
        ks = workloads.sample_indices(wl.K, nks, 8)
        sub = wl.subset(ks)
        _, _, Us = orc.windows(wl.n, wl.lo, wl.hi, sub.mu, sub.sigma)
        t0 = time.perf_counter()
        Po, _ = orc.propagate(wl.n, wl.lo, wl.hi, b, wl.B, sub.mu, sub.sigma, nthreads=nthreads)
        tc = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": Us / tc, "unit": "updates/s", "cores": nthreads, "kind": "oracle",
            "sample": f"FP64 oracle propagation of {nks} of {wl.K} distributions "
                      f"(seeded sample, {Us:.3e} updates, {tc:.1f} s)"}
        log(f"[bench] cpu oracle {Us / tc:.3e} updates/s on {nthreads} threads ({tc:.1f} s)")
        if Ps is not None:
            ke = workloads.sample_indices(wl.K, 64, 8)
            result["error_vs_fp64_oracle"] = _errors_vs_fp64(
                orc, wl, b, e, {p: P.cpu().numpy()[ke] for p, P in Ps.items()},
                {p: tuple(a[ke] for a in v) for p, v in stats.items()}, ke)
            # the banded form's precisions on its family (sampled rows)
            m_s, rows = sep_keep["m"], sep_keep["rows"]
            Msep = len(m_s)
            mu_s = np.zeros((len(rows), 1, 2))
            mu_s[:, 0, 0] = m_s[rows // Msep]
            mu_s[:, 0, 1] = m_s[rows % Msep]
            fs = orc.eval_grid((1024, 1024), (-3.0, -3.0), (3.0, 3.0), "sincos2")
            Pso, _ = orc.propagate((1024, 1024), (-3.0, -3.0), (3.0, 3.0),
                                   orc.bins(fs, orc.uniform_edges(fs, 256)), 256, mu_s,
                                   np.full_like(mu_s, 0.25))
            for prec in ("fp32", "bf16", "bf16x2"):
                err = float(np.abs(sep_keep[prec].astype(np.float64) - Pso).sum(axis=1).max())
                tgt = result["variants"]["propagate_separable"]
                (tgt if prec == "fp32" else tgt[prec])["P_L1_vs_fp64_oracle_64_rows"] = err
            for name, (wv, kv, Pv, sv) in kept.items():
                fo = orc.eval_grid(wv.n, wv.lo, wv.hi, wv.model, wv.theta)
                eo = orc.uniform_edges(fo, wv.B)
                result["variants"][name]["error_vs_fp64_oracle"] = _errors_vs_fp64(
                    orc, wv, orc.bins(fo, eo), eo, Pv, sv, kv)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
