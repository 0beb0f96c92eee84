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
the roofline of the dominant kernel (propagation) from HIP events; and the
CPU oracle's own throughput on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 FP32 lanes per clock x 2.4 GHz, non-packed VALU issue.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
# algorithmic VALU work per update of the propagation: one multiply (density
# = row factor x fastest-axis factor) and one add into the bin
OPS_PER_UPDATE = 2


def main():
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
              "communication, and multi-GPU runs are not part of this build.", file=sys.stderr)
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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    prop_ms = []

    def step(time_prop=False):
        f = vup.eval_grid(g, wl.model, wl.theta)
        e = vup.uniform_edges(f, wl.B)
        mm = vup.build_model_matrix(g, f, e, want_bin=False)
        if time_prop:
            ev[0].record(stream)
        P, _ = vup.propagate(mm, mu, sigma, None, "fp32", want_Z=False)
        if time_prop:
            ev[1].record(stream)
        mean, var, _ = vup.moments(mm, mu, sigma)
        mh, vh, ent = vup.ipsa(mm, P)
        return mm, P

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(time_prop=True)
        # event pair of the last step is read after the loop; collect per step
        ev[1].synchronize()
        prop_ms.append(ev[0].elapsed_time(ev[1]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the per-step event read adds a host sync per step; time the steps again
    # back to back without it for the headline number
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ms_step = (t3 - t2) * 1e3 / args.steps
    value = U / (ms_step * 1e-3)
    t_prop = float(np.mean(prop_ms)) * 1e-3
    achieved = OPS_PER_UPDATE * U / t_prop
    log(f"[bench] step {ms_step:.3f} ms (synced-per-step {1e3 * (t1 - t0) / args.steps:.3f} ms), "
        f"propagate {1e3 * t_prop:.3f} ms")

    result = {
        "metric": "cell-distribution updates/sec (FP32 densities, full VUP+IPSA step)",
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
                               "Gaussians, sigma~U[0.05,0.5], 4-sigma truncation",
                   "grid": list(wl.n), "B": wl.B, "K": wl.K, "updates_per_step": U},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                     "kernel": "k_propagate<FP32>", "kernel_ms": 1e3 * t_prop,
                     "ops_per_update": OPS_PER_UPDATE},
    }

    # ---- variants on the same workload -------------------------------------
    if not args.no_variants:
        mm, _ = step()
        torch.cuda.synchronize()
        variants = {}
        Ps = {}
        for prec in ("fp32", "bf16", "bf16x2", "fp8e4m3"):
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
            err = {}
            ke = ks[:64]
            Po64 = Po[:64]
            for prec, P in Ps.items():
                Pg = P[torch.from_numpy(ke).to(dev)].cpu().numpy().astype(np.float64)
                err[prec] = float(np.abs(Pg - Po64).sum(axis=1).max())
            result["error_vs_fp64_oracle"] = {"metric": "max column L1 of P over 64 sampled k",
                                              **err}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
