#!/usr/bin/env python3
"""Packets reconstructed per second on one MI355X: FGGC against the direct sum.

    python bench.py [--steps K] [--warmup W] [--workload cfg1] [--no-cpu-baseline]

One step reconstructs one batch of packets, already resident in HBM, into the
wave function on the grid: pass A times K FGGC reconstructions
(fggc_reconstruct: correction, scatter, FFT over q, band multiply, inverse
FFT) and then K direct sums (fggc_direct_sum) of the same packets, each pass
bracketed by device synchronisations.  `value` is FGGC packets per second;
the direct sum's rate and the speedup sit beside it.  Pass B repeats both
with the library's per-stage HIP events on (fggc_profile) to time the kernels
for the roofline entry.  The CPU-baseline leg times the FP64 oracle on a
bounded sample of the same workload and checks the GPU results on that sample
against it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
FP64_PEAK_T = 78.6  # FP64 vector TFLOP/s
FP32_MFMA_PEAK_T = 157.3  # dense FP32 matrix-core TFLOP/s
# VALU issue slots: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one non-packed op per lane per cycle)
VALU_SLOT_PEAK_T = 256 * 64 * 2.4e9 / 1e12

WORKLOADS = {
    "cfg0": 0,
    "cfg1": 1,
    "cfg2": 2,
    "cfg3": 3,
}


def measured_traffic(workload, stage):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) of a stage, from the
    committed counter run of this workload -- None when there is none or when the
    kernel sources have changed since the counters were taken."""
    from paper_2504_21785_amd import rocprof_summary as RS
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != RS.source_digest():
        return None
    st = t.get("stages", {}).get(stage)
    if not st or "fetch_size_bytes" not in st or "write_size_bytes" not in st:
        return None
    return st["fetch_size_bytes"] + st["write_size_bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(u, ref):
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))


def fggc_alg_bytes(ps, st, slices, es=8):
    """Bytes the FGGC reconstruction must move: packets in, the cell array
    written and read, the grid spectrum written and read, u written."""
    d = ps.d
    nq = int(np.prod([st.Nq[k] for k in range(d)]))
    cells = slices * nq
    mpts = int(np.prod(ps.M))
    return ps.N * ((2 * d + 1) * 8 + 16) + 2 * cells * es + 3 * mpts * es


def direct_slots_per_pair(d):
    """Minimal VALU issue slots of one (packet, point) evaluation in the FP32
    path: displacement (d FMA), |y|^2 (d), exponent (1 FMA), window select (2),
    phase (d FP64 FMA + fract + convert), two FMAs of the accumulation, and
    three transcendentals (exp, sin, cos) at four slots each."""
    return d + d + 1 + 2 + (d + 2) + 2 + 3 * 4


def serving_bench(ctx, F, W, torch, n_pool, n_req, loads, n_streams):
    """Serving stream: a pool of distinct requests of the stream's distribution
    (device-resident), warmed so that each shape has run eagerly and been
    captured; the capacity from a closed batch of n_req submissions; then
    open-loop Poisson arrivals at each offered load (a fraction of that
    capacity), reporting p50/p99 latency (submit to completion) and packets/s."""
    log(f"serving: generating {n_pool} requests")
    pool = []
    for r in range(n_pool):
        ps = W.serving_request(r)
        st = F.default_strategy(ps.d, ps.eps, "Q4P2")
        dev = tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (ps.Q, ps.P, ps.S, ps.a))
        pool.append((ps, st, dev))
    torch.cuda.synchronize()
    srv = F.Server(ctx, n_streams)

    def submit(i):
        ps, st, dev = pool[i]
        return srv.submit(*dev, ps.eps, ps.M, st)

    def wait_all(tks):
        for tk, _ in tks:
            rc = srv.wait(tk, 300.0)
            if rc != F.FGGC_OK:
                raise RuntimeError(f"served request failed: {rc} {F.last_error()}")

    try:
        for _ in range(2):  # first sighting runs eagerly, the second captures its graph
            wait_all([submit(i) for i in range(n_pool)])
        rng = np.random.default_rng(W.BASE_SEED * 1000 + 4)
        srv.reset_stats()
        order = rng.integers(0, n_pool, n_req)
        t0 = time.perf_counter()
        wait_all([submit(int(i)) for i in order])
        t_cap = time.perf_counter() - t0
        cap = {"requests_per_s": n_req / t_cap,
               "packets_per_s": float(sum(pool[int(i)][0].N for i in order)) / t_cap,
               "graphs": srv.counters()}
        log("serving capacity:", cap)
        res = []
        for rho in loads:
            srv.reset_stats()
            lam = rho * cap["requests_per_s"]
            arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
            order = rng.integers(0, n_pool, n_req)
            tks = []
            t0 = time.perf_counter()
            for i in range(n_req):
                while True:
                    dt = arrivals[i] - (time.perf_counter() - t0)
                    if dt <= 0:
                        break
                    time.sleep(min(dt, 0.002) if dt > 0.0005 else 0)
                tks.append(submit(int(order[i])))
            wait_all(tks)
            s = srv.stats()
            r = {"offered_load": rho, "offered_requests_per_s": lam, "requests": n_req,
                 "p50_ms": s["p50_s"] * 1e3, "p99_ms": s["p99_s"] * 1e3,
                 "packets_per_s": s["packets_per_s"], "graphs": srv.counters()}
            log("serving load", rho, r)
            res.append(r)
    finally:
        srv.close()
    return {"workload": "cfg4: " + W.CONFIG_NAMES[4], "n_streams": n_streams, "pool_requests": n_pool,
            "mean_packets": float(np.mean([p[0].N for p in pool])), "capacity": cap, "loads": res}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg1", choices=sorted(WORKLOADS))
    ap.add_argument("--strategy", default=None, help="Q2P2, Q4P2, Q2P4 or Q4P4 (default Q4P2; Q2P2 in 3D)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream measurement")
    ap.add_argument("--cpu-points", type=int, default=4096,
                    help="grid points sampled by the oracle in 2D and 3D")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run a plain elementwise copy (read and write this many MiB) before timing, "
                         "to scale HBM counters read under a profiler")
    ap.add_argument("--serving-pool", type=int, default=48)
    ap.add_argument("--serving-requests", type=int, default=200)
    ap.add_argument("--serving-streams", type=int, default=4)
    ap.add_argument("--cpu-target-s", type=float, default=12.0,
                    help="approximate CPU seconds for the oracle sample")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_21785_amd import fggc as F
    from paper_2504_21785_amd import workloads as W

    k = WORKLOADS[args.workload]
    ps = W.config(k)
    log(f"generated {args.workload}: {ps.N} packets")
    d = ps.d
    sname = args.strategy or ("Q2P2" if d == 3 else "Q4P2")
    st = F.default_strategy(d, ps.eps, sname)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    Q, P, S, a = t(ps.Q), t(ps.P), t(ps.S), t(ps.a)
    ctx = F.Context(0)
    u_f = torch.empty(ps.M, dtype=torch.complex64, device=dev)
    u_d = torch.empty(ps.M, dtype=torch.complex64, device=dev)
    do_direct = True  # the direct sum on the whole grid (in 3D its parity is checked on a sub-box)

    def step_fggc():
        ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32, out=u_f)

    def step_direct():
        ctx.direct_sum(Q, P, S, a, ps.eps, ps.M, ps.R, precision=F.FP32, out=u_d)

    log(f"workload {args.workload}: d={d} N={ps.N} M={ps.M} eps={ps.eps} strategy={sname}")
    for i in range(args.warmup):
        step_fggc()
        if do_direct:
            step_direct()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1} of {args.warmup} done")

    if args.calib_copy_mb > 0:
        cx = torch.ones(args.calib_copy_mb << 18, dtype=torch.float32, device=dev)
        cy = torch.empty_like(cx)
        for _ in range(3):
            torch.mul(cx, 2.0, out=cy)
        torch.cuda.synchronize()
        del cx, cy

    # ---- pass A: timed steps -------------------------------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_fggc()
    torch.cuda.synchronize()
    fggc_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"FGGC: {fggc_ms:.4f} ms/step")
    direct_ms = None
    if do_direct:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_direct()
        torch.cuda.synchronize()
        direct_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        log(f"direct: {direct_ms:.4f} ms/step")

    # the separable (box-window, matrix-core) direct sum: 2D only
    sep = None
    if d == 2:
        u_s = torch.empty(ps.M, dtype=torch.complex64, device=dev)

        def step_sep():
            ctx.direct_sum_separable(Q, P, S, a, ps.eps, ps.M, ps.R, out=u_s)

        for _ in range(max(1, args.warmup)):
            step_sep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step_sep()
        torch.cuda.synchronize()
        sep_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        ctx.profile(True)
        for _ in range(args.steps):
            step_sep()
        torch.cuda.synchronize()
        kms, kcnt = ctx.stage_time("ds_kernel")
        ctx.profile(False)
        kms = kms / max(kcnt, 1)
        # algorithmic work: one complex multiply-add (8 flops) per (packet, point)
        # pair inside the box window
        pairs = ps.N * np.prod([2 * ps.R / (2 * math.pi / m) for m in ps.M])
        ach = pairs * 8 / (kms * 1e-3) / 1e12
        sep = {"value": ps.N / (sep_ms * 1e-3), "ms_per_step": sep_ms, "window": "box, half-width R",
               "roofline": {"kernel": "ds_sep2_kernel", "bound": "mfma", "achieved": ach,
                            "peak": FP32_MFMA_PEAK_T, "unit": "TFLOP/s", "frac": ach / FP32_MFMA_PEAK_T,
                            "pairs_per_launch": float(pairs), "avg_launch_ms": kms}}
        log(f"separable direct: {sep_ms:.4f} ms/step, kernel {kms:.4f} ms")

    # ---- pass B: per-stage HIP events ---------------------------------------
    ctx.profile(True)
    for _ in range(args.steps):
        step_fggc()
        if do_direct:
            step_direct()
    torch.cuda.synchronize()
    log("profiled pass done")
    stage_names = ["prepass", "fggc_sort", "fggc_coef", "fggc_accum", "fggc_fft_q",
                   "fggc_band_mac", "fggc_contract", "fggc_ifft", "ds_prep",
                   "ds_sort", "ds_kernel", "ds_reduce"]
    stages = {}
    for sn in stage_names:
        ms, cnt = ctx.stage_time(sn)
        if cnt:
            stages[sn] = {"avg_ms": ms / cnt, "launches": cnt}
    ctx.profile(False)
    log("stages:", json.dumps(stages))

    # FGGC vs direct on the full workload (GPU outputs only)
    fvd = None
    u_fggc = u_f.cpu().numpy()
    u_direct = u_d.cpu().numpy() if do_direct else None
    if do_direct:
        fvd = rel(u_fggc.astype(np.complex128), u_direct.astype(np.complex128))
        log(f"FGGC vs direct rel-L2 {fvd:.3e}")
    if sep is not None:
        u_sep = u_s.cpu().numpy().astype(np.complex128)
        sep["rel_l2_vs_direct"] = rel(u_sep, u_direct.astype(np.complex128))
        sep["fggc_rel_l2_vs_it"] = rel(u_fggc.astype(np.complex128), u_sep)
        sep["speedup_fggc_vs_it"] = sep["ms_per_step"] / fggc_ms

    # ---- roofline of the dominant FGGC kernel --------------------------------
    lo, n = ctx.cell_box(Q, P, S, a, st)
    slices = int(np.prod(n))
    fstages = {k2: v for k2, v in stages.items() if k2.startswith("fggc_")}
    dom = max(fstages, key=lambda s2: fstages[s2]["avg_ms"])
    nq = int(np.prod([st.Nq[i] for i in range(d)]))
    cells_b = slices * nq * 8
    mpts = int(np.prod(ps.M))
    n1 = int(st.nq * st.np)
    n1b = 4 if n1 <= 4 else (8 if n1 <= 8 else 16)
    rec_b = 16 * ((8 * d + 15) // 16) + d * n1b * 8
    ns = 1 if d == 1 else 2 ** d
    # (bound, amount per launch, unit of the amount, peak in that unit per second)
    per_launch = {
        # FP64: two complex n1 x n1 mat-vecs per dimension, rhs and shift, Kronecker weights
        "fggc_coef": ("alu", ps.N * (d * (16 * n1 * n1 + 60 * n1) + 6 * n1 ** d) / 1e12,
                      "TFLOP/s", FP64_PEAK_T),
        # records in, the dense cell array written once
        "fggc_accum": ("hbm", (ps.N * rec_b + cells_b) / 1e9, "GB/s", HBM_PEAK_GBS),
        # packets' Q and P in; keys, ranks and positions
        "fggc_sort": ("hbm", ps.N * (2 * d * 8 + 12 * ns) / 1e9, "GB/s", HBM_PEAK_GBS),
        "fggc_fft_q": ("hbm", 2 * cells_b / 1e9, "GB/s", HBM_PEAK_GBS),
        "fggc_band_mac": ("hbm", (cells_b + mpts * 8) / 1e9, "GB/s", HBM_PEAK_GBS),
        # separable finish (d >= 2): read the cell array, write the grid spectrum
        "fggc_contract": ("hbm", (cells_b + mpts * 8) / 1e9, "GB/s", HBM_PEAK_GBS),
        "fggc_ifft": ("hbm", 2 * mpts * 8 / 1e9, "GB/s", HBM_PEAK_GBS),
    }
    bound, amount, unit, peak = per_launch.get(dom, ("hbm", 0.0, "GB/s", HBM_PEAK_GBS))
    dom_ms = stages[dom]["avg_ms"]
    achieved = amount / (dom_ms * 1e-3)
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": measured_traffic(args.workload, dom),
                "algorithmic_per_launch": amount, "avg_launch_ms": dom_ms}
    direct_roofline = None
    if do_direct and "ds_kernel" in stages:
        ball = {1: 2 * ps.R, 2: math.pi * ps.R ** 2, 3: 4.0 / 3.0 * math.pi * ps.R ** 3}[d]
        pairs = ps.N * ball / np.prod([2 * math.pi / m for m in ps.M])
        slots = pairs * direct_slots_per_pair(d)
        ach = slots / (stages["ds_kernel"]["avg_ms"] * 1e-3) / 1e12
        direct_roofline = {"kernel": "ds_kernel", "bound": "alu", "achieved": ach,
                           "peak": VALU_SLOT_PEAK_T, "unit": "T VALU slots/s",
                           "frac": ach / VALU_SLOT_PEAK_T, "pairs_per_launch": pairs,
                           "slots_per_pair": direct_slots_per_pair(d),
                           "pairs_per_s": pairs / (stages["ds_kernel"]["avg_ms"] * 1e-3)}

    # ---- CPU baseline: the oracle on a bounded sample -----------------------
    # The oracle's FGGC cost is mostly per cell and per grid point, and its
    # direct sum's per grid point, so the sample is all packets and a set of
    # grid points: the whole grid in 1D (each run repeated until about
    # cpu_target_s / 2 seconds have passed), a random sample of points in 2D and
    # 3D, timed and scaled by (grid points / sampled points).
    cpu = None
    accuracy = {}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        cores = oracle.num_threads()
        sd = st.describe()
        mpts = int(np.prod(ps.M))
        if d == 1:
            pts = None
            npts = mpts
        else:
            rng = np.random.default_rng(11)
            npts = min(mpts, args.cpu_points)
            pts = np.unique(rng.integers(0, mpts, npts))
            npts = len(pts)

        def run_f():
            return oracle.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:d], sd["dp"][:d],
                               sd["dq_off"], sd["dp_off"], pts=pts)

        def run_d():
            return oracle.direct_sum(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, ps.R, pts=pts)

        def timed(fn):
            n, t0 = 0, time.perf_counter()
            while True:
                out_ = fn()
                n += 1
                el = time.perf_counter() - t0
                if el >= args.cpu_target_s / 2 or n >= 50:
                    return out_, el / n, n

        log(f"cpu baseline: {ps.N} packets, {npts} of {mpts} grid points, {cores} threads")
        ref_f, t_of, n_f = timed(run_f)
        scale_pts = mpts / npts
        samp = "all packets, whole grid" if pts is None else \
            f"all packets, {npts} random grid points of {mpts}, time scaled by {scale_pts:.4g}"
        cpu = {"value": ps.N / (t_of * scale_pts), "unit": "packets/s", "cores": cores, "kind": "oracle",
               "sample": f"FP64 FGGC oracle (cells, then plain evaluation of eq. 2.24 with window "
                         f"8 sqrt(eps)): {samp}; mean of {n_f} runs",
               "seconds_per_run": t_of}
        # one thread, one run: what a single core of the box does
        prev = oracle.set_threads(1)
        t0 = time.perf_counter()
        run_f()
        cpu["single_thread"] = {"value": ps.N / ((time.perf_counter() - t0) * scale_pts), "unit": "packets/s",
                                "cores": 1, "sample": f"the same FGGC oracle sample, one run on one thread"}
        oracle.set_threads(prev)
        try:
            with open("/proc/cpuinfo") as f:
                cpu["host_cpu"] = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
        except OSError:
            cpu["host_cpu"] = None
        cpu["host_threads"] = os.cpu_count()
        ref_d = None
        if do_direct:
            ref_d, t_od, n_d = timed(run_d)
            cpu["direct_sum"] = {"value": ps.N / (t_od * scale_pts), "unit": "packets/s",
                                 "seconds_per_run": t_od,
                                 "sample": f"FP64 windowed direct-sum oracle: {samp}; mean of {n_d} runs"}
        # the GPU result of the timed workload against the oracle on the same points
        pick = (lambda u: u.reshape(-1)) if pts is None else (lambda u: u.reshape(-1)[pts])
        accuracy["fggc_fp32_vs_oracle_rel_l2"] = rel(pick(u_fggc).astype(np.complex128), ref_f)
        if ref_d is not None and u_direct is not None:
            accuracy["direct_fp32_vs_oracle_rel_l2"] = rel(pick(u_direct).astype(np.complex128), ref_d)
        accuracy["oracle_points"] = npts
        log("accuracy:", accuracy)
    if fvd is not None:
        accuracy["fggc_vs_direct_rel_l2"] = fvd

    serving = None
    if not args.no_serving:
        serving = serving_bench(ctx, F, W, torch, args.serving_pool, args.serving_requests, (0.5, 0.8),
                                args.serving_streams)

    value = ps.N / (fggc_ms * 1e-3)
    out = {
        "metric": "packets reconstructed/sec at rel-L2<=1e-6: FGGC vs direct sum; serving p50/p99",
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fggc_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W.CONFIG_NAMES[k]}", "strategy": sname,
                   "N": ps.N, "grid": list(ps.M), "eps": ps.eps, "p_slices": slices,
                   "Nq": [int(st.Nq[i]) for i in range(d)]},
        "direct_sum": None if direct_ms is None else {"value": ps.N / (direct_ms * 1e-3),
                                                      "ms_per_step": direct_ms,
                                                      "roofline": direct_roofline},
        "speedup_vs_direct": None if direct_ms is None else direct_ms / fggc_ms,
        "direct_sum_separable": sep,
        "accuracy": accuracy,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "stages_ms": {k2: v["avg_ms"] for k2, v in stages.items()},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
