#!/usr/bin/env python3
"""Packets reconstructed per second on one MI355X: FGGC against the direct sum.

    python bench.py [--steps K] [--warmup W] [--workload cfg3] [--no-cpu-baseline]

One step reconstructs one batch of packets, already resident in HBM, into the
wave function on the grid.  The headline workload is the 3D set (N = 2^24
packets, 256^3 grid): pass A times K FGGC reconstructions (fggc_reconstruct:
correction, scatter, FFT over q, band multiply, inverse FFT) and then the
direct sum (fggc_direct_sum) of the same packets on the whole grid, over
fewer steps in 3D (stated in the line), each pass bracketed by device
synchronisations.  `value` is FGGC packets per second, reported only when the
FGGC result agrees with the FP64 oracle on the sampled points within
rel-L2 <= 1e-6; otherwise it is null.  Pass B repeats FGGC with the library's
per-stage HIP events on (fggc_profile) to time the kernels for the roofline.
The CPU-baseline leg times the FP64 oracle on a bounded sample of the same
workload and checks the GPU results on that sample against it.  The 1D and 2D
workloads are timed too and reported under `other_workloads`.  Prints one
JSON line.
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
FP32_VEC_PEAK_T = 157.3  # FP32 vector TFLOP/s (256 CUs x 128 FMA lanes x 2 x 2.4 GHz)
# VALU issue slots: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one non-packed op per lane per cycle)
VALU_SLOT_PEAK_T = 256 * 64 * 2.4e9 / 1e12
ACCURACY_BOUND = 1e-6

WORKLOADS = {"cfg0": 0, "cfg1": 1, "cfg2": 2, "cfg3": 3}
WORKLOAD_DIM = {"cfg0": 1, "cfg1": 1, "cfg2": 2, "cfg3": 3}
ROOT = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(u, ref):
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))


def maxabs(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def committed_profile(name):
    """A committed counter summary (profiles/NAME.json), or None when missing or
    when the kernel sources have changed since it was taken."""
    from paper_2504_21785_amd import rocprof_summary as RS
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != RS.source_digest():
        return None
    return t


def measured_traffic(workload, stage):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) of a stage's
    kernels, from the committed counter run of this workload."""
    t = committed_profile(f"traffic_{workload}.json")
    if t is None:
        return None
    st = t.get("stages", {}).get(stage)
    if not st or "fetch_size_bytes" not in st or "write_size_bytes" not in st:
        return None
    return st["fetch_size_bytes"] + st["write_size_bytes"]


def direct_valu_slots(workload):
    """VALU lane issue slots per ds_kernel launch from committed SQ counters:
    every wave instruction holds its SIMD for 4 cycles, a quarter-rate
    transcendental for 16, and a SIMD cycle is 16 lane slots."""
    t = committed_profile(f"valu_{workload}.json")
    if t is None:
        return None
    k = t.get("kernels", {}).get("ds_kernel")
    if not k:
        return None
    valu, trans = k["SQ_INSTS_VALU"], k["SQ_INSTS_VALU_TRANS_F32"]
    return ((valu - trans) * 4 + trans * 16) * 16


def fused_valu_busy(workload, ms):
    """Share of the VALU issue slots the fused 3D kernel keeps busy, from the
    committed SQ counters of this workload (SQ_INSTS_VALU per dispatch, 4
    cycles of its SIMD per wave instruction, 64 lane slots per instruction)."""
    t = committed_profile(f"valu_{workload}.json")
    if t is None:
        return None
    k = t.get("kernels", {}).get("fggc_fused_kernel")
    if not k or "SQ_INSTS_VALU" not in k:
        return None
    slots = k["SQ_INSTS_VALU"] * 64
    return {"lane_slots_per_launch": slots, "achieved_T": slots / (ms * 1e-3) / 1e12,
            "peak_T": VALU_SLOT_PEAK_T, "frac": slots / (ms * 1e-3) / 1e12 / VALU_SLOT_PEAK_T,
            "source": f"profiles/valu_{workload}.json (SQ_INSTS_VALU per dispatch)"}


def sample_points(ps, n_heavy, n_rand, seed):
    """Grid points (flat) nearest the centres of the heaviest packets (every
    eighth of the heaviest, so that they spread) and random ones; chosen from
    the inputs alone."""
    rng = np.random.default_rng(seed)
    M = np.array(ps.M)
    order = np.argsort(-np.abs(ps.a))[: 8 * n_heavy: 8]
    m = np.rint((ps.Q[:, order] + math.pi) / (2 * math.pi) * M[:, None]).astype(np.int64) % M[:, None]
    r = np.stack([rng.integers(0, Mk, n_rand) for Mk in M])
    return np.unique(np.ravel_multi_index(tuple(np.concatenate([m, r], axis=1)), tuple(M)))


def stage_work(ps, st, sn, fused=False, cK=6.0):
    """Algorithmic work per step of each FGGC stage: (bound, amount, unit, peak,
    launches per step, kernel).  Bytes count what the stage must read and write
    once; multi-pass stages count each pass's own input and output."""
    d, N = ps.d, ps.N
    Nq = [int(st.Nq[k]) for k in range(d)]
    M = [int(m) for m in ps.M]
    sn = [int(v) for v in sn]
    es = 8
    cells = int(np.prod(sn)) * int(np.prod(Nq))
    mpts = int(np.prod(M))
    n1 = int(st.nq * st.np)
    n1b = 4 if n1 <= 4 else (8 if n1 <= 8 else 16)
    rec_b = 16 + d * n1b * es  # one 16-byte word of indices, then the coefficients
    ns = 1 if d == 1 else 2 ** d
    w = {
        # FP64: two complex n1 x n1 mat-vecs per dimension, rhs and shift, Kronecker weights
        "fggc_coef": ("alu", N * (d * (16 * n1 * n1 + 60 * n1) + 6 * n1 ** d) / 1e12, "TFLOP/s", FP64_PEAK_T, 1,
                      "fggc_coef_kernel"),
        # packets' Q and P in; keys, ranks and positions of every key slot
        "fggc_sort": ("hbm", N * (2 * d * 8 + 12 * ns) / 1e9, "GB/s", HBM_PEAK_GBS, None, "sort kernels"),
        "fggc_ifft": ("hbm", 2 * mpts * es / 1e9, "GB/s", HBM_PEAK_GBS, None, "fft_axis_kernel"),
    }
    if d == 1:
        # records in, the slices' q-spectra written once
        w["fggc_accum"] = ("hbm", (N * rec_b + cells * es) / 1e9, "GB/s", HBM_PEAK_GBS, 2,
                           "fggc_agg1_kernel + fggc_stencil_fft1_kernel")
        w["fggc_band_mac"] = ("hbm", (cells + mpts) * es / 1e9, "GB/s", HBM_PEAK_GBS, 1, "band_mac1_kernel")
    else:
        # records in, the dense cell array written once
        w["fggc_accum"] = ("hbm", (N * rec_b + cells * es) / 1e9, "GB/s", HBM_PEAK_GBS, 1,
                           "fggc_accum_wave_kernel")

        def pass_bytes(k):
            # the separable pass over dimension k reads its input once and
            # writes its (smaller) output once
            O, A, B = int(np.prod(sn[:k])), int(np.prod(Nq[:k])), int(np.prod(M[k + 1:]))
            return (O * sn[k] * A * Nq[k] * B + O * A * M[k] * B) * es

        if fused:
            # the accumulation fused with the pass over the last dimension.
            # It reads one record per packet and writes the pass's output once
            # (a few GB: far from the HBM roof), so it is priced by its FP32
            # arithmetic: the Kronecker contributions (one complex multiply and
            # add, 8 flops, per packet and (q, p) basis triple), the q2-DFT of
            # every line of every slice (5 N log2 N flops) and the fold of each
            # slice's band into the grid frequencies (a real weight times a
            # complex value added, 4 flops, per line, slice and band frequency)
            kl = d - 1
            O, A = int(np.prod(sn[:kl])), int(np.prod(Nq[:kl]))
            lines = int(np.prod(sn)) * A
            band = math.floor(2 * cK / math.sqrt(ps.eps)) + 1
            flops = (N * n1 ** d * 8 + lines * 5 * Nq[kl] * math.log2(Nq[kl]) + lines * band * 4)
            w["fggc_fused"] = ("alu", flops / 1e12, "TFLOP/s", FP32_VEC_PEAK_T, 1, "fggc_fused_kernel")
            w["fggc_fused_bytes"] = (N * rec_b + O * A * M[kl] * es) / 1e9
            w["fggc_contract"] = ("hbm", sum(pass_bytes(k) for k in range(d - 2, -1, -1)) / 1e9, "GB/s",
                                  HBM_PEAK_GBS, d - 1, "fft_contract_kernel")
        else:
            w["fggc_contract"] = ("hbm", sum(pass_bytes(k) for k in range(d - 1, -1, -1)) / 1e9, "GB/s",
                                  HBM_PEAK_GBS, d, "fft_contract_kernel")
    method_bytes = N * ((2 * d + 1) * 8 + 16) + 2 * cells * es + 3 * mpts * es
    if fused:
        # no cell array: packets in, the records written and read once, the
        # first pass's output written and read once, spectrum and u
        O, A = int(np.prod(sn[:d - 1])), int(np.prod(Nq[:d - 1]))
        method_bytes = N * ((2 * d + 1) * 8 + 16) + 2 * N * rec_b + 2 * O * A * M[d - 1] * es + 3 * mpts * es
    return w, method_bytes


def time_steps(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def measure(ctx, F, W, torch, name, steps, warmup, direct_steps, strategy=None):
    """Timed FGGC and direct-sum steps of one workload (device-resident inputs)."""
    k = WORKLOADS[name]
    ps = W.config(k)
    d = ps.d
    sname = strategy or ("Q2P2" if d == 3 else "Q4P2")
    st = F.default_strategy(d, ps.eps, sname)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    Q, P, S, a = t(ps.Q), t(ps.P), t(ps.S), t(ps.a)
    u_f = torch.empty(ps.M, dtype=torch.complex64, device=dev)
    u_d = torch.empty(ps.M, dtype=torch.complex64, device=dev)

    def step_fggc():
        ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32, out=u_f)

    def step_direct():
        ctx.direct_sum(Q, P, S, a, ps.eps, ps.M, ps.R, precision=F.FP32, out=u_d)

    log(f"workload {name}: d={d} N={ps.N} M={ps.M} eps={ps.eps} strategy={sname}")
    for i in range(warmup):
        step_fggc()
        torch.cuda.synchronize()
        log(f"{name}: FGGC warmup step {i + 1} of {warmup} done")
    step_direct()
    torch.cuda.synchronize()
    log(f"{name}: direct warmup step done")
    fggc_ms = time_steps(step_fggc, steps, torch)
    log(f"{name}: FGGC {fggc_ms:.4f} ms/step over {steps} steps")
    direct_ms = time_steps(step_direct, direct_steps, torch)
    log(f"{name}: direct {direct_ms:.4f} ms/step over {direct_steps} steps")
    return {"ps": ps, "st": st, "sname": sname, "dev": (Q, P, S, a), "u_f": u_f, "u_d": u_d,
            "fggc_ms": fggc_ms, "direct_ms": direct_ms, "step_fggc": step_fggc, "step_direct": step_direct}


def profile_stages(ctx, torch, step, steps, names):
    ctx.profile(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    out = {}
    for sn in names:
        ms, cnt = ctx.stage_time(sn)
        if cnt:
            out[sn] = {"ms_per_step": ms / steps, "scopes": cnt}
    ctx.profile(False)
    return out


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
    ap.add_argument("--workload", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--direct-steps-3d", type=int, default=3,
                    help="timed direct-sum steps for 3D workloads (about 2 s each on the whole grid)")
    ap.add_argument("--strategy", default=None, help="Q2P2, Q4P2, Q2P4 or Q4P4 (default Q4P2; Q2P2 in 3D)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream measurement")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads")
    ap.add_argument("--cpu-points", type=int, default=4096,
                    help="random grid points sampled by the oracle in 2D")
    ap.add_argument("--cpu-points-3d", type=int, default=32,
                    help="grid points sampled by the oracle in 3D (3/4 under the heaviest packets)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run a plain elementwise copy (read and write this many MiB) before timing, "
                         "to scale HBM counters read under a profiler")
    ap.add_argument("--serving-pool", type=int, default=48)
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-streams", type=int, default=4)
    ap.add_argument("--cpu-target-s", type=float, default=12.0,
                    help="approximate CPU seconds for the oracle sample in 1D")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_21785_amd import fggc as F
    from paper_2504_21785_amd import workloads as W

    ctx = F.Context(0)
    dev = torch.device("cuda:0")
    k = WORKLOADS[args.workload]
    d = WORKLOAD_DIM[args.workload]
    direct_steps = args.direct_steps_3d if d == 3 else args.steps
    R = measure(ctx, F, W, torch, args.workload, args.steps, args.warmup, direct_steps, args.strategy)
    ps, st, sname = R["ps"], R["st"], R["sname"]
    Q, P, S, a = R["dev"]
    fggc_ms, direct_ms = R["fggc_ms"], R["direct_ms"]

    if args.calib_copy_mb > 0:
        cx = torch.ones(args.calib_copy_mb << 18, dtype=torch.float32, device=dev)
        cy = torch.empty_like(cx)
        for _ in range(3):
            torch.mul(cx, 2.0, out=cy)
        torch.cuda.synchronize()
        del cx, cy

    # the separable (box-window, matrix-core) direct sum: 2D only
    sep = None
    if d == 2:
        u_s = torch.empty(ps.M, dtype=torch.complex64, device=dev)

        def step_sep():
            ctx.direct_sum_separable(Q, P, S, a, ps.eps, ps.M, ps.R, out=u_s)

        step_sep()
        sep_ms = time_steps(step_sep, args.steps, torch)
        prof = profile_stages(ctx, torch, step_sep, args.steps, ["ds_kernel"])
        kms = prof["ds_kernel"]["ms_per_step"]
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
    fstages = profile_stages(ctx, torch, R["step_fggc"], args.steps,
                             ["prepass", "fggc_sort", "fggc_coef", "fggc_accum", "fggc_fft_q",
                              "fggc_band_mac", "fggc_fused", "fggc_contract", "fggc_ifft"])
    dstages = profile_stages(ctx, torch, R["step_direct"], direct_steps,
                             ["prepass", "ds_prep", "ds_sort", "ds_kernel", "ds_reduce"])
    log("stages:", json.dumps(fstages), json.dumps(dstages))

    u_fggc = R["u_f"].cpu().numpy()
    u_direct = R["u_d"].cpu().numpy()
    fvd = rel(u_fggc.astype(np.complex128), u_direct.astype(np.complex128))
    log(f"FGGC vs direct rel-L2 {fvd:.3e}")
    if sep is not None:
        u_sep = u_s.cpu().numpy().astype(np.complex128)
        sep["rel_l2_vs_direct"] = rel(u_sep, u_direct.astype(np.complex128))
        sep["fggc_rel_l2_vs_it"] = rel(u_fggc.astype(np.complex128), u_sep)
        sep["speedup_fggc_vs_it"] = sep["ms_per_step"] / fggc_ms

    # ---- roofline of the dominant FGGC stage ---------------------------------
    lo, n = ctx.cell_box(Q, P, S, a, st)
    slices = int(np.prod(n))
    work, method_bytes = stage_work(ps, st, n, fused="fggc_fused" in fstages)
    cand = {s2: v for s2, v in fstages.items() if s2 in work and isinstance(work[s2], tuple) and work[s2][4]}
    dom = max(cand, key=lambda s2: cand[s2]["ms_per_step"])
    bound, amount, unit, peak, launches, kname = work[dom]
    dom_ms = fstages[dom]["ms_per_step"]
    achieved = amount / (dom_ms * 1e-3)
    tr = measured_traffic(args.workload, dom)
    roofline = {"kernel": kname, "stage": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": tr,
                "algorithmic_per_launch": amount / launches, "avg_launch_ms": dom_ms / launches,
                "launches_per_step": launches,
                "note": "amount per launch = the stage's algorithmic work per step / its launches per step"}
    if dom == "fggc_fused":
        fb = work["fggc_fused_bytes"]
        roofline["algorithmic_flops_per_launch"] = amount * 1e12
        roofline["note"] += ("; FP32 flops: Kronecker contributions 8 per packet and basis triple, 5 N log2 N per "
                             "q2-line DFT, 4 per (line, slice, band frequency) of the fold")
        roofline["hbm"] = {"algorithmic_bytes_per_launch": fb * 1e9, "achieved_GBs": fb / (dom_ms * 1e-3),
                           "frac": fb / (dom_ms * 1e-3) / HBM_PEAK_GBS,
                           "bytes": "one record per packet read, the pass output written once"}
        sq = fused_valu_busy(args.workload, dom_ms)
        if sq is not None:
            roofline["valu_busy"] = sq
    end_to_end = {"algorithmic_bytes": method_bytes,
                  "achieved_GBs": method_bytes / 1e9 / (fggc_ms * 1e-3),
                  "frac": method_bytes / 1e9 / (fggc_ms * 1e-3) / HBM_PEAK_GBS,
                  "note": ("packets in, the records written and read once, the first separable pass's output "
                           "written and read once (no cell array: the accumulation is fused with that pass), grid "
                           "spectrum written and read, u written; over the whole FGGC step")
                  if "fggc_fused" in fstages else
                  ("packets in, the dense cell array written and read once, grid spectrum written and "
                   "read, u written; over the whole FGGC step")}
    stage_rates = {}
    for s2, v in fstages.items():
        if s2 in work and isinstance(work[s2], tuple):
            b2, amt, u2, pk2, _, kn2 = work[s2]
            ach2 = amt / (v["ms_per_step"] * 1e-3)
            stage_rates[s2] = {"ms_per_step": v["ms_per_step"], "achieved": ach2, "unit": u2, "frac": ach2 / pk2}
    direct_roofline = None
    if "ds_kernel" in dstages:
        ball = {1: 2 * ps.R, 2: math.pi * ps.R ** 2, 3: 4.0 / 3.0 * math.pi * ps.R ** 3}[d]
        pairs = ps.N * ball / np.prod([2 * math.pi / m for m in ps.M])
        kms = dstages["ds_kernel"]["ms_per_step"]
        slots = direct_valu_slots(args.workload)
        direct_roofline = {"kernel": "ds_kernel", "bound": "alu", "peak": VALU_SLOT_PEAK_T,
                           "unit": "T VALU lane-slots/s", "pairs_per_launch": pairs, "avg_launch_ms": kms,
                           "pairs_per_s": pairs / (kms * 1e-3)}
        if slots is not None:
            ach = slots / (kms * 1e-3) / 1e12
            direct_roofline.update({"achieved": ach, "frac": ach / VALU_SLOT_PEAK_T,
                                    "slots_per_pair": slots / pairs,
                                    "slots_source": f"profiles/valu_{args.workload}.json (SQ_INSTS_VALU, "
                                                    "SQ_INSTS_VALU_TRANS_F32 per dispatch)"})
        else:
            direct_roofline.update({"achieved": None, "frac": None,
                                    "slots_source": "no committed SQ counters for the current sources"})

    # ---- the other workloads (before the CPU baseline, whose host threads
    # would otherwise share the host with their launches) ----------------------
    others = {}
    if not args.no_others:
        for name in ("cfg1", "cfg2", "cfg3"):
            if name == args.workload:
                continue
            dd = WORKLOAD_DIM[name]
            Ro = measure(ctx, F, W, torch, name, args.steps, args.warmup,
                         args.direct_steps_3d if dd == 3 else args.steps)
            uf, ud = Ro["u_f"].cpu().numpy().astype(np.complex128), Ro["u_d"].cpu().numpy().astype(np.complex128)
            others[name] = {"workload": f"{name}: {W.CONFIG_NAMES[WORKLOADS[name]]}", "strategy": Ro["sname"],
                            "fggc_packets_per_s": Ro["ps"].N / (Ro["fggc_ms"] * 1e-3),
                            "fggc_ms_per_step": Ro["fggc_ms"],
                            "direct_packets_per_s": Ro["ps"].N / (Ro["direct_ms"] * 1e-3),
                            "direct_ms_per_step": Ro["direct_ms"],
                            "speedup_vs_direct": Ro["direct_ms"] / Ro["fggc_ms"],
                            "fggc_vs_direct_rel_l2": rel(uf, ud), "fggc_vs_direct_max_abs": maxabs(uf, ud)}
            del Ro, uf, ud
            torch.cuda.empty_cache()

    # ---- CPU baseline: the oracle on a bounded sample -----------------------
    cpu = None
    accuracy = {"fggc_vs_direct_rel_l2": fvd,
                "fggc_vs_direct_max_abs": maxabs(u_fggc.astype(np.complex128), u_direct.astype(np.complex128))}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        cores = oracle.num_threads()
        sd = st.describe()
        mpts = int(np.prod(ps.M))
        if d == 1:
            pts = None
            npts = mpts
            how = "all packets, whole grid"
        elif d == 2:
            rng = np.random.default_rng(11)
            pts = np.unique(rng.integers(0, mpts, min(mpts, args.cpu_points)))
            npts = len(pts)
            how = f"all packets, {npts} random grid points of {mpts}"
        else:
            nh = (3 * args.cpu_points_3d) // 4
            pts = sample_points(ps, nh, args.cpu_points_3d - nh, 11)
            npts = len(pts)
            how = (f"all packets, {npts} grid points of {mpts} ({nh} under the heaviest packets, the rest "
                   f"random); the oracle keeps only the cells within its window of those points")

        def run_f(p=pts):
            return oracle.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:d], sd["dp"][:d],
                               sd["dq_off"], sd["dp_off"], pts=p)

        def run_d(p=pts):
            return oracle.direct_sum(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, ps.R, pts=p)

        def timed(fn, target):
            n_, t0 = 0, time.perf_counter()
            while True:
                out_ = fn()
                n_ += 1
                el = time.perf_counter() - t0
                if el >= target or n_ >= 50:
                    return out_, el / n_, n_

        log(f"cpu baseline: {ps.N} packets, {npts} of {mpts} grid points, {cores} threads")
        tgt = args.cpu_target_s / 2 if d == 1 else 0.0  # one run in 2D and 3D
        ref_f, t_of, n_f = timed(run_f, tgt)
        scale_pts = mpts / npts
        cpu = {"value": ps.N / (t_of * scale_pts), "unit": "packets/s", "cores": cores, "kind": "oracle",
               "sample": f"FP64 FGGC oracle (cells, then plain evaluation of eq. 2.24 with window "
                         f"8 sqrt(eps)): {how}; time scaled by grid points / sampled points "
                         f"({scale_pts:.4g}); mean of {n_f} runs",
               "seconds_per_run": t_of}
        # one thread: what a single core of the box does (on a smaller sample in 2D/3D)
        prev = oracle.set_threads(1)
        sub = None if pts is None else pts[:: max(1, len(pts) // (4 if d == 3 else 256))]
        t0 = time.perf_counter()
        run_f(sub)
        t1 = time.perf_counter() - t0
        nsub = mpts if sub is None else len(sub)
        cpu["single_thread"] = {"value": ps.N / (t1 * mpts / nsub), "unit": "packets/s", "cores": 1,
                                "sample": f"the same FGGC oracle on {nsub} of the sampled points, one run "
                                          f"on one thread"}
        oracle.set_threads(prev)
        try:
            with open("/proc/cpuinfo") as f:
                cpu["host_cpu"] = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
        except OSError:
            cpu["host_cpu"] = None
        cpu["host_threads"] = os.cpu_count()
        ref_d, t_od, n_d = timed(run_d, tgt)
        cpu["direct_sum"] = {"value": ps.N / (t_od * scale_pts), "unit": "packets/s", "seconds_per_run": t_od,
                             "sample": f"FP64 windowed direct-sum oracle: {how}; mean of {n_d} runs"}
        pick = (lambda u: u.reshape(-1)) if pts is None else (lambda u: u.reshape(-1)[pts])
        gf, gd = pick(u_fggc).astype(np.complex128), pick(u_direct).astype(np.complex128)
        accuracy.update({"fggc_fp32_vs_oracle_rel_l2": rel(gf, ref_f), "fggc_fp32_vs_oracle_max_abs": maxabs(gf, ref_f),
                         "direct_fp32_vs_oracle_rel_l2": rel(gd, ref_d),
                         "direct_fp32_vs_oracle_max_abs": maxabs(gd, ref_d),
                         "oracle_points": npts, "max_abs_is": "max|u - ref| / max|ref| over the points"})
        log("accuracy:", accuracy)

    serving = None
    if not args.no_serving:
        serving = serving_bench(ctx, F, W, torch, args.serving_pool, args.serving_requests, (0.5, 0.8),
                                args.serving_streams)

    acc = accuracy.get("fggc_fp32_vs_oracle_rel_l2")
    ok = acc is not None and acc <= ACCURACY_BOUND
    value = ps.N / (fggc_ms * 1e-3) if ok else None
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
        "value_note": None if ok else ("no oracle check of the FGGC result (--no-cpu-baseline)" if acc is None
                                       else f"FGGC rel-L2 against the oracle {acc:.3e} above {ACCURACY_BOUND}"),
        "direct_sum": {"value": ps.N / (direct_ms * 1e-3), "ms_per_step": direct_ms, "steps": direct_steps,
                       "roofline": direct_roofline},
        "speedup_vs_direct": direct_ms / fggc_ms,
        "direct_sum_separable": sep,
        "accuracy": accuracy,
        "roofline": roofline,
        "end_to_end": end_to_end,
        "stage_rates": stage_rates,
        "cpu_baseline": cpu,
        "other_workloads": others,
        "serving": serving,
        "stages_ms": {k2: v["ms_per_step"] for k2, v in {**fstages, **dstages}.items()},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
