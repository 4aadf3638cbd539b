"""The paper's Examples 1 and 2 (Sec. 4) end to end on the GPU.

u0 -> initial decomposition (2.7) on the (q, p) mesh dq = sqrt(eps)/2,
dp = pi sqrt(eps)/8 -> RK4 flow (2.3)-(2.6) to T = 0.8 with dt = 1e-4 ->
reconstruction by FGGC (Q4P2) and by the direct sum (the FGA).  Printed per
eps: packets kept, the time of each stage, and the FGGC-vs-FGA rel-L2 (the
paper's "LSA error").

- Example 1: u0 = (64/pi)^{1/4} exp(-32 x^2 + i x / eps), V = 1 - cos(pi x).
- Example 2: u0 = (64/pi)^{1/2} exp(-32 |x|^2 + i (x + y) / eps) with
  V2 = |x|^2 / 2, or V1 read as 1 - exp(-|x|^2).
The domain is the library's periodic [-pi, pi)^d (the paper's [-2, 2]^d holds
the same solution: the wave stays far from the boundary up to T = 0.8), on a
power-of-two grid with dx <= eps.  Packets whose |A(0)| is below 1e-12 of
the largest are dropped before the flow.

Usage: python -m paper_2504_21785_amd.examples --example 1 --eps 64,256,1024
Everything runs through libfggc; torch only holds device memory.
"""
import argparse
import json
import math
import sys
import time


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run(example: int, inv_eps: int, potential: str, T: float, dt: float, precision: str):
    import torch
    from paper_2504_21785_amd import fggc as F

    eps = 1.0 / inv_eps
    d = 1 if example == 1 else 2
    n = 1 << int(math.ceil(math.log2(2 * math.pi / eps)))  # dx <= eps
    n = min(n, 4096 if d == 2 else (8192 if precision == "fp64" else 16384))
    if 1.5 / eps >= n / 2:
        raise ValueError(f"eps = 1/{inv_eps}: momenta up to 1.5 need a grid above {n} points per axis")
    M = (n,) * d
    dev = torch.device("cuda:0")
    axes = [torch.arange(n, dtype=torch.float64, device=dev) * (2 * math.pi / n) - math.pi for _ in range(d)]
    X = torch.meshgrid(*axes, indexing="ij")
    r2 = sum(x * x for x in X)
    u0 = (64 / math.pi) ** (d / 4) * torch.exp(-32 * r2 + 1j * sum(X) / eps)
    if example == 1:
        V = F.potential(c0=1.0, c1=-1.0, kappa=math.pi)
    elif potential == "V1":
        V = F.potential(c0=1.0, c2=-1.0, c3=-1.0)
    else:
        V = F.potential(w=(1.0, 1.0))
    # (q, p) mesh over the support of u0 (|x| < 0.8) and of its transform in p:
    # per dimension |u0^| ~ exp(-(p - 1)^2 / (2 eps + 128 eps^2)), below 1e-12
    # of its peak outside |p - 1| = sqrt(27.7 (2 eps + 128 eps^2))
    dq, dp = math.sqrt(eps) / 2, math.pi * math.sqrt(eps) / 8
    ph = math.sqrt(27.7 * (2 * eps + 128 * eps * eps)) + 2 * dp
    q1 = torch.arange(-0.8, 0.8 + 1e-12, dq, dtype=torch.float64, device=dev)
    p1 = 1.0 + torch.arange(-ph, ph + 1e-12, dp, dtype=torch.float64, device=dev)
    ctx = F.Context(0)
    st = F.default_strategy(d, eps, "Q4P2")
    scale = (dq * dp) ** d / (2 * math.pi * eps) ** (1.5 * d)
    prec = F.FP64 if precision == "fp64" else F.FP32
    times = {}

    def tick(name, t0):
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t0

    # decomposition in chunks of q-rows (the full mesh of a small eps in 2D is large)
    t0 = time.perf_counter()
    keepQ, keepP, keepA = [], [], []
    amax = 0.0
    qs = torch.meshgrid(*([q1] * d), indexing="ij")
    qs = torch.stack([g.reshape(-1) for g in qs])
    ps = torch.meshgrid(*([p1] * d), indexing="ij")
    ps = torch.stack([g.reshape(-1) for g in ps])
    chunk = max(1, (1 << 24) // ps.shape[1])
    parts = []
    for i in range(0, qs.shape[1], chunk):
        qq = qs[:, i:i + chunk].repeat_interleave(ps.shape[1], dim=1).contiguous()
        pp = ps.repeat(1, min(chunk, qs.shape[1] - i)).contiguous()
        A = ctx.decompose(u0.reshape(-1).contiguous(), eps, M, 8 * math.sqrt(eps), qq, pp)
        amax = max(amax, float(A.abs().max()))
        parts.append((qq, pp, A))
    for qq, pp, A in parts:
        k = A.abs() > 1e-12 * amax
        keepQ.append(qq[:, k])
        keepP.append(pp[:, k])
        keepA.append(A[k])
    Q = torch.cat(keepQ, dim=1).contiguous()
    P = torch.cat(keepP, dim=1).contiguous()
    A = torch.cat(keepA).contiguous()
    del parts
    tick("decompose_s", t0)
    N = A.shape[0]
    S = torch.zeros(N, dtype=torch.float64, device=dev)
    nsteps = int(round(T / dt))
    t0 = time.perf_counter()
    ctx.propagate(Q, P, S, A, V, dt, nsteps)
    tick("propagate_s", t0)
    ctx.reconstruct(Q, P, S, A, eps, M, st, scale=scale, precision=prec)  # plan and graph warm-up
    t0 = time.perf_counter()
    uf = ctx.reconstruct(Q, P, S, A, eps, M, st, scale=scale, precision=prec)
    tick("fggc_s", t0)
    t0 = time.perf_counter()
    ud = ctx.direct_sum(Q, P, S, A, eps, M, 6 * math.sqrt(eps), scale=scale, precision=prec)
    tick("direct_s", t0)
    lsa = float(torch.linalg.vector_norm(uf.to(torch.complex128) - ud.to(torch.complex128))
                / torch.linalg.vector_norm(ud.to(torch.complex128)))
    ctx.close()
    return {"example": example, "potential": "1-cos(pi x)" if example == 1 else potential,
            "eps": f"1/{inv_eps}", "grid": list(M), "packets": N, "steps": nsteps, "precision": precision,
            **{k: round(v, 6) for k, v in times.items()}, "fggc_vs_fga_rel_l2": lsa}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--example", type=int, default=1, choices=[1, 2])
    ap.add_argument("--eps", default=None, help="values of 1/eps (default 64,256,1024 in 1D; 64,256 in 2D)")
    ap.add_argument("--potential", default="V2", choices=["V1", "V2"], help="Example 2's potential")
    ap.add_argument("--T", type=float, default=0.8)
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp64"])
    args = ap.parse_args()
    eps_list = args.eps or ("64,256,1024" if args.example == 1 else "64,256")
    for ie in (int(v) for v in eps_list.split(",")):
        log(f"example {args.example}, eps = 1/{ie}")
        print(json.dumps(run(args.example, ie, args.potential, args.T, args.dt, args.precision)), flush=True)


if __name__ == "__main__":
    main()
