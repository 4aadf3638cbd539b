"""Multi-step FGGC (Alg. 3) on the GPU, through libfggc.

T_final = T_multi * T_evo.  Each run
- decomposes the current u on a fixed (q, p) mesh (fggc_decompose, or
  fggc_decompose_mesh for a product mesh on grid points, eq. 2.7),
- evolves over T_evo only the mesh points that no earlier run has seen
  (fggc_propagate, eq. 2.3-2.6) and keeps what the flow maps them to,
- and reconstructs u by FGGC (fggc_reconstruct).

The flow is linear in A, so what a mesh point "learns" is its final
(Q, P, S) and the ratio A(T_evo) / A(0), obtained by evolving A(0) = 1; a
later run reuses it with its own A(0).  Mesh points whose |A(0)| is below
`prune` times the largest are skipped in that run.

This module only sequences library calls: the prune mask, the index
compaction, the gathers and the product A(0) * ratio run in the library
(fggc_learn_select, fggc_learn_start, fggc_learn_store, fggc_learn_packets);
torch only allocates the device buffers.
"""
import math

from paper_2504_21785_amd import fggc as F


class MultiStep:
    def __init__(self, ctx, eps: float, M, qm, pm, V, dt: float, steps: int, strategy,
                 R_dec: float = None, prune: float = 1e-12, precision: int = F.FP64, mesh=None):
        """mesh: None, or (Nq, q_lo, q_n, dp, p_lo, p_n) when (qm, pm) is that product
        mesh listed q-major with q on grid points; the decomposition then runs as
        batched GEMMs (fggc_decompose_mesh, box window)."""
        import torch
        self.torch = torch
        self.ctx, self.eps, self.M = ctx, float(eps), tuple(int(m) for m in M)
        self.d = len(self.M)
        self.qm, self.pm = qm.contiguous(), pm.contiguous()  # [d][Nm] float64 on the GPU
        self.V, self.dt, self.steps, self.st = V, float(dt), int(steps), strategy
        self.R_dec = 8 * math.sqrt(eps) if R_dec is None else float(R_dec)
        self.prune, self.precision, self.mesh = float(prune), precision, mesh
        Nm = self.qm.shape[1]
        dev = self.qm.device
        self.learned = torch.zeros(Nm, dtype=torch.uint8, device=dev)
        self.Qf = torch.zeros_like(self.qm)
        self.Pf = torch.zeros_like(self.pm)
        self.Sf = torch.zeros(Nm, dtype=torch.float64, device=dev)
        self.ratio = torch.zeros(Nm, dtype=torch.complex128, device=dev)
        self.keep_idx = torch.empty(Nm, dtype=torch.int64, device=dev)
        self.new_idx = torch.empty(Nm, dtype=torch.int64, device=dev)
        dq = [2 * math.pi / strategy.Nq[k] for k in range(self.d)]
        self.scale = math.prod(dq[k] * strategy.dp[k] for k in range(self.d)) / (2 * math.pi * eps) ** (1.5 * self.d)
        self.evolved = []

    def run(self, u, runs: int):
        """Carry u ([prod M] or grid-shaped complex tensor) over `runs` runs of T_evo."""
        torch = self.torch
        for _ in range(int(runs)):
            u64 = u.reshape(-1).to(torch.complex128).contiguous()
            if self.mesh is not None:
                A0 = self.ctx.decompose_mesh(u64, self.eps, self.M, self.R_dec, *self.mesh)
            else:
                A0 = self.ctx.decompose(u64, self.eps, self.M, self.R_dec, self.qm, self.pm)
            ctx = self.ctx
            nk, nn = ctx.learn_select(A0, self.prune, self.learned, self.keep_idx, self.new_idx)
            if nn:
                dev = A0.device
                Q = torch.empty((self.d, nn), dtype=torch.float64, device=dev)
                P = torch.empty_like(Q)
                S = torch.empty(nn, dtype=torch.float64, device=dev)
                A = torch.empty(nn, dtype=torch.complex128, device=dev)
                ctx.learn_start(self.new_idx, nn, self.qm, self.pm, Q, P, S, A)
                ctx.propagate(Q, P, S, A, self.V, self.dt, self.steps)
                ctx.learn_store(self.new_idx, nn, Q, P, S, A, self.Qf, self.Pf, self.Sf, self.ratio)
            self.evolved.append(int(nn))
            dev = A0.device
            Qk = torch.empty((self.d, nk), dtype=torch.float64, device=dev)
            Pk = torch.empty_like(Qk)
            Sk = torch.empty(nk, dtype=torch.float64, device=dev)
            ak = torch.empty(nk, dtype=torch.complex128, device=dev)
            ctx.learn_packets(self.keep_idx, nk, self.Qf, self.Pf, self.Sf, self.ratio, A0, Qk, Pk, Sk, ak)
            u = ctx.reconstruct(Qk, Pk, Sk, ak, self.eps, self.M, self.st, scale=self.scale,
                                precision=self.precision)
        return u
