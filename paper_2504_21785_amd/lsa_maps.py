"""Coefficient and error maps of the least-squares approximation (Sec. 2.2).

    python -m paper_2504_21785_amd.lsa_maps [--strategy Q2P2] [--n 21] [--out maps.json]

The paper's illustration approximates an off-grid packet G(x; Q, P), with
(Q, P) in the first cell [0, dq) x [0, dp), by its on-grid neighbours and
shows the coefficients and the relative L2 error as functions of (Q, P)
(d = 1, Q2P2, eps = 1/64, dq = 1/16, dp = pi/32, i.e. Cq = dq / sqrt(eps) = 1/2
and Cp = dp / sqrt(eps) = pi/4).  By Theorem 3 both depend on (Q, P) only
through s = Q/dq, t = P/dp and on the mesh only through (Cq, Cp), so the maps
are computed here at those Cq, Cp on the library's periodic mesh: Nq = 128
q-points (dq = 2 pi / 128) and eps = (dq / Cq)^2, so that dq / sqrt(eps) = Cq.

Everything is computed by the library on the GPU:
- the coefficients by the reconstruction's own coefficient kernel
  (fggc_coefficients, FP64), for an n x n sweep of the cell in one call;
- the error E_LSA = ||G - sum_k c_k G_k|| / ||G|| of each sweep point from the
  direct sum (fggc_direct_sum, FP64) of the packet with amplitude 1 and its
  neighbours with amplitudes -c_k on a fine grid (the window 6 sqrt(eps)
  leaves terms below exp(-18)); the norms are the grid sums.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from paper_2504_21785_amd import fggc as F

STRATEGIES = {"Q2P2": ([0, 1], [0, 1]), "Q4P2": ([-1, 0, 1, 2], [0, 1]),
              "Q2P4": ([0, 1], [-1, 0, 1, 2]), "Q4P4": ([-1, 0, 1, 2], [-1, 0, 1, 2])}


def maps(ctx, name: str = "Q2P2", Cq: float = 0.5, Cp: float = math.pi / 4, n: int = 21, Nq: int = 128,
         M: int = 8192, cutoff: float = 0.0):
    import torch
    dq_off, dp_off = STRATEGIES[name]
    dqm = 2 * math.pi / Nq
    se = dqm / Cq
    eps = se * se
    dpm = Cp * se
    st = F.make_strategy(1, [Nq], [dpm], dq_off, dp_off, cutoff=cutoff)
    s1 = np.arange(n) / n  # the half-open cell [0, 1)
    ss, tt = [g.ravel() for g in np.meshgrid(s1, s1, indexing="ij")]
    npt = ss.size
    dev = torch.device("cuda:0")
    Q = torch.from_numpy((ss * dqm)[None, :].copy()).to(dev)
    P = torch.from_numpy((tt * dpm)[None, :].copy()).to(dev)
    S = torch.zeros(npt, dtype=torch.float64, device=dev)
    a = torch.ones(npt, dtype=torch.complex128, device=dev)
    c, _ = ctx.coefficients(Q, P, S, a, eps, st)
    c = c.cpu().numpy()
    qk = np.array([u for u in dq_off for v in dp_off], dtype=np.float64) * dqm
    pk = np.array([v for u in dq_off for v in dp_off], dtype=np.float64) * dpm
    nb = qk.size
    R = 6.0 * se
    E = np.zeros(npt)
    for j in range(npt):
        Qj = np.concatenate([[ss[j] * dqm], qk])[None, :]
        Pj = np.concatenate([[tt[j] * dpm], pk])[None, :]
        aj = np.concatenate([[1.0 + 0.0j], -c[j]])
        zs = np.zeros(nb + 1)
        r = ctx.direct_sum(Qj, Pj, zs, aj, eps, (M,), R, precision=F.FP64)
        g = ctx.direct_sum(Qj[:, :1].copy(), Pj[:, :1].copy(), zs[:1].copy(), aj[:1].copy(), eps, (M,), R,
                           precision=F.FP64)
        r, g = np.asarray(r).reshape(-1), np.asarray(g).reshape(-1)
        E[j] = math.sqrt(float(np.sum(np.abs(r) ** 2)) / float(np.sum(np.abs(g) ** 2)))
    shape = (n, n)
    return {"strategy": name, "Cq": Cq, "Cp": Cp, "eps": eps, "Nq": Nq, "dq": dqm, "dp": dpm,
            "s": s1.tolist(), "t": s1.tolist(),
            "basis": [[int(u), int(v)] for u in dq_off for v in dp_off],
            "E_LSA": E.reshape(shape).tolist(),
            "coef_abs": [np.abs(c[:, k]).reshape(shape).tolist() for k in range(nb)],
            "coef_arg": [np.angle(c[:, k]).reshape(shape).tolist() for k in range(nb)],
            "summary": {"max_E": float(E.max()), "E_at_cell_centre": float(E.reshape(shape)[n // 2, n // 2]),
                        "max_abs_coef": float(np.abs(c).max())}}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--strategy", default="Q2P2", choices=sorted(STRATEGIES))
    ap.add_argument("--n", type=int, default=21, help="sweep points per axis of the cell")
    ap.add_argument("--Cq", type=float, default=0.5)
    ap.add_argument("--Cp", type=float, default=math.pi / 4)
    ap.add_argument("--out", default=None, help="write the maps as JSON here (default: summary only)")
    args = ap.parse_args(argv)
    ctx = F.Context(0)
    try:
        m = maps(ctx, args.strategy, args.Cq, args.Cp, args.n)
    finally:
        ctx.close()
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(m, fh)
    print(json.dumps({k: m[k] for k in ("strategy", "Cq", "Cp", "eps", "Nq", "basis", "summary")}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
