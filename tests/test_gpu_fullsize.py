"""Full-size 2D and 3D workloads on the GPU (through the C ABI).

cfg2 (2D, N = 2^22, grid 1024^2): FGGC against the FP64 oracle's FGGC on
sampled grid points; FGGC against the direct sum on the whole grid (they
differ by the least-squares error of the strategy, ~1e-7 for Q4P2).
cfg3 (3D, N = 2^24, grid 256^3, 8.6e9 cells, so cell offsets pass 2^32):
FGGC (Q2P2, FP32) against the FP64 oracle's FGGC at heavy and random points
of the whole grid -- the oracle keeps only the cells within its evaluation
window of those points; the direct sum on the central 64^3 sub-box against
the oracle's direct sum; FGGC against that direct sum on the sub-box, at the
Q2P2 least-squares level.  Every comparison bounds rel-L2 and max-abs.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2504_21785_amd import fggc as F  # noqa: E402
from paper_2504_21785_amd import workloads as W  # noqa: E402
from parity import check  # noqa: E402


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = F.Context(0)
    yield c
    c.close()


def t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def heavy_points(ps, n_heavy, n_rand, seed, box_lo=None, box_n=None):
    """Grid points (flat) nearest the heaviest packets' centres plus random ones,
    chosen from the inputs alone; optionally restricted to a box."""
    rng = np.random.default_rng(seed)
    M = np.array(ps.M)
    order = np.argsort(-np.abs(ps.a))
    m = np.rint((ps.Q[:, order] + math.pi) / (2 * math.pi) * M[:, None]).astype(np.int64) % M[:, None]
    if box_lo is not None:
        lo, n = np.array(box_lo)[:, None], np.array(box_n)[:, None]
        inside = np.all((m >= lo) & (m < lo + n), axis=0)
        m = m[:, inside]
    m = m[:, : 8 * n_heavy: 8]
    if box_lo is None:
        r = np.stack([rng.integers(0, Mk, n_rand) for Mk in M])
    else:
        r = np.stack([rng.integers(box_lo[k], box_lo[k] + box_n[k], n_rand) for k in range(len(M))])
    flat = np.ravel_multi_index(tuple(np.concatenate([m, r], axis=1)), tuple(M))
    return np.unique(flat)


@pytest.fixture(scope="module")
def cfg2():
    return W.config(2)


def test_cfg2_fggc_fp32_vs_oracle_sampled(ctx, orc, cfg2):
    ps = cfg2
    st = F.default_strategy(2, ps.eps, "Q4P2")
    log("cfg2 fggc", ps.N, ps.M, st.describe())
    u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, st, precision=F.FP32)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(-1).astype(np.complex128)
    pts = heavy_points(ps, 48, 16, 3)
    sd = st.describe()
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:2], sd["dp"][:2], sd["dq_off"],
                   sd["dp_off"], pts=pts)
    check(u[pts], ref, 1e-6, f"cfg2 fggc fp32 vs oracle ({len(pts)} points)")


def test_cfg2_fggc_vs_direct(ctx, cfg2):
    ps = cfg2
    Q, P, S, a = t(ps.Q), t(ps.P), t(ps.S), t(ps.a)
    st = F.default_strategy(2, ps.eps, "Q4P2")
    uf = ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32)
    ud = ctx.direct_sum(Q, P, S, a, ps.eps, ps.M, ps.R, precision=F.FP32)
    torch.cuda.synchronize()
    check(uf.cpu().numpy(), ud.cpu().numpy(), 2e-6, "cfg2 fggc vs direct (Q4P2 LS level)")


SUB_LO, SUB_N = (96, 96, 96), (64, 64, 64)


@pytest.fixture(scope="module")
def cfg3():
    return W.config(3)


def test_cfg3_fggc_fp32_vs_oracle_sampled(ctx, orc, cfg3):
    """The whole 256^3 grid, FP32 FGGC against the FP64 FGGC oracle at 48 points
    under the heaviest packets and 24 random points (anywhere in the grid, so
    every region of the cell array and of each contraction pass is sampled)."""
    ps = cfg3
    st = F.default_strategy(3, ps.eps, "Q2P2")
    log("cfg3 fggc", ps.N, ps.M, st.describe())
    u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, st, precision=F.FP32)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(-1)
    pts = heavy_points(ps, 48, 24, 7)
    # random points far from the heavy packets carry tiny values: the max-abs
    # bound is relative to the largest sampled value
    sd = st.describe()
    log("cfg3 oracle on", len(pts), "points")
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:3], sd["dp"][:3], sd["dq_off"],
                   sd["dp_off"], pts=pts)
    check(u[pts], ref, 1e-6, f"cfg3 fggc fp32 vs oracle ({len(pts)} points of the whole grid)")


def test_cfg3_direct_subbox_vs_oracle(ctx, orc, cfg3):
    ps = cfg3
    log("cfg3 direct sub-box", ps.N, ps.M)
    u = ctx.direct_sum_box(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, SUB_LO, SUB_N, ps.R,
                           precision=F.FP32)
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    pts = heavy_points(ps, 40, 24, 5, SUB_LO, SUB_N)
    ref = orc.direct_sum(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, ps.R, pts=pts)
    m = np.stack(np.unravel_index(pts, ps.M))
    got = u[m[0] - SUB_LO[0], m[1] - SUB_LO[1], m[2] - SUB_LO[2]]
    check(got, ref, 1e-6, f"cfg3 direct sub-box fp32 vs oracle ({len(pts)} points)")


def test_cfg3_fggc_vs_direct_subbox(ctx, cfg3):
    ps = cfg3
    Q, P, S, a = t(ps.Q), t(ps.P), t(ps.S), t(ps.a)
    st = F.default_strategy(3, ps.eps, "Q2P2")
    log("cfg3 fggc", st.describe())
    uf = ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32)
    torch.cuda.synchronize()
    sub = uf[SUB_LO[0]:SUB_LO[0] + SUB_N[0], SUB_LO[1]:SUB_LO[1] + SUB_N[1],
             SUB_LO[2]:SUB_LO[2] + SUB_N[2]].cpu().numpy()
    del uf
    ud = ctx.direct_sum_box(Q, P, S, a, ps.eps, ps.M, SUB_LO, SUB_N, ps.R, precision=F.FP32)
    torch.cuda.synchronize()
    # the Q2P2 least-squares error at C_q = 0.555, C_p = pi/8 is below ~1e-3 per
    # packet (the sup of E_LSA over the cell, 9.0e-4); it is not rounding, so it
    # must also be clearly above the FP32 level
    e, m = check(sub, ud.cpu().numpy(), 2e-3, "cfg3 fggc (Q2P2) vs direct on the sub-box", max_tol=5e-3)
    assert e > 1e-6
