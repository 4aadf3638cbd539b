"""Separable direct sum (box window, matrix cores) against the FP64 oracle.

fggc_direct_sum_separable evaluates eq. (2.10) with the window |y_k| <= R per
dimension.  The oracle's box-window sum is the reference; the bar is the FP32
path's rel-L2 <= 1e-6.  Cases cover ragged 32 x 32 tiles, grids smaller than
a tile plus its window (every candidate treated as visible), packets on the
periodic seam, a window wide enough that the corners of the box carry weight,
and the full 2D workload on sampled points.
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


def rel(u, ref):
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))


def random_set(seed, N, p_mean=0.5, p_std=0.3, edge=False):
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-math.pi, math.pi, (2, N))
    if edge:  # packets on the periodic seam, on both sides
        e = N // 8
        Q[:, :e] = -math.pi + rng.uniform(-1e-9, 1e-9, (2, e))
        Q[:, e: 2 * e] = math.pi - rng.uniform(0, 1e-3, (2, e))
    P = p_mean + p_std * rng.standard_normal((2, N))
    S = rng.uniform(0, 2 * math.pi, N)
    a = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) * 0.5
    return Q, P, S, a


def run_sep(ctx, Q, P, S, a, eps, M, R, scale=1.0):
    out = ctx.direct_sum_separable(t(Q), t(P), t(S), t(a), eps, M, R, scale=scale)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(-1).astype(np.complex128)


@pytest.mark.parametrize("M,N,eps,R", [
    ((128, 128), 4000, 1.0 / 256, None),   # whole tiles
    ((96, 80), 1500, 1.0 / 256, None),     # ragged tiles in both dimensions
    ((48, 40), 700, 1.0 / 64, None),       # grid narrower than tile + window
    ((256, 64), 3000, 1.0 / 1024, None),
    ((64, 64), 500, 1.0, 1.5),             # wide window: the box corners matter
])
def test_small_sets(ctx, orc, M, N, eps, R):
    R = 6 * math.sqrt(eps) if R is None else R
    Q, P, S, a = random_set(11 + N, N, edge=True)
    log("separable", M, N, eps, R)
    u = run_sep(ctx, Q, P, S, a, eps, M, R, scale=0.37)
    ref = orc.direct_sum(Q, P, S, a, eps, M, R, scale=0.37, window="box")
    check(u, ref, 1e-6, f"separable M={M} N={N} eps={eps}")
    if R > 1.0:
        # the ball of the same radius drops the corners: not what was computed
        ball = orc.direct_sum(Q, P, S, a, eps, M, R, scale=0.37)
        assert rel(u, ball) > 1e-3


def test_single_packet_on_grid_point(ctx):
    # a packet on a grid point with P = 0: |u| is the product of two 1D
    # Gaussians, symmetric about the point, with |u| = |a| there
    M = (128, 96)
    m = (40, 70)
    Q = np.array([[-math.pi + m[0] * 2 * math.pi / M[0]], [-math.pi + m[1] * 2 * math.pi / M[1]]])
    eps, R = 1.0 / 64, 0.75
    u = run_sep(ctx, Q, np.zeros((2, 1)), np.zeros(1), np.array([2.0 + 0j]), eps, M, R).reshape(M)
    assert abs(u[m] - 2.0) < 1e-6
    assert np.allclose(u[m[0] + 1: m[0] + 6, m[1]], u[m[0] - 1: m[0] - 6: -1, m[1]], rtol=1e-6, atol=0)
    assert np.allclose(u[m[0], m[1] + 1: m[1] + 6], u[m[0], m[1] - 1: m[1] - 6: -1], rtol=1e-6, atol=0)
    # separable: u(m0 + i, m1 + j) u(m0, m1) = u(m0 + i, m1) u(m0, m1 + j)
    assert abs(u[m[0] + 3, m[1] + 4] * u[m] - u[m[0] + 3, m[1]] * u[m[0], m[1] + 4]) < 1e-6


def test_empty_host_and_errors(ctx, orc):
    Q = np.zeros((2, 0)); P = np.zeros((2, 0)); S = np.zeros(0); a = np.zeros(0, complex)
    assert np.all(run_sep(ctx, Q, P, S, a, 1 / 64, (64, 64), 0.75) == 0)
    Q, P, S, a = random_set(5, 300)
    out = ctx.direct_sum_separable(Q, P, S, a, 1 / 64, (64, 32), 0.75)  # host buffers
    ref = orc.direct_sum(Q, P, S, a, 1 / 64, (64, 32), 0.75, window="box")
    check(out.reshape(-1), ref, 1e-6, "separable host buffers")
    with pytest.raises(F.FggcError) as ei:
        ctx.direct_sum_separable(Q, P, S, a, 1 / 64, (64, 32), 0.75, precision=F.FP64)
    assert ei.value.code == F.FGGC_EUNSUPPORTED
    with pytest.raises(F.FggcError) as ei:
        ctx.direct_sum_separable(Q[:1], P[:1], S, a, 1 / 64, (64,), 0.75)
    assert ei.value.code == F.FGGC_EUNSUPPORTED
    with pytest.raises(F.FggcError) as ei:
        ctx.direct_sum_separable(Q, P, S, a, 1 / 64, (64, 32), math.pi)
    assert ei.value.code == F.FGGC_EINVAL


def test_repeated_calls(ctx, orc):
    Q, P, S, a = random_set(9, 2000)
    ref = orc.direct_sum(Q, P, S, a, 1 / 256, (128, 96), 0.375, window="box")
    for _ in range(3):
        check(run_sep(ctx, Q, P, S, a, 1 / 256, (128, 96), 0.375), ref, 1e-6, "separable repeated call")


def test_cfg2_full_size_sampled(ctx, orc):
    ps = W.config(2)
    log("cfg2 separable", ps.N, ps.M)
    u = run_sep(ctx, ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, ps.R)
    rng = np.random.default_rng(3)
    pts = np.sort(rng.choice(int(np.prod(ps.M)), 192, replace=False))
    ref = orc.direct_sum(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, ps.R, pts=pts, window="box")
    check(u[pts], ref, 1e-6, "cfg2 separable sampled")
    # against the ball-window direct sum of the same radius: the corners add
    # terms below exp(-18) of the packet peaks
    ub = ctx.direct_sum(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, ps.R)
    torch.cuda.synchronize()
    check(u, ub.cpu().numpy(), 1e-6, "cfg2 separable vs ball window")
