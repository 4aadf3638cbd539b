"""FGGC stages on the GPU (through the C ABI) against the FP64 CPU oracle.

- the batched FFT against numpy's FFT (FP64 1e-13, FP32 1e-6 relative);
- the cell array of eq. (2.25) against the oracle's cells (Q2P2, FP64:
  well conditioned, so the coefficients themselves are comparable);
- the whole reconstruction against the oracle's plain evaluation of (2.24):
  FP64 with Q2P2 at 1e-12; FP64 with Q4P2 at the conditioning floor of the
  least-squares solve; FP32 at 1e-6;
- every neighbour strategy of the M_LSA tables (Q2P2, Q4P2, Q2P4, Q4P4) on
  three meshes in 1D, and the four-shift p-sets in 2D, FP64 at a tolerance
  derived from the conditioning of the solve and FP32 at 1e-6.
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

Q2 = [0, 1]
Q4 = [-1, 0, 1, 2]


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


@pytest.mark.parametrize("prec,tol", [(F.FP64, 1e-13), (F.FP32, 1e-6)])
@pytest.mark.parametrize("dims,batch", [((2,), 3), ((8,), 5), ((64,), 7), ((512,), 33),
                                        ((2048,), 2), ((8192,), 1), ((8192,), 3), ((16, 32), 3),
                                        ((256, 256), 2), ((8, 16, 4), 3), ((32, 32, 32), 2)])
def test_fft_against_numpy(ctx, prec, tol, dims, batch):
    rng = np.random.default_rng(len(dims) * 100 + dims[0])
    x = rng.standard_normal((batch, *dims)) + 1j * rng.standard_normal((batch, *dims))
    axes = tuple(range(1, len(dims) + 1))
    dt = torch.complex128 if prec == F.FP64 else torch.complex64
    for direction in (-1, 1):
        xd = torch.from_numpy(x).to(dt).cuda().contiguous()
        ctx.fft(xd, dims, batch, direction, prec)
        torch.cuda.synchronize()
        got = xd.cpu().numpy().astype(np.complex128)
        ref = np.fft.fftn(x, axes=axes) if direction < 0 else np.fft.ifftn(x, axes=axes) * np.prod(dims)
        check(got, ref, tol, f"fft {dims} x{batch} dir {direction} prec {prec}")


def test_fft_16384_fp32(ctx):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(16384) + 1j * rng.standard_normal(16384)
    xd = torch.from_numpy(x).to(torch.complex64).cuda()
    ctx.fft(xd, (16384,), 1, 1, F.FP32)
    torch.cuda.synchronize()
    check(xd.cpu().numpy(), np.fft.ifft(x) * 16384, 1e-6, "fft 16384 fp32")


@pytest.mark.parametrize("prec,tol", [(F.FP64, 1e-13), (F.FP32, 1e-6)])
@pytest.mark.parametrize("dims,batch", [((3,), 4), ((5,), 3), ((6,), 5), ((96,), 7), ((1000,), 3),
                                        ((1536,), 2), ((3375,), 1), ((6000,), 2), ((64, 96), 2),
                                        ((96, 40), 3), ((1000, 6), 1), ((12, 20, 30), 2), ((48, 32, 45), 1)])
def test_fft_mixed_radix_against_numpy(ctx, prec, tol, dims, batch):
    # lengths 2^a 3^b 5^c: the mixed-radix passes (radix 4, 2, 3, 5), strides
    # that are not powers of two, and the four-step form above 4096 points
    rng = np.random.default_rng(7 + sum(dims))
    x = rng.standard_normal((batch, *dims)) + 1j * rng.standard_normal((batch, *dims))
    axes = tuple(range(1, len(dims) + 1))
    dt = torch.complex128 if prec == F.FP64 else torch.complex64
    for direction in (-1, 1):
        log(f"fft mixed {dims} x{batch} dir {direction} prec {prec}")
        xd = torch.from_numpy(x).to(dt).cuda().contiguous()
        ctx.fft(xd, dims, batch, direction, prec)
        torch.cuda.synchronize()
        got = xd.cpu().numpy().astype(np.complex128)
        ref = np.fft.fftn(x, axes=axes) if direction < 0 else np.fft.ifftn(x, axes=axes) * np.prod(dims)
        check(got, ref, tol, f"fft {dims} x{batch} dir {direction} prec {prec}")


def test_fft_sizes_refused(ctx):
    for dims in ((7,), (14,), (1,)):
        x = torch.zeros(int(np.prod(dims)), dtype=torch.complex64, device="cuda")
        with pytest.raises(RuntimeError, match="FFT sizes"):
            ctx.fft(x, dims, 1, -1, F.FP32)
    y = torch.zeros(2 * 4500, dtype=torch.complex64, device="cuda")
    with pytest.raises(RuntimeError, match="FFT sizes"):  # above 4096 in 2D: powers of two only
        ctx.fft(y, (2, 4500), 1, -1, F.FP32)


def small_1d(seed, N=2000, eps=1.0 / 64, M=1024):
    ps = W.gen_1d(max(1, N // 50), 50, eps, M, seed)
    return ps


@pytest.mark.parametrize("layout", [(Q2, Q2), (Q4, Q2)])
def test_cells_match_oracle_fp64(ctx, orc, layout):
    ps = small_1d(11)
    eps = ps.eps
    st = F.default_strategy(1, eps, "Q2P2")
    st = F.make_strategy(1, [st.Nq[0]], [st.dp[0]], layout[0], layout[1])
    cells, lo, n = ctx.cells(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), eps, st, scale=0.5, precision=F.FP64)
    ref, slo, sn = orc.fggc_cells(ps.Q, ps.P, ps.S, ps.a, eps, [st.Nq[0]], [st.dp[0]], layout[0],
                                  layout[1], scale=0.5)
    assert list(lo) == list(slo) and list(n) == list(sn)
    # coefficients carry the conditioning of the Gram matrix: u * cond ~ 2e-11
    # for Q2P2 (cond ~1e5); Q4P2 (cond ~1e11) agrees only in the function the
    # cells represent (checked by the reconstruction tests), so loosely here
    tol = 1e-10 if layout == (Q2, Q2) else 1e-4
    check(cells, ref, tol, f"cells {layout}")


def fggc_case(ctx, orc, ps, name, prec, layout=None, pts=None, scale=1.0):
    d = ps.d
    st = F.default_strategy(d, ps.eps, name)
    if layout is not None:
        st = F.make_strategy(d, list(st.Nq)[:d], list(st.dp)[:d], layout[0], layout[1])
    u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, st, scale=scale, precision=prec)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(-1).astype(np.complex128)
    sd = st.describe()
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:d], sd["dp"][:d], sd["dq_off"],
                   sd["dp_off"], scale=scale, pts=pts)
    return (u if pts is None else u[pts]), ref


@pytest.mark.parametrize("prec,name,tol", [(F.FP64, "Q2P2", 1e-12), (F.FP64, "Q4P2", 1e-10),
                                           (F.FP32, "Q4P2", 1e-6), (F.FP32, "Q2P2", 1e-6)])
def test_reconstruct_1d_small(ctx, orc, prec, name, tol):
    ps = small_1d(12, N=3000)
    u, ref = fggc_case(ctx, orc, ps, name, prec, scale=0.8)
    check(u, ref, tol, f"fggc 1d {name} prec {prec}")


def test_reconstruct_cfg0_fp64(ctx, orc):
    ps = W.config(0)
    u, ref = fggc_case(ctx, orc, ps, "Q2P2", F.FP64)
    check(u, ref, 1e-12, "fggc cfg0 fp64 Q2P2")


def heavy_points(ps, n_heavy, n_rand, seed):
    """Grid points nearest the centres of the heaviest packets, plus random ones
    (chosen from the inputs alone, so that sampled values are not all tails)."""
    rng = np.random.default_rng(seed)
    M = np.array(ps.M)
    idx = np.argsort(-np.abs(ps.a))[: 4 * n_heavy: 4]
    m = np.rint((ps.Q[:, idx] + math.pi) / (2 * math.pi) * M[:, None]).astype(np.int64) % M[:, None]
    flat = np.ravel_multi_index(tuple(m), tuple(M))
    pts = np.concatenate([flat, rng.choice(int(np.prod(M)), n_rand, replace=False)])
    return np.unique(pts)


def test_reconstruct_1d_wide_shifts(ctx, orc):
    # a coarse strategy with Cq Cp > 1 (Nq = 32 and dp = 2 sqrt(eps) at
    # eps = 1/64): the right-hand side's phases take the general path of the
    # coefficient kernel instead of the small-angle series
    ps = small_1d(13, N=3000)
    eps = ps.eps
    cq = 2 * math.pi / 32 / math.sqrt(eps)
    cp = 2.0
    assert cq * cp > 1.0
    st = F.make_strategy(1, [32], [cp * math.sqrt(eps)], [0, 1], [0, 1])
    u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), eps, ps.M, st, precision=F.FP64)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(-1)
    sd = st.describe()
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, eps, ps.M, sd["Nq"][:1], sd["dp"][:1], sd["dq_off"],
                   sd["dp_off"])
    check(u, ref, 1e-12, "fggc 1d wide shifts (Cq Cp = %.2f)" % (cq * cp))


@pytest.mark.parametrize("prec,tol", [(F.FP32, 1e-6), (F.FP64, 1e-10)])
def test_reconstruct_1d_crowded_bins(ctx, orc, prec, tol):
    # a coarse mesh (eps = 1/64: 128 q-cells, 4 q-tiles) with 655360 packets
    # puts several thousand records in each bin, so that the one-dimensional
    # aggregate splits bins over several workgroups and copies of A
    ps = W.gen_1d(1024, 640, 1.0 / 64, 1024, seed=21)
    pts = heavy_points(ps, 48, 16, 2)
    u, ref = fggc_case(ctx, orc, ps, "Q4P2", prec, pts=pts)
    check(u, ref, tol, f"fggc 1d crowded bins prec {prec}")


STRATEGIES = {"Q2P2": (Q2, Q2), "Q4P2": (Q4, Q2), "Q2P4": (Q2, Q4), "Q4P4": (Q4, Q4)}


def strategy_cutoff_and_tol(name, Cq, Cp):
    """Eigenvalue cutoff and FP64 tolerance for a neighbour strategy (Sec. 3.1).

    Exact least squares where the Gram matrix (3.22) has kappa < 1e12; above
    that the paper's reading of a truncated pseudo-inverse (eigenvalues below
    1e-10 of the largest dropped), on both sides.  Two rounding terms, with
    kappa the ratio of the largest to the smallest kept eigenvalue and
    |c|_1 = O(1):
    - the library's FP64 solve moves c by ~kappa u along the eigenvectors of
      the smallest kept eigenvalue, which changes u by at most
      sqrt(lambda_min) kappa u |c| = sqrt(lambda_max kappa) u (u = 1.1e-16,
      a factor 2 of margin);
    - the oracle's truncated solve forms the pseudo-inverse explicitly in long
      double: its entries, of size 1/lambda_min, carry a rounding error of
      ~u_ld kappa relative that spreads over every direction (u_ld = 5.4e-20).
    """
    ev, _ = F.plan_gram(*STRATEGIES[name], Cq, Cp)
    lmax = float(ev.max())
    kappa = lmax / ev.min() if ev.min() > 0 else math.inf
    cutoff = 0.0 if kappa < 1e12 else 1e-10
    kept = ev[ev > cutoff * lmax] if cutoff > 0 else ev
    kappa_eff = lmax / float(kept.min())
    oracle_term = 5.4e-20 * kappa_eff if cutoff > 0 else 0.0
    return cutoff, max(1e-12, 2.2e-16 * math.sqrt(lmax * kappa_eff), oracle_term)


@pytest.mark.parametrize("C", [math.pi / 4, math.pi / 8, math.pi / 16], ids=["pi/4", "pi/8", "pi/16"])
@pytest.mark.parametrize("name", ["Q2P2", "Q4P2", "Q2P4", "Q4P4"])
def test_reconstruct_1d_strategies(ctx, orc, name, C):
    # every neighbour strategy of the M_LSA tables at Cq = Cp = C (eps = 1/64:
    # Nq = 64, 128, 256), FP64 against the oracle with the same cutoff, and
    # FP32 at the FP32 bound
    ps = small_1d(14, N=3000)
    eps = ps.eps
    Nq = int(round(2 * math.pi / (C * math.sqrt(eps))))
    dq_off, dp_off = STRATEGIES[name]
    cutoff, tol = strategy_cutoff_and_tol(name, C, C)
    st = F.make_strategy(1, [Nq], [C * math.sqrt(eps)], dq_off, dp_off, cutoff=cutoff)
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, eps, ps.M, [Nq], [C * math.sqrt(eps)], dq_off, dp_off,
                   rcond=cutoff)
    for prec, bound in ((F.FP64, tol), (F.FP32, 1e-6)):
        u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), eps, ps.M, st, precision=prec)
        torch.cuda.synchronize()
        check(u.cpu().numpy(), ref, bound, f"fggc 1d {name} C = {C:.4f} cutoff {cutoff} prec {prec}")


@pytest.mark.parametrize("name", ["Q2P4", "Q4P4"])
def test_reconstruct_2d_strategies(ctx, orc, name):
    # the p-shift sets of four (n1 = 8 and 16, n1^2 = 64 and 256 coefficients
    # per packet) in 2D at the default mesh (C = pi/8)
    ps = W.gen_mesh(2, 16, 6, 0.5, (0.5, 0.3), 1.0 / 256, 128, seed=6)
    pts = heavy_points(ps, 150, 50, 3)
    st0 = F.default_strategy(2, ps.eps, name)
    Cq = 2 * math.pi / st0.Nq[0] / math.sqrt(ps.eps)
    Cp = st0.dp[0] / math.sqrt(ps.eps)
    cutoff, tol = strategy_cutoff_and_tol(name, Cq, Cp)
    sd = st0.describe()
    st = F.make_strategy(2, sd["Nq"][:2], sd["dp"][:2], sd["dq_off"], sd["dp_off"], cutoff=cutoff)
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:2], sd["dp"][:2], sd["dq_off"],
                   sd["dp_off"], rcond=cutoff, pts=pts)
    for prec, bound in ((F.FP64, 2 * tol), (F.FP32, 1e-6)):
        u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, st, precision=prec)
        torch.cuda.synchronize()
        check(u.cpu().numpy().reshape(-1)[pts], ref, bound, f"fggc 2d {name} cutoff {cutoff} prec {prec}")


@pytest.mark.parametrize("prec,name,tol", [(F.FP64, "Q2P2", 1e-12), (F.FP32, "Q4P2", 1e-6)])
def test_reconstruct_2d_small(ctx, orc, prec, name, tol):
    ps = W.gen_mesh(2, 16, 6, 0.5, (0.5, 0.3), 1.0 / 256, 128, seed=5)
    pts = heavy_points(ps, 150, 50, 1)
    u, ref = fggc_case(ctx, orc, ps, name, prec, pts=pts)
    check(u, ref, tol, f"fggc 2d {name} prec {prec}")


@pytest.mark.parametrize("prec,tol", [(F.FP32, 1e-6), (F.FP64, 1e-10)])
def test_reconstruct_2d_crowded_bins(ctx, orc, prec, tol):
    # 147456 packets in 3 x 3 p-cells (a p-range of 0.06 per dimension):
    # about 250 records per bin, so that a workgroup of the two-dimensional
    # accumulation (one slice, one q-tile: 2 x 2 bins) takes some sixteen
    # chunks of 64 records with a ragged last one -- the FP32 records are
    # loaded a chunk ahead, the FP64 ones are not
    ps = W.gen_mesh(2, 48, 8, 0.06, (0.5, 0.3), 1.0 / 256, 128, seed=23)
    pts = heavy_points(ps, 60, 20, 3)
    u, ref = fggc_case(ctx, orc, ps, "Q4P2", prec, pts=pts)
    check(u, ref, tol, f"fggc 2d crowded bins prec {prec}")


def test_reconstruct_3d_small(ctx, orc):
    ps = W.gen_mesh(3, 8, 3, 0.5, (0.5, 0.3, 0.3), 1.0 / 64, 64, seed=9)
    pts = heavy_points(ps, 80, 20, 2)
    u, ref = fggc_case(ctx, orc, ps, "Q2P2", F.FP64, pts=pts)
    check(u, ref, 1e-12, "fggc 3d fp64")


def test_cells_3d_match_oracle_and_sub_box(ctx, orc):
    """3D Q2P2 cells (the atomic scatter) against the oracle's cells of eq. (2.25);
    a caller-chosen box that cuts the packets' p-cells is refused."""
    # eps = 1/16: 64^3 q-cells per slice and ~5 slices per axis (~0.5 GB of FP64 cells)
    ps = W.gen_mesh(3, 8, 3, 0.3, (0.5, 0.3, 0.3), 1.0 / 16, 64, seed=12)
    st = F.default_strategy(3, ps.eps, "Q2P2")
    lo0, n0 = ctx.cell_box(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), st)
    assert np.prod(np.asarray(n0) + 2) * np.prod(list(st.Nq)[:3]) * 16 < 2e9
    sd = st.describe()
    args = (t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, st)
    cells, lo, n = ctx.cells(*args, scale=0.5, precision=F.FP64)
    ref, slo, sn = orc.fggc_cells(ps.Q, ps.P, ps.S, ps.a, ps.eps, sd["Nq"][:3], sd["dp"][:3], sd["dq_off"],
                                  sd["dp_off"], scale=0.5)
    assert list(lo) == list(slo) and list(n) == list(sn)
    check(cells, ref, 1e-10, "cells 3d")
    assert min(n) >= 3
    with pytest.raises(F.FggcError) as ei:
        ctx.cells(*args, scale=0.5, precision=F.FP64, box=(np.asarray(lo) + 1, np.asarray(n) - 2))
    assert ei.value.code == F.FGGC_EINVAL
    # a larger box holds the same cells, surrounded by zeros
    big, _, _ = ctx.cells(*args, scale=0.5, precision=F.FP64, box=(np.asarray(lo) - 1, np.asarray(n) + 2))
    inner = big.reshape(*[int(v) + 2 for v in n], -1)[1:-1, 1:-1, 1:-1].reshape(cells.shape)
    assert np.max(np.abs(inner - cells)) <= 1e-13 * np.max(np.abs(cells))
    assert np.count_nonzero(big) == np.count_nonzero(cells)


def test_fggc_vs_direct_cfg1(ctx):
    """FGGC and the direct sum agree at the LSA level (Q4P2 ~ 3e-7 at C = pi/8)."""
    ps = W.config(1)
    Q, P, S, a = t(ps.Q), t(ps.P), t(ps.S), t(ps.a)
    st = F.default_strategy(1, ps.eps, "Q4P2")
    uf = ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32)
    ud = ctx.direct_sum(Q, P, S, a, ps.eps, ps.M, ps.R, precision=F.FP32)
    torch.cuda.synchronize()
    check(uf.cpu().numpy(), ud.cpu().numpy(), 2e-6, "cfg1 fggc vs direct (Q4P2 LS level)")


def test_repeated_calls_replay_graph_with_live_data(ctx, orc):
    # Device-resident calls with the same buffers run eagerly, are captured,
    # then replayed from a cached graph: every run must read the buffers as
    # they are at that call (a replay after an in-place update sees the update).
    ps = small_1d(21, N=3000, eps=1.0 / 256, M=2048)
    st = F.default_strategy(1, ps.eps, "Q4P2")
    Q, P, S, a = t(ps.Q), t(ps.P), t(ps.S), t(ps.a)
    u = torch.empty(ps.M, dtype=torch.complex64, device="cuda")
    sd = st.describe()
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:1], sd["dp"][:1], sd["dq_off"],
                   sd["dp_off"])
    outs = []
    for i in range(4):
        ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32, out=u)
        torch.cuda.synchronize()
        outs.append(u.cpu().numpy().copy())
        check(outs[-1], ref, 1e-6, f"call {i} vs oracle")
    a.mul_(2.0)  # the same buffers, new values
    torch.cuda.synchronize()
    ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32, out=u)
    torch.cuda.synchronize()
    check(u.cpu().numpy(), 2 * ref, 1e-6, "replay after in-place update")


def test_calls_on_two_streams_are_ordered(ctx, orc):
    # one context, two streams: the second call's stream waits for the first
    # call's use of the shared workspace
    ps1 = small_1d(31, N=2500, eps=1.0 / 256, M=2048)
    ps2 = small_1d(32, N=4000, eps=1.0 / 64, M=1024)
    st1 = F.default_strategy(1, ps1.eps, "Q4P2")
    st2 = F.default_strategy(1, ps2.eps, "Q2P2")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    d1 = [t(x) for x in (ps1.Q, ps1.P, ps1.S, ps1.a)]
    d2 = [t(x) for x in (ps2.Q, ps2.P, ps2.S, ps2.a)]
    torch.cuda.synchronize()
    u1 = torch.empty(ps1.M, dtype=torch.complex64, device="cuda")
    u2 = torch.empty(ps2.M, dtype=torch.complex64, device="cuda")
    for _ in range(3):
        with torch.cuda.stream(s1):
            ctx.reconstruct(*d1, ps1.eps, ps1.M, st1, precision=F.FP32, out=u1, stream=s1)
        with torch.cuda.stream(s2):
            ctx.direct_sum(*d2, ps2.eps, ps2.M, ps2.R, precision=F.FP32, out=u2, stream=s2)
    torch.cuda.synchronize()
    sd = st1.describe()
    r1 = orc.fggc(ps1.Q, ps1.P, ps1.S, ps1.a, ps1.eps, ps1.M, sd["Nq"][:1], sd["dp"][:1], sd["dq_off"],
                  sd["dp_off"])
    r2 = orc.direct_sum(ps2.Q, ps2.P, ps2.S, ps2.a, ps2.eps, ps2.M, ps2.R)
    check(u1.cpu().numpy(), r1, 1e-6, "two streams: fggc")
    check(u2.cpu().numpy(), r2, 1e-6, "two streams: direct")


def test_repeated_3d_calls_on_two_level_sort_path(ctx, orc):
    # A 3D layout with more than 2^15 bins sorts in two counting levels.  With
    # the same buffers, the first call runs eagerly, the second is captured in
    # a graph and the later ones replay it: every call must match the oracle.
    ps = W.gen_mesh(3, 8, 3, 0.5, (0.5, 0.3, 0.3), 1.0 / 64, 64, seed=9)
    st = F.default_strategy(3, ps.eps, "Q2P2")
    Q, P, S, a = t(ps.Q), t(ps.P), t(ps.S), t(ps.a)
    u = torch.empty(ps.M, dtype=torch.complex64, device="cuda")
    pts = heavy_points(ps, 40, 10, 4)
    sd = st.describe()
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:3], sd["dp"][:3], sd["dq_off"],
                   sd["dp_off"], pts=pts)
    for i in range(4):
        log(f"3d two-level-sort call {i}")
        ctx.reconstruct(Q, P, S, a, ps.eps, ps.M, st, precision=F.FP32, out=u)
        torch.cuda.synchronize()
        check(u.cpu().numpy().reshape(-1)[pts], ref, 1e-6, f"3d call {i} vs oracle")


def edge_packets(d, eps, st, seed):
    """Packets on the q- and p-mesh points of strategy `st` (s = t = 0 up to the
    rounding of Q / dq), at -pi and just below pi (the periodic seam), at
    negative momenta, and one at a random point."""
    rng = np.random.default_rng(seed)
    sd = st.describe()
    dq = [2 * math.pi / sd["Nq"][k] for k in range(d)]
    dp = [sd["dp"][k] for k in range(d)]
    Qs, Ps = [], []
    for i in (-(sd["Nq"][0] // 2), -3, 0, 5, sd["Nq"][0] // 2 - 1):
        for l in (-7, -1, 0, 2, 9):
            Qs.append([-math.pi + (i + sd["Nq"][0] // 2) * dq[k] for k in range(d)])
            Ps.append([l * dp[k] for k in range(d)])
    Qs.append([-math.pi] * d)
    Ps.append([-0.3] * d)
    Qs.append([math.pi - 1e-12] * d)
    Ps.append([0.45] * d)
    Qs.append(list(rng.uniform(-math.pi, math.pi, d)))
    Ps.append(list(rng.uniform(-0.5, 0.5, d)))
    Q = np.ascontiguousarray(np.array(Qs).T)
    P = np.ascontiguousarray(np.array(Ps).T)
    N = Q.shape[1]
    S = rng.uniform(0, 2 * math.pi, N)
    a = rng.normal(size=N) + 1j * rng.normal(size=N)
    return Q, P, S, a


@pytest.mark.parametrize("d,M", [(1, 512), (2, 64)])
@pytest.mark.parametrize("prec,tol", [(F.FP64, 1e-12), (F.FP32, 1e-6)])
def test_reconstruct_edge_cases(ctx, orc, d, M, prec, tol):
    eps = 1.0 / 64
    st = F.default_strategy(d, eps, "Q2P2")
    sd = st.describe()
    grid = (M,) * d
    # no packets: zeros
    e0 = np.zeros((d, 0))
    u = ctx.reconstruct(t(e0), t(e0), t(np.zeros(0)), t(np.zeros(0, complex)), eps, grid, st, precision=prec)
    torch.cuda.synchronize()
    assert u.shape[-1] == M and not torch.any(u != 0)
    Q, P, S, a = edge_packets(d, eps, st, seed=20 + d)
    for sel in (slice(0, 1), slice(-1, None), slice(None)):  # a single packet, another one, all
        q, p, s_, a_ = (np.ascontiguousarray(Q[:, sel]), np.ascontiguousarray(P[:, sel]),
                        np.ascontiguousarray(S[sel]), np.ascontiguousarray(a[sel]))
        u = ctx.reconstruct(t(q), t(p), t(s_), t(a_), eps, grid, st, precision=prec)
        torch.cuda.synchronize()
        u = u.cpu().numpy().reshape(-1).astype(np.complex128)
        ref = orc.fggc(q, p, s_, a_, eps, grid, sd["Nq"][:d], sd["dp"][:d], sd["dq_off"], sd["dp_off"])
        check(u, ref, tol, f"edge d={d} prec={prec} N={q.shape[1]}")


def mesh3(seed, M, Nq=None, dp=None, eps=1.0 / 64, nq=8, npd=3, width=0.5):
    """A 3D packet set on grid M (per dimension), with an optional strategy mesh."""
    ps = W.gen_mesh(3, nq, npd, width, (0.5, 0.3, 0.3), eps, M[0], seed=seed)
    ps.M = tuple(M)
    return ps


@pytest.mark.parametrize("name,prec,tol,M,Nq", [
    ("Q2P2", F.FP64, 1e-12, (64, 64, 64), None),
    ("Q2P2", F.FP32, 1e-6, (64, 64, 64), None),
    ("Q4P2", F.FP32, 1e-6, (64, 64, 64), None),
    ("Q2P4", F.FP32, 1e-6, (64, 64, 64), None),
    # unequal meshes and grids: 4 x 4 line tiles over 64 x 32 q-cells, a q2
    # line of 256, and a last-dimension grid (32) narrower than the band union
    ("Q2P2", F.FP64, 1e-12, (32, 64, 32), (64, 32, 256)),
    ("Q2P2", F.FP32, 1e-6, (128, 32, 64), (128, 64, 64)),
    ("Q4P2", F.FP64, 1e-9, (64, 32, 128), (64, 64, 128)),
])
def test_reconstruct_3d_fused(ctx, orc, name, prec, tol, M, Nq):
    # the three-dimensional finish (accumulation fused with the pass over the
    # last dimension) for every shift set it takes, both precisions, and
    # meshes and grids that differ per dimension
    ps = mesh3(31, M)
    st0 = F.default_strategy(3, ps.eps, name)
    sd0 = st0.describe()
    Nq = list(sd0["Nq"][:3]) if Nq is None else list(Nq)
    st = F.make_strategy(3, Nq, sd0["dp"][:3], sd0["dq_off"], sd0["dp_off"])
    sd = st.describe()
    pts = heavy_points(ps, 60, 40, 5)
    log(f"3d fused {name} prec {prec} M={M} Nq={Nq}")
    u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, st, scale=0.7, precision=prec)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(-1)[pts].astype(np.complex128)
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:3], sd["dp"][:3], sd["dq_off"],
                   sd["dp_off"], scale=0.7, pts=pts)
    check(u, ref, tol, f"fggc 3d {name} prec {prec} M={M} Nq={Nq}")


@pytest.mark.parametrize("d,name,prec,tol,M,Nq", [
    (1, "Q2P2", F.FP64, 1e-12, (1536,), (96,)),
    (1, "Q4P2", F.FP32, 1e-6, (1536,), (96,)),
    (1, "Q2P2", F.FP32, 1e-6, (1000,), (96,)),
    (1, "Q4P2", F.FP64, 1e-9, (1000,), (90,)),
    (2, "Q2P2", F.FP64, 1e-12, (240, 360), (96, 160)),
    (2, "Q4P2", F.FP32, 1e-6, (1000, 1536), (96, 192)),
    (2, "Q2P2", F.FP32, 1e-6, (1000, 1000), (96, 96)),
    (2, "Q4P2", F.FP64, 1e-9, (96, 1000), (192, 96)),
    (3, "Q2P2", F.FP64, 1e-12, (48, 40, 60), (48, 40, 30)),
    (3, "Q2P2", F.FP32, 1e-6, (60, 64, 48), (24, 64, 96)),
    (3, "Q2P2", F.FP32, 1e-6, (60, 40, 48), (32, 32, 64)),  # the fused finish on grids of 60, 40, 48
])
def test_reconstruct_mixed_radix_sizes(ctx, orc, d, name, prec, tol, M, Nq):
    # grids and q-meshes of the form 2^a 3^b 5^c (even q-meshes), per
    # dimension, against the oracle's evaluation of eq. (2.24)
    if d == 1:
        ps = small_1d(41, N=3000)
    elif d == 2:
        ps = W.gen_mesh(2, 16, 6, 0.5, (0.5, 0.3), 1.0 / 256, 128, seed=43)
    else:
        ps = W.gen_mesh(3, 8, 3, 0.5, (0.5, 0.3, 0.3), 1.0 / 64, 64, seed=47)
    ps.M = tuple(M)
    st0 = F.default_strategy(d, ps.eps, name)
    sd0 = st0.describe()
    st = F.make_strategy(d, list(Nq), sd0["dp"][:d], sd0["dq_off"], sd0["dp_off"])
    sd = st.describe()
    pts = None if d == 1 else heavy_points(ps, 120, 60, 9)
    log(f"mixed sizes d={d} {name} prec {prec} M={M} Nq={Nq}")
    u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, st, scale=0.9, precision=prec)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(-1).astype(np.complex128)
    if pts is not None:
        u = u[pts]
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:d], sd["dp"][:d], sd["dq_off"],
                   sd["dp_off"], scale=0.9, pts=pts)
    check(u, ref, tol, f"fggc mixed d={d} {name} prec {prec} M={M} Nq={Nq}")


def test_3d_box_wider_than_record_indices_refused(ctx):
    # three-dimensional records hold 16-bit p-cell indices: a box of more than
    # 65535 p-cells along a dimension is refused before any kernel runs
    eps = 1.0 / 64
    st = F.default_strategy(3, eps, "Q2P2")
    dp = st.describe()["dp"][0]
    Q = np.zeros((3, 2))
    P = np.zeros((3, 2))
    P[0, 1] = 70000 * dp
    S = np.zeros(2)
    a = np.ones(2, dtype=np.complex128)
    with pytest.raises(RuntimeError, match="65535"):
        ctx.reconstruct(t(Q), t(P), t(S), t(a), eps, (32, 32, 32), st, precision=F.FP32)


def test_mixed_radix_sizes_refused(ctx):
    ps = W.gen_mesh(2, 16, 6, 0.5, (0.5, 0.3), 1.0 / 256, 128, seed=43)
    st0 = F.default_strategy(2, ps.eps, "Q4P2")
    sd0 = st0.describe()
    args = (t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps)
    cases = [((128, 128), (75, 64), "Nq must be an even"),       # odd q-mesh
             ((128, 128), (14, 64), "Nq must be an even"),       # factor 7
             ((128, 126), (64, 64), "grid sizes"),               # grid with a factor 7
             ((128, 128), (90, 64), "power-of-two factor")]      # 90 = 2 x 45 < the Q4 span
    for M, Nq, msg in cases:
        st = F.make_strategy(2, list(Nq), sd0["dp"][:2], sd0["dq_off"], sd0["dp_off"])
        with pytest.raises(RuntimeError, match=msg):
            ctx.reconstruct(*args, M, st, precision=F.FP32)


@pytest.mark.parametrize("name,prec,tol,eps,M,Nq", [
    ("Q2P2", F.FP64, 1e-12, 1.0 / 256, (128, 128), None),
    ("Q4P2", F.FP32, 1e-6, 1.0 / 256, (256, 128), None),
    ("Q2P4", F.FP32, 1e-6, 1.0 / 256, (128, 256), None),
    ("Q4P2", F.FP64, 1e-9, 1.0 / 256, (128, 128), None),     # FP64 records of 272 bytes: read in two steps
    ("Q2P2", F.FP32, 1e-6, 1.0 / 256, (64, 96), (128, 64)),  # unequal meshes; a grid of 96 along the lines
    ("Q4P2", F.FP32, 1e-6, 1.0 / 1024, (256, 256), (256, 512)),  # 512-point lines
    ("Q2P2", F.FP32, 1e-6, 1.0 / 1024, (512, 512), (512, 512)),  # 512-point lines, wide band union
    ("Q2P2", F.FP32, 1e-6, 1.0 / 1024, (256, 1024), (256, 512)),  # two blocks of frequencies per thread
    ("Q4P2", F.FP32, 1e-6, 1.0 / 1024, (128, 1024), (256, 256)),
])
def test_reconstruct_2d_fused(ctx, orc, name, prec, tol, eps, M, Nq):
    # the two-dimensional fused finish (accumulation with the pass over the
    # last dimension) for each shift set it takes, both precisions, lines of
    # up to 512 points, meshes and grids that differ per dimension
    ps = W.gen_mesh(2, 16, 6, 0.5, (0.5, 0.3), eps, 128, seed=53)
    ps.M = tuple(M)
    st0 = F.default_strategy(2, ps.eps, name)
    sd0 = st0.describe()
    Nq = list(sd0["Nq"][:2]) if Nq is None else list(Nq)
    st = F.make_strategy(2, Nq, sd0["dp"][:2], sd0["dq_off"], sd0["dp_off"])
    sd = st.describe()
    pts = heavy_points(ps, 120, 60, 5)
    log(f"2d fused {name} prec {prec} eps {eps} M={M} Nq={Nq}")
    u = ctx.reconstruct(t(ps.Q), t(ps.P), t(ps.S), t(ps.a), ps.eps, ps.M, st, scale=0.7, precision=prec)
    torch.cuda.synchronize()
    u = u.cpu().numpy().reshape(-1)[pts].astype(np.complex128)
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:2], sd["dp"][:2], sd["dq_off"],
                   sd["dp_off"], scale=0.7, pts=pts)
    check(u, ref, tol, f"fggc 2d fused {name} prec {prec} eps {eps} M={M} Nq={Nq}")


@pytest.mark.parametrize("prec,tol", [(F.FP64, 1e-12), (F.FP32, 1e-6)])
def test_reconstruct_3d_edge_cases(ctx, orc, prec, tol):
    # no packets; single packets; packets on q- and p-mesh points, on the
    # periodic seam and at negative momenta (a compact p-range keeps the
    # oracle's cells few), compared around each packet's centre
    eps = 1.0 / 64
    M = (32, 32, 32)
    st = F.default_strategy(3, eps, "Q2P2")
    sd = st.describe()
    e0 = np.zeros((3, 0))
    u = ctx.reconstruct(t(e0), t(e0), t(np.zeros(0)), t(np.zeros(0, complex)), eps, M, st, precision=prec)
    torch.cuda.synchronize()
    assert tuple(u.shape) == M and not torch.any(u != 0)
    Nq, dp = sd["Nq"][:3], sd["dp"][:3]
    dq = [2 * math.pi / n for n in Nq]
    Qs, Ps = [], []
    for i in (-(Nq[0] // 2), -3, 0, Nq[0] // 2 - 1):
        for l in (-1, 0, 2):
            Qs.append([-math.pi + (i + Nq[0] // 2) * dq[k] for k in range(3)])
            Ps.append([l * dp[k] for k in range(3)])
    Qs.append([-math.pi] * 3)
    Ps.append([-0.5 * dp[0]] * 3)
    Qs.append([math.pi - 1e-12, -math.pi, 0.3])
    Ps.append([1.5 * dp[0], -0.9 * dp[1], 0.0])
    Q = np.ascontiguousarray(np.array(Qs).T)
    P = np.ascontiguousarray(np.array(Ps).T)
    rng = np.random.default_rng(40)
    N = Q.shape[1]
    S = rng.uniform(0, 2 * math.pi, N)
    a = rng.normal(size=N) + 1j * rng.normal(size=N)
    # the grid points around every packet's centre (a single packet's values at
    # random points are mostly tails far below the rounding of its peak), and
    # some random ones
    Mv = np.array(M)
    near = []
    for j in range(Q.shape[1]):
        c = np.rint((Q[:, j] + math.pi) / (2 * math.pi) * Mv).astype(np.int64)
        for off in np.ndindex(3, 3, 3):
            near.append(np.ravel_multi_index(tuple((c + np.array(off) - 1) % Mv), M))
    pts = np.unique(np.concatenate([np.array(near), rng.choice(int(np.prod(M)), 32, replace=False)]))
    for sel in (slice(0, 1), slice(-1, None), slice(None)):
        q, p, s_, a_ = (np.ascontiguousarray(Q[:, sel]), np.ascontiguousarray(P[:, sel]),
                        np.ascontiguousarray(S[sel]), np.ascontiguousarray(a[sel]))
        log(f"3d edge prec {prec} N={q.shape[1]}")
        u = ctx.reconstruct(t(q), t(p), t(s_), t(a_), eps, M, st, precision=prec)
        torch.cuda.synchronize()
        u = u.cpu().numpy().reshape(-1)[pts].astype(np.complex128)
        ref = orc.fggc(q, p, s_, a_, eps, M, Nq, dp, sd["dq_off"], sd["dp_off"], pts=pts)
        check(u, ref, tol, f"3d edge prec={prec} N={q.shape[1]}")


@pytest.mark.parametrize("name", ["Q2P2", "Q4P2", "Q2P4"])
def test_device_coefficients_match_oracle_lsa(ctx, orc, name):
    # the coefficient kernel's least-squares coefficients (fggc_coefficients)
    # on an 11 x 11 sweep of the first cell (Q = s dq, P = t dp: the shift of
    # eq. 3.13 is 1 there) against the oracle's solve in the eps-free form
    # (Theorem 3); the E_LSA of the device coefficients, by quadrature,
    # against the oracle's E_LSA.  Q2P2 (kappa ~ 1e5) also fixes c itself;
    # the sets of four are compared through E (c is not unique beyond their
    # conditioning).
    eps, C = 1.0 / 64, math.pi / 8
    se = math.sqrt(eps)
    Nq = int(round(2 * math.pi / (C * se)))
    dqm, dpm = 2 * math.pi / Nq, C * se
    Cq, Cp = dqm / se, dpm / se
    dq_off, dp_off = STRATEGIES[name]
    st = F.make_strategy(1, [Nq], [dpm], dq_off, dp_off)
    s1 = np.linspace(0.0, 0.999, 11)
    ss, tt = [g.ravel() for g in np.meshgrid(s1, s1, indexing="ij")]
    Q, P = (ss * dqm)[None, :], (tt * dpm)[None, :]
    N = Q.shape[1]
    c, cells = ctx.coefficients(t(Q), t(P), t(np.zeros(N)), t(np.ones(N, complex)), eps, st)
    torch.cuda.synchronize()
    c, cells = c.cpu().numpy(), cells.cpu().numpy()
    assert np.all(cells[:, 0, 0] == Nq // 2) and np.all(cells[:, 1, 0] == 0)
    qk = np.array([a for a in dq_off for b in dp_off]) * dqm
    pk = np.array([b for a in dq_off for b in dp_off]) * dpm
    x = np.linspace(-14 * se, 14 * se + dqm, 40001)
    h = x[1] - x[0]
    worst_c, worst_e = 0.0, 0.0
    for j in range(N):
        cr, Er = orc.lsa([a for a in dq_off for b in dp_off], [b for a in dq_off for b in dp_off], Cq, Cp,
                         ss[j], tt[j])
        g = np.exp(1j * P[0, j] * (x - Q[0, j]) / eps - (x - Q[0, j]) ** 2 / (2 * eps))
        basis = np.exp(1j * pk[None, :] * (x[:, None] - qk[None, :]) / eps - (x[:, None] - qk[None, :]) ** 2 / (2 * eps))
        r = g - basis @ c[j]
        E = math.sqrt(np.sum(np.abs(r) ** 2) * h / (np.sum(np.abs(g) ** 2) * h))
        # relative to E, with an absolute floor for the mesh points (E ~ 0)
        worst_e = max(worst_e, abs(E - Er) / (Er + 1e-6))
        if name == "Q2P2":
            worst_c = max(worst_c, float(np.max(np.abs(c[j] - cr))) / float(np.max(np.abs(cr))))
    log(f"{name}: worst relative E_LSA difference {worst_e:.2e}, worst coefficient difference {worst_c:.2e}")
    assert worst_e < 1e-3, worst_e
    if name == "Q2P2":
        assert worst_c < 1e-10, worst_c


def test_lsa_maps_error_matches_oracle(ctx, orc):
    # the coefficient and error maps of Sec. 2.2 (Q2P2, Cq = 1/2, Cp = pi/4),
    # computed by the library (coefficient kernel + FP64 direct sum of the
    # residual): E_LSA at every sweep point against the oracle's
    from paper_2504_21785_amd import lsa_maps
    m = lsa_maps.maps(ctx, "Q2P2", 0.5, math.pi / 4, n=5)
    E = np.array(m["E_LSA"])
    worst = 0.0
    for i, s_ in enumerate(m["s"]):
        for j, t_ in enumerate(m["t"]):
            _, Er = orc.lsa([0, 0, 1, 1], [0, 1, 0, 1], 0.5, math.pi / 4, s_, t_)
            if Er < 1e-9:  # a mesh point: both vanish
                assert E[i, j] < 1e-7
                continue
            worst = max(worst, abs(E[i, j] / Er - 1))
    log(f"lsa maps: worst relative E_LSA difference {worst:.2e}, max E {m['summary']['max_E']:.3e}")
    assert worst < 1e-4, worst
