"""Serving (fggc_server_*) on the GPU through the C ABI.

Each request's result from the server, submitted in a mix with others and
repeated so that its pipeline runs eagerly, is captured into a graph and is
replayed (per slot), must equal the same request run alone through the synchronous entry
point, within the FP32 tolerance.  Requests follow the serving stream's
distribution (mixed 1D/2D, eps, grid) with packet counts kept small here.
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


def rel(u, ref):
    n = np.linalg.norm(ref)
    return float(np.linalg.norm(u - ref) / n) if n > 0 else float(np.linalg.norm(u))


def small_requests(n_max=2 ** 17, count=8):
    """The first `count` requests of the serving stream with N <= n_max,
    covering both dimensions."""
    out = []
    for r in range(400):
        u = W.uniform(W.BASE_SEED * 1000 + r, 10, 4)
        N = int(math.floor(2.0 ** (12 + 10 * u[1])))
        if N <= n_max:
            out.append(W.serving_request(r))
        if len(out) == count:
            break
    assert {p.d for p in out} == {1, 2}
    return out


@pytest.fixture(scope="module")
def ctx():
    c = F.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def reqs():
    return small_requests()


def t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def alone(ctx, ps, fggc=True):
    st = F.default_strategy(ps.d, ps.eps, "Q4P2") if fggc else None
    if fggc:
        u = ctx.reconstruct(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, st, precision=F.FP32)
    else:
        u = ctx.direct_sum(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, 6 * math.sqrt(ps.eps), precision=F.FP32)
    return np.asarray(u)


def test_server_mix_equals_alone_host_inputs(ctx, reqs):
    ref = [alone(ctx, ps) for ps in reqs]
    srv = F.Server(ctx, n_streams=3)
    # a shape runs eagerly on its first sighting and is captured on its second;
    # a graph belongs to the slot that captured it, so a repeat may land on a
    # slot that captures it anew -- at most once per (shape, slot): with 8
    # shapes and 3 slots, 6 rounds leave at least 48 - 8 - 24 replays
    rounds = 6
    try:
        for rnd in range(rounds):
            tickets = []
            for ps in reqs:
                st = F.default_strategy(ps.d, ps.eps, "Q4P2")
                tickets.append(srv.submit(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, st))
            for i, (tk, out) in enumerate(tickets):
                rc = srv.wait(tk, 120.0)
                assert rc == F.FGGC_OK, (i, rc, F.last_error())
                check(out, ref[i], 1e-6, f"round {rnd} req {reqs[i].name} d={reqs[i].d} N={reqs[i].N} "
                      f"M={reqs[i].M} eps={reqs[i].eps:.5f}: mix vs alone")
        c = srv.counters()
        log("counters", c, srv.stats())
        assert c["captured"] >= 1 and c["replayed"] >= 1
        assert c["eager"] + c["captured"] + c["replayed"] == rounds * len(reqs)
        s = srv.stats()
        assert s["completed"] == rounds * len(reqs) and s["p99_s"] >= s["p50_s"] > 0
    finally:
        srv.close()


def test_server_device_inputs_and_direct(ctx, reqs):
    srv = F.Server(ctx, n_streams=2)
    try:
        sub = reqs[:4]
        dev = [(t(ps.Q), t(ps.P), t(ps.S), t(ps.a)) for ps in sub]
        torch.cuda.synchronize()
        tickets = []
        for ps, (Q, P, S, a) in zip(sub, dev):
            st = F.default_strategy(ps.d, ps.eps, "Q4P2")
            tickets.append(("fggc", ps, srv.submit(Q, P, S, a, ps.eps, ps.M, st)))
            tickets.append(("direct", ps, srv.submit(Q, P, S, a, ps.eps, ps.M, None)))
        for kind, ps, (tk, out) in tickets:
            rc = srv.wait(tk, 120.0)
            assert rc == F.FGGC_OK, (kind, rc, F.last_error())
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            check(got, alone(ctx, ps, fggc=(kind == "fggc")), 1e-6, f"device {kind} {ps.name}")
    finally:
        srv.close()


def test_server_against_oracle(ctx, orc):
    # a small 2D request with M = 256 < Nq = 512 (eps = 1/1024), sampled points
    rng = np.random.default_rng(7)
    N, eps = 3000, 1.0 / 1024
    q = rng.uniform(-math.pi, math.pi, (2, N)) * 0.5
    p = np.array([0.5, 0.3])[:, None] - 0.25 + 0.5 * rng.uniform(size=(2, N))
    a = np.exp(-10 * np.sum(q * q, axis=0)) * np.exp(1j * rng.uniform(0, 2 * math.pi, N))
    ps = W.PacketSet("srv2d", 2, eps, (256, 256), np.ascontiguousarray(W.wrap(q + 0.5 * p)),
                     np.ascontiguousarray(p), rng.uniform(0, 2 * math.pi, N), a, 6 * math.sqrt(eps))
    st = F.default_strategy(2, ps.eps, "Q4P2")
    srv = F.Server(ctx, n_streams=1)
    try:
        tk, out = srv.submit(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, st)
        assert srv.wait(tk, 120.0) == F.FGGC_OK, F.last_error()
    finally:
        srv.close()
    sd = st.describe()
    order = np.argsort(-np.abs(ps.a))[:40]
    m = np.rint((ps.Q[:, order] + math.pi) / (2 * math.pi) * 256).astype(np.int64) % 256
    pts = np.unique(np.ravel_multi_index((m[0], m[1]), (256, 256)))
    ref = orc.fggc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, sd["Nq"][:2], sd["dp"][:2], sd["dq_off"],
                   sd["dp_off"], pts=pts)
    check(out.reshape(-1)[pts], ref, 1e-6, "server 2D (M < Nq) vs oracle FGGC, sampled")


def test_server_budget_and_timeout(ctx):
    small = F.Context(0, hbm_budget_bytes=96 << 20)
    srv = F.Server(small, n_streams=2)
    try:
        big = W.gen_mesh(2, 64, 32, 0.5, (0.5, 0.3), 1.0 / 256, 1024, seed=5)  # ~4M packets
        st = F.default_strategy(2, big.eps, "Q4P2")
        with pytest.raises(F.FggcError) as ei:
            srv.submit(big.Q, big.P, big.S, big.a, big.eps, big.M, st)
        assert ei.value.code == F.FGGC_EBUDGET
        ps = W.gen_1d(64, 64, 1.0 / 256, 2048, seed=6)
        st1 = F.default_strategy(1, ps.eps, "Q4P2")
        tk, out = srv.submit(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, st1)
        assert srv.wait(tk, 120.0) == F.FGGC_OK
        assert rel(out, alone(ctx, ps)) <= 1e-6
        assert srv.wait(tk, 1.0) == F.FGGC_EINVAL  # already waited
        # empty request completes at once with zeros
        e = np.zeros((1, 0))
        tk, out = srv.submit(e, e, np.zeros(0), np.zeros(0, complex), ps.eps, ps.M, st1)
        assert srv.wait(tk, 10.0) == F.FGGC_OK and not np.any(out)
    finally:
        srv.close()
        small.close()


def test_server_tiny_requests_padding(ctx):
    # N below the smallest bucket (64) or just above a bucket edge: the
    # zero-amplitude padding copies wrap around the real packets several times
    srv = F.Server(ctx, n_streams=2)
    try:
        for d in (1, 2):
            for N in (1, 5, 37, 65, 300):
                base = W.serving_request(0 if d == 1 else 1)
                assert base.d == d
                sel = np.sort(np.argsort(-np.abs(base.a))[:N])  # packets that matter in FP32
                ps = W.PacketSet(f"tiny{d}_{N}", d, base.eps, base.M, np.ascontiguousarray(base.Q[:, sel]),
                                 np.ascontiguousarray(base.P[:, sel]), np.ascontiguousarray(base.S[sel]),
                                 np.ascontiguousarray(base.a[sel]), base.R)
                ref = alone(ctx, ps)
                st = F.default_strategy(d, ps.eps, "Q4P2")
                for rep in range(3):  # eager, captured, replayed
                    tk, out = srv.submit(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, st)
                    assert srv.wait(tk, 120.0) == F.FGGC_OK, F.last_error()
                    e = rel(out, ref)
                    log(f"tiny d={d} N={N} rep {rep}: server vs alone {e:.2e}")
                    assert e <= 1e-6
    finally:
        srv.close()


def test_server_padding_keeps_cells_balanced(ctx):
    # A 2D request at eps = 1/1024 (radix-sorted, so it runs eagerly every
    # time) padded by ~17% to its bucket.  Copies of a single packet would
    # crowd one cell, whose bin one wave accumulates alone; the server then
    # took over ten times the synchronous call.  Loose bound: 4x + 10 ms.
    import time
    ps = W.serving_request(11)
    assert ps.d == 2 and ps.eps == 1.0 / 1024
    st = F.default_strategy(2, ps.eps, "Q4P2")
    dev = (t(ps.Q), t(ps.P), t(ps.S), t(ps.a))
    torch.cuda.synchronize()
    ctx.reconstruct(*dev, ps.eps, ps.M, st)
    torch.cuda.synchronize()
    t_sync = 1e9
    for _ in range(3):
        t0 = time.perf_counter()
        ctx.reconstruct(*dev, ps.eps, ps.M, st)
        torch.cuda.synchronize()
        t_sync = min(t_sync, time.perf_counter() - t0)
    srv = F.Server(ctx, n_streams=1)
    try:
        t_srv = 1e9
        for _ in range(3):
            t0 = time.perf_counter()
            tk, _ = srv.submit(*dev, ps.eps, ps.M, st)
            assert srv.wait(tk, 120.0) == F.FGGC_OK, F.last_error()
            t_srv = min(t_srv, time.perf_counter() - t0)
    finally:
        srv.close()
    log(f"N={ps.N}: server {t_srv * 1e3:.2f} ms, synchronous {t_sync * 1e3:.2f} ms")
    assert t_srv <= 4 * t_sync + 0.010


def test_server_replays_a_two_level_sort_shape(ctx):
    # A 2D eps = 1/1024 request has more than 2^15 sort bins, so it sorts in two
    # counting levels; its pipeline is captured on its second sighting and
    # replayed after, and every result equals the request run alone.
    ps = None
    for r in range(2000):
        u = W.uniform(W.BASE_SEED * 1000 + r, 10, 4)
        N = int(math.floor(2.0 ** (12 + 10 * u[1])))
        if u[0] >= 0.5 and min(int(u[2] * 3), 2) == 2 and N <= 2 ** 16:
            ps = W.serving_request(r)
            break
    assert ps is not None and ps.d == 2 and ps.eps == 1.0 / 1024
    log(f"request {ps.name}: N={ps.N} M={ps.M}")
    ref = alone(ctx, ps)
    dev = tuple(t(x) for x in (ps.Q, ps.P, ps.S, ps.a))
    st = F.default_strategy(2, ps.eps, "Q4P2")
    srv = F.Server(ctx, n_streams=1)
    try:
        for i in range(4):
            out = torch.empty(ps.M, dtype=torch.complex64, device="cuda")
            tk, _ = srv.submit(*dev, ps.eps, ps.M, st, out=out)
            assert srv.wait(tk, 120.0) == F.FGGC_OK, F.last_error()
            check(out.cpu().numpy(), ref, 1e-6, f"served call {i} vs alone")
        c = srv.counters()
        log("graph counters", c)
        assert c["captured"] >= 1 and c["replayed"] >= 1, c
    finally:
        srv.close()
