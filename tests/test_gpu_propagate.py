"""The steps either side of the reconstruction on the GPU, against the oracle.

- Packet flow (eq. 2.3-2.6, RK4): both sides integrate the same ODEs with the
  same steps in FP64, so they agree to rounding (rel-L2 <= 1e-11 on Q, P, S,
  A and the Jacobians) over the paper's potentials (1D cosine, 2D Gaussian
  well, 3D harmonic) and mixed ones.
- Initial decomposition (2.7): the same windowed quadrature, <= 1e-12.
- The whole chain u0 -> (2.7) -> flow -> FGGC / direct sum, against the oracle
  chain and a split-step spectral reference written for the tests.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import flow  # noqa: E402
from paper_2504_21785_amd import fggc as F  # noqa: E402
from parity import check  # noqa: E402


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = F.Context(0)
    yield c
    c.close()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def start(d, N, seed):
    rng = np.random.default_rng(seed)
    q = rng.uniform(-0.7, 0.7, (d, N))
    p = 1.0 + 0.5 * rng.standard_normal((d, N))
    S = rng.uniform(0, 1, N)
    A0 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return q, p, S, A0


CASES = {
    "free-1d": (1, dict()),
    "cos-1d": (1, dict(c0=1.0, c1=-1.0, kappa=math.pi)),
    "well-2d": (2, dict(c0=1.0, c2=-1.0, c3=-1.0)),
    "mixed-2d": (2, dict(c0=0.3, w=(0.5, 2.0), c1=0.2, kappa=2.0, c2=0.4, c3=-1.5)),
    "harmonic-3d": (3, dict(w=(1.0, 1.0, 1.0))),
    "mixed-3d": (3, dict(w=(1.0, 0.5, 2.0), c1=0.3, kappa=1.5, c2=-0.5, c3=-1.0)),
}


def jac_to_oracle(jac, d):
    """[N][2][d][d] -> JQ, JP as [d][d][N]."""
    return np.moveaxis(jac[:, 0], 0, -1), np.moveaxis(jac[:, 1], 0, -1)


@pytest.mark.parametrize("name", list(CASES))
def test_flow_matches_oracle(ctx, name):
    d, kw = CASES[name]
    N, n, dt = 777, 400, 2e-3
    q, p, S0, A0 = start(d, N, 5 + d)
    Qd = torch.from_numpy(q.copy()).cuda()
    Pd = torch.from_numpy(p.copy()).cuda()
    Sd = torch.from_numpy(S0.copy()).cuda()
    Ad = torch.from_numpy(A0.copy()).cuda()
    jac = np.zeros((N, 2, d, d), dtype=np.complex128)
    jac[:, 0] = np.eye(d)
    jac[:, 1] = -1j * np.eye(d)
    jd = torch.from_numpy(jac).cuda()
    ctx.propagate(Qd, Pd, Sd, Ad, F.potential(**kw), dt, n, jac=jd)
    torch.cuda.synchronize()
    ref = flow.propagate(q, p, S0, A0, flow.potential(**kw), dt, n)
    jq, jp = jac_to_oracle(jd.cpu().numpy(), d)
    errs = [rel(Qd.cpu().numpy(), ref[0]), rel(Pd.cpu().numpy(), ref[1]), rel(Sd.cpu().numpy(), ref[2]),
            rel(Ad.cpu().numpy(), ref[3]), rel(jq, ref[4]), rel(jp, ref[5])]
    log(name, "rel-L2 Q P S A JQ JP", errs)
    assert max(errs) <= 1e-11


def test_without_jacobian_and_continuation(ctx):
    # jac = NULL starts from dz Q = I, dz P = -i I; two calls with a carried
    # Jacobian equal one call of the summed steps, bit for bit
    d, kw = CASES["well-2d"]
    N, dt = 300, 1e-3
    q, p, S0, A0 = start(d, N, 11)
    V = F.potential(**kw)
    one = [torch.from_numpy(x.copy()).cuda() for x in (q, p, S0, A0)]
    ctx.propagate(*one, V, dt, 300)
    two = [torch.from_numpy(x.copy()).cuda() for x in (q, p, S0, A0)]
    jac = np.zeros((N, 2, d, d), dtype=np.complex128)
    jac[:, 0] = np.eye(d)
    jac[:, 1] = -1j * np.eye(d)
    jd = torch.from_numpy(jac).cuda()
    ctx.propagate(*two, V, dt, 120, jac=jd)
    ctx.propagate(*two, V, dt, 180, jac=jd)
    torch.cuda.synchronize()
    for a, b in zip(one, two):
        assert torch.equal(a, b)
    ref = flow.propagate(q, p, S0, A0, flow.potential(**kw), dt, 300)
    check(one[3].cpu().numpy(), ref[3], 1e-11, "propagate: one[3].cpu().numpy()")


def test_paper_time_step_1d(ctx):
    # the paper's integration: T = 0.8 with dt = 1e-4 (8000 steps), cosine potential
    d, kw = CASES["cos-1d"]
    N = 256
    q, p, S0, A0 = start(d, N, 13)
    xs = [torch.from_numpy(x.copy()).cuda() for x in (q, p, S0, A0)]
    ctx.propagate(*xs, F.potential(**kw), 1e-4, 8000)
    torch.cuda.synchronize()
    ref = flow.propagate(q, p, S0, A0, flow.potential(**kw), 1e-4, 8000)
    errs = [rel(x.cpu().numpy(), r) for x, r in zip(xs, ref[:4])]
    log("T = 0.8, dt = 1e-4:", errs)
    assert max(errs) <= 1e-11


def test_host_buffers_and_errors(ctx):
    d, kw = CASES["mixed-2d"]
    q, p, S0, A0 = start(d, 100, 17)
    Q, P, S, A = q.copy(), p.copy(), S0.copy(), A0.copy()
    ctx.propagate(Q, P, S, A, F.potential(**kw), 1e-3, 200)
    ref = flow.propagate(q, p, S0, A0, flow.potential(**kw), 1e-3, 200)
    assert max(rel(Q, ref[0]), rel(A, ref[3])) <= 1e-11
    # nsteps = 0 and N = 0 change nothing
    Q2 = q.copy()
    ctx.propagate(Q2, p.copy(), S0.copy(), A0.copy(), F.potential(**kw), 1e-3, 0)
    assert np.array_equal(Q2, q)
    e = np.zeros((2, 0))
    ctx.propagate(e, e.copy(), np.zeros(0), np.zeros(0, complex), F.potential(), 1e-3, 10)
    for bad in (dict(dt=math.nan), dict(nsteps=-1)):
        args = dict(dt=1e-3, nsteps=10)
        args.update(bad)
        with pytest.raises(F.FggcError) as ei:
            ctx.propagate(q.copy(), p.copy(), S0.copy(), A0.copy(), F.potential(), args["dt"], args["nsteps"])
        assert ei.value.code == F.FGGC_EINVAL
    with pytest.raises(F.FggcError) as ei:
        ctx.propagate(q.copy(), p.copy(), S0.copy(), A0.copy(), F.potential(c1=math.inf), 1e-3, 10)
    assert ei.value.code == F.FGGC_EINVAL


# --------------------------------------------------------------------------
# initial decomposition (2.7) and the whole chain on the GPU
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,M,eps,N", [(1, (1024,), 1 / 64, 500), (1, (4096,), 1 / 1024, 300),
                                       (2, (128, 96), 1 / 64, 200)])
def test_decompose_matches_oracle(ctx, d, M, eps, N):
    rng = np.random.default_rng(21 + d)
    axes = [-math.pi + 2 * math.pi * np.arange(m) / m for m in M]
    X = np.meshgrid(*axes, indexing="ij")
    r2 = sum(x * x for x in X)
    u0 = (np.exp(-20 * r2 + 1j * sum(X) / eps) * (1 + 0.3 * np.cos(3 * X[0]))).astype(np.complex128)
    q = rng.uniform(-0.6, 0.6, (d, N))
    p = 1.0 + 0.4 * rng.standard_normal((d, N))
    R = 6 * math.sqrt(eps)
    A = ctx.decompose(torch.from_numpy(u0.ravel().copy()).cuda(), eps, M, R,
                      torch.from_numpy(q).cuda(), torch.from_numpy(p).cuda())
    torch.cuda.synchronize()
    ref = flow.decompose(u0.ravel(), eps, list(M), R, q, p)
    check(A.cpu().numpy(), ref, 1e-12, f"decompose d={d} M={M}")
    # host buffers
    Ah = ctx.decompose(u0.ravel().copy(), eps, M, R, q, p)
    check(Ah, ref, 1e-12, "propagate: Ah")


def test_chain_on_gpu_matches_spectral_reference(ctx, orc):
    """u0 -> decomposition -> RK4 flow -> FGGC, all through the library:
    for the harmonic potential the FGA is exact and the chain meets the
    split-step solution; for Example 1's 1 - cos(pi x) the chain's FGA sum
    equals the oracle chain's, and FGGC (Q4P2) differs from it at the LSA level."""
    eps, M, T, n = 1 / 64, 2048, 0.5, 500
    x = -math.pi + 2 * math.pi * np.arange(M) / M
    u0 = (64 / math.pi) ** 0.25 * np.exp(-32 * x * x + 1j * x / eps)
    dq, dp = math.sqrt(eps) / 2, math.pi * math.sqrt(eps) / 8
    qs = np.arange(-0.8, 0.8 + 1e-12, dq)
    ps_ = 1.0 + np.arange(-1.2, 1.2 + 1e-12, dp)
    qq, pp = [g.ravel()[None, :] for g in np.meshgrid(qs, ps_, indexing="ij")]
    scale = dq * dp / (2 * math.pi * eps) ** 1.5
    st = F.default_strategy(1, eps, "Q4P2")
    for name, kw, Vx in (("harmonic", dict(w=(1.0,)), 0.5 * x * x),
                         ("cos", dict(c0=1.0, c1=-1.0, kappa=math.pi), 1 - np.cos(math.pi * x))):
        Qd = torch.from_numpy(qq.copy()).cuda()
        Pd = torch.from_numpy(pp.copy()).cuda()
        A = ctx.decompose(torch.from_numpy(u0.copy()).cuda(), eps, (M,), 8 * math.sqrt(eps), Qd, Pd)
        Sd = torch.zeros(qq.shape[1], dtype=torch.float64, device="cuda")
        ctx.propagate(Qd, Pd, Sd, A, F.potential(**kw), T / n, n)
        uf = ctx.reconstruct(Qd, Pd, Sd, A, eps, (M,), st, scale=scale, precision=F.FP64)
        ud = ctx.direct_sum(Qd, Pd, Sd, A, eps, (M,), 6 * math.sqrt(eps), scale=scale, precision=F.FP64)
        torch.cuda.synchronize()
        uf, ud = uf.cpu().numpy(), ud.cpu().numpy()
        ref = split_step_1d(u0, Vx, eps, T, 4000)
        # the oracle chain on the same inputs
        A0 = flow.decompose(u0, eps, [M], 8 * math.sqrt(eps), qq, pp)
        Qo, Po, So, Ao, _, _ = flow.propagate(qq, pp, np.zeros(qq.shape[1]), A0, flow.potential(**kw), T / n, n)
        uo = orc.direct_sum(Qo, Po, So, Ao, eps, [M], 6 * math.sqrt(eps), scale)
        e_ref = rel(ud, ref)
        log("chain", name, "FGA vs split-step", e_ref)
        check(ud, uo, 1e-11, f"chain {name}: FGA gpu vs oracle")
        check(uf, ud, 1e-6, f"chain {name}: FGGC vs FGA")
        if name == "harmonic":
            assert e_ref <= 5e-7
            check(uf, ref, 1e-6, "propagate: uf")


def split_step_1d(u0, Vx, eps, T, nsteps):
    """Strang splitting of i eps u_t = -eps^2/2 u_xx + V u (test reference)."""
    M = u0.size
    k = np.fft.fftfreq(M, d=1.0 / M)
    dt = T / nsteps
    half = np.exp(-1j * Vx * dt / (2 * eps))
    kin = np.exp(-1j * eps * k * k * dt / 2)
    u = u0.copy()
    for _ in range(nsteps):
        u = half * np.fft.ifft(kin * np.fft.fft(half * u))
    return u


@pytest.mark.parametrize("M,Nq,eps,q_n,p_n", [((1024,), (128,), 1 / 64, (40,), (23,)),
                                              ((256, 128), (64, 32), 1 / 64, (8, 4), (6, 5)),
                                              ((512, 512), (128, 128), 1 / 256, (4, 5), (5, 4))])
def test_decompose_mesh_matches_oracle(ctx, M, Nq, eps, q_n, p_n):
    """The GEMM form of (2.7) on a mesh with q on grid points, against the
    oracle's quadrature with the same box window on the same (q, p) list."""
    d = len(M)
    axes = [-math.pi + 2 * math.pi * np.arange(m) / m for m in M]
    X = np.meshgrid(*axes, indexing="ij")
    u0 = (np.exp(-20 * sum(x * x for x in X) + 1j * sum(X) / eps) * (1 + 0.3 * np.cos(3 * X[0]))).astype(np.complex128)
    dp = [math.pi * math.sqrt(eps) / 8] * d
    q_lo = [Nq[k] // 2 - q_n[k] // 2 for k in range(d)]
    p_lo = [int(round(1.0 / dp[k])) - p_n[k] // 2 for k in range(d)]  # about the momentum of u0
    R = 8 * math.sqrt(eps)
    A = ctx.decompose_mesh(torch.from_numpy(u0.ravel().copy()).cuda(), eps, M, R, Nq, q_lo, q_n, dp, p_lo, p_n)
    torch.cuda.synchronize()
    qs = [-math.pi + (q_lo[k] + np.arange(q_n[k])) * 2 * math.pi / Nq[k] for k in range(d)]
    ps = [(p_lo[k] + np.arange(p_n[k])) * dp[k] for k in range(d)]
    qg = np.stack([g.ravel() for g in np.meshgrid(*qs, indexing="ij")])
    pg = np.stack([g.ravel() for g in np.meshgrid(*ps, indexing="ij")])
    qm = np.repeat(qg, pg.shape[1], axis=1)
    pm = np.tile(pg, (1, qg.shape[1]))
    ref = flow.decompose(u0.ravel(), eps, list(M), R, qm, pm, window="box")
    check(A.cpu().numpy(), ref, 1e-12, f"decompose_mesh M={M} Nq={Nq}")
    Ah = ctx.decompose_mesh(u0.ravel().copy(), eps, M, R, Nq, q_lo, q_n, dp, p_lo, p_n)
    check(Ah, ref, 1e-12, "propagate: Ah")
    # the ball-window quadrature differs by terms below exp(-32)
    Ab = ctx.decompose(torch.from_numpy(u0.ravel().copy()).cuda(), eps, M, R, torch.from_numpy(qm).cuda(),
                       torch.from_numpy(pm).cuda())
    check(Ab.cpu().numpy(), ref, 1e-12, "propagate: Ab.cpu().numpy()")


def test_decompose_mesh_errors(ctx):
    u0 = np.zeros(256, dtype=np.complex128)
    for kw in (dict(Nq=(100,)), dict(q_lo=(-1,)), dict(q_n=(200,)), dict(p_n=(0,)), dict(R=math.pi)):
        args = dict(Nq=(128,), q_lo=(0,), q_n=(4,), p_n=(3,), R=0.5)
        args.update(kw)
        with pytest.raises(F.FggcError) as ei:
            ctx.decompose_mesh(u0, 1 / 64, (256,), args["R"], args["Nq"], args["q_lo"], args["q_n"], (0.05,), (0,),
                               args["p_n"])
        assert ei.value.code == F.FGGC_EINVAL
    with pytest.raises(F.FggcError) as ei:
        ctx.decompose_mesh(np.zeros(8 ** 3, dtype=np.complex128), 1 / 64, (8, 8, 8), 0.5, (8, 8, 8), (0, 0, 0),
                           (2, 2, 2), (0.1,) * 3, (0, 0, 0), (2, 2, 2))
    assert ei.value.code == F.FGGC_EUNSUPPORTED
