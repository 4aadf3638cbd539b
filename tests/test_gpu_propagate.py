"""Packet flow (eq. 2.3-2.6, RK4) on the GPU against the flow oracle.

Both integrate the same ODEs with the same RK4 steps in FP64, so they agree
to rounding: rel-L2 <= 1e-11 on Q, P, S, A and the Jacobians, over the
paper's potentials (1D cosine, 2D Gaussian well, 3D harmonic) and a mixed
one, from initial packets and from a given Jacobian state.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import flow  # noqa: E402
from paper_2504_21785_amd import fggc as F  # noqa: E402


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
    assert rel(one[3].cpu().numpy(), ref[3]) <= 1e-11


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
