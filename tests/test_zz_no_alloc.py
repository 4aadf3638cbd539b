"""fggc_direct_sum_noalloc (the entry point that allocates nothing) against
fggc_direct_sum, through the C ABI.

Both run the same kernels, so the bar is the direct sum's own: FP32 rel-L2 and
max-abs <= 1e-6, FP64 <= 1e-12.  Two calls in a row on the shared scratch, the
second with a smaller input (its result must not see the first call's
scratch contents), then a 2D call, and a request over the scratch limit, which
must fail with FGGC_EBUDGET and leave the output untouched.
"""
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


def dev(ps):
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t(ps.Q), t(ps.P), t(ps.S), t(ps.a)


def out_like(ps, precision):
    dt = torch.complex64 if precision == F.FP32 else torch.complex128
    return torch.full(tuple(ps.M), complex(7.0, -3.0), dtype=dt, device="cuda")


def test_noalloc_matches_direct_sum_on_two_calls():
    ctx = F.Context(0)
    try:
        cases = [
            ("1D N=2^18 M=8192 FP32", W.gen_1d(512, 512, 1.0 / 1024, 8192, seed=W.BASE_SEED + 71), F.FP32, 1e-6),
            ("1D N=2^11 M=1024 FP32 (smaller)", W.gen_1d(64, 32, 1.0 / 64, 1024, seed=W.BASE_SEED + 72), F.FP32,
             1e-6),
            ("1D N=2^12 M=2048 FP64", W.gen_1d(64, 64, 1.0 / 256, 2048, seed=W.BASE_SEED + 73), F.FP64, 1e-12),
            ("2D N=2^14 M=256^2 FP32", W.gen_mesh(2, 32, 4, 0.5, (0.5, 0.3), 1.0 / 256, 256,
                                                  seed=W.BASE_SEED + 74), F.FP32, 1e-6),
        ]
        for what, ps, prec, tol in cases:
            log(f"case {what}: N={ps.N} M={ps.M}")
            Q, P, S, a = dev(ps)
            ref = ctx.direct_sum(Q, P, S, a, ps.eps, ps.M, ps.R, precision=prec)
            u = out_like(ps, prec)
            ctx.direct_sum_noalloc(Q, P, S, a, ps.eps, ps.M, ps.R, u, precision=prec)
            torch.cuda.synchronize()
            check(u.cpu().numpy(), ref.cpu().numpy(), tol, f"noalloc vs direct_sum, {what}")
    finally:
        ctx.close()


def test_noalloc_rejects_requests_over_the_scratch_limit():
    ctx = F.Context(0)
    try:
        # ~3e6 packets need more than the fixed scratch (records alone are 96 B each)
        N = 3 * (1 << 20)
        M = 16384
        Q = torch.zeros((1, N), dtype=torch.float64, device="cuda")
        P = torch.full((1, N), 0.5, dtype=torch.float64, device="cuda")
        S = torch.zeros(N, dtype=torch.float64, device="cuda")
        a = torch.zeros(N, dtype=torch.complex128, device="cuda")
        u = torch.full((M,), complex(7.0, -3.0), dtype=torch.complex64, device="cuda")
        log(f"over-limit request: N={N} M={M}")
        with pytest.raises(F.FggcError) as ei:
            ctx.direct_sum_noalloc(Q, P, S, a, 1.0 / 1024, (M,), 6.0 / 32.0, u)
        assert ei.value.code == F.FGGC_EBUDGET, ei.value
        torch.cuda.synchronize()
        assert bool(torch.all(u == complex(7.0, -3.0)).item())
        # host buffers are refused (staging them would allocate)
        ps = W.gen_1d(16, 16, 1.0 / 64, 256, seed=W.BASE_SEED + 75)
        with pytest.raises(F.FggcError) as ei:
            ctx.direct_sum_noalloc(ps.Q, ps.P, ps.S, ps.a, ps.eps, ps.M, ps.R, u[:256])
        assert ei.value.code == F.FGGC_EINVAL, ei.value
    finally:
        ctx.close()
