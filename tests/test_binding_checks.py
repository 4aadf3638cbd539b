"""The binding refuses buffers the kernels would read or write out of bounds.

Every check runs before any library call, so these tests need no GPU: a
Context object is made without a device context, and each call must raise
ValueError (or TypeError) on its arguments alone.
"""
import numpy as np
import pytest

from paper_2504_21785_amd import fggc as F


@pytest.fixture
def ctx():
    return object.__new__(F.Context)  # no device context: only the argument checks can run


def packets(d=1, N=10):
    rng = np.random.default_rng(1)
    return (rng.standard_normal((d, N)), rng.standard_normal((d, N)), rng.standard_normal(N),
            rng.standard_normal(N) + 1j * rng.standard_normal(N))


def test_check_packets_accepts_good_sets():
    for d in (1, 2, 3):
        assert F.check_packets(*packets(d, 7)) == (d, 7)
    assert F.check_packets(*packets(2, 0)) == (2, 0)


@pytest.mark.parametrize("bad", [
    lambda Q, P, S, a: (Q.astype(np.float32), P, S, a),          # float32 centres
    lambda Q, P, S, a: (Q, P.astype(np.float32), S, a),
    lambda Q, P, S, a: (Q, P, S.astype(np.float32), a),
    lambda Q, P, S, a: (Q, P, S, a.astype(np.complex64)),        # complex64 amplitudes
    lambda Q, P, S, a: (Q, P, S, a.real.copy()),                 # real amplitudes
    lambda Q, P, S, a: (Q, P[:, :-1].copy(), S, a),              # N mismatch
    lambda Q, P, S, a: (Q, P, S[:-1].copy(), a),
    lambda Q, P, S, a: (Q, P, S, a[:-1].copy()),
    lambda Q, P, S, a: (Q, np.vstack([P, P]), S, a),             # d mismatch
    lambda Q, P, S, a: (Q[0].copy(), P, S, a),                   # Q not [d][N]
    lambda Q, P, S, a: (np.asfortranarray(np.vstack([Q, Q])), np.vstack([P, P]), S, a),  # not contiguous
    lambda Q, P, S, a: (np.zeros((4, Q.shape[1])), np.zeros((4, Q.shape[1])), S, a),     # d = 4
])
def test_bad_packets_refused(ctx, bad):
    Q, P, S, a = bad(*packets(1, 10))
    with pytest.raises((ValueError, TypeError)):
        F.check_packets(Q, P, S, a)
    with pytest.raises((ValueError, TypeError)):
        ctx.reconstruct(Q, P, S, a, 1 / 64, (64,), F.Strategy())
    with pytest.raises((ValueError, TypeError)):
        ctx.direct_sum(Q, P, S, a, 1 / 64, (64,), 0.5)


def test_bad_out_refused(ctx):
    Q, P, S, a = packets(2, 10)
    st = F.Strategy()
    cases = [
        (np.zeros((64, 64), np.complex128), F.FP32),   # FP64 buffer for the FP32 path
        (np.zeros((64, 64), np.complex64), F.FP64),    # FP32 buffer for the FP64 path
        (np.zeros((64, 63), np.complex64), F.FP32),    # too small
        (np.zeros((65, 64), np.complex64), F.FP32),    # too large
        (np.zeros((64, 64), np.float64), F.FP32),      # real
        (np.zeros((64, 128), np.complex64)[:, ::2], F.FP32),  # strided view
    ]
    for out, prec in cases:
        with pytest.raises((ValueError, TypeError)):
            ctx.reconstruct(Q, P, S, a, 1 / 64, (64, 64), st, precision=prec, out=out)
        with pytest.raises((ValueError, TypeError)):
            ctx.direct_sum(Q, P, S, a, 1 / 64, (64, 64), 0.5, precision=prec, out=out)
    with pytest.raises(ValueError):
        ctx.reconstruct(Q, P, S, a, 1 / 64, (64, 64), st, precision=7)
    with pytest.raises(ValueError):
        ctx.reconstruct(Q, P, S, a, 1 / 64, (64, 64, 64), st)  # grid rank != d
    with pytest.raises(ValueError):
        ctx.direct_sum_box(Q, P, S, a, 1 / 64, (64, 64), (0, 0), (8, 8), 0.5,
                           out=np.zeros(63, np.complex64))


def test_torch_cpu_and_dtype_checks(ctx):
    torch = pytest.importorskip("torch")
    Q, P, S, a = (torch.from_numpy(x) for x in packets(1, 12))
    assert F.check_packets(Q, P, S, a) == (1, 12)
    with pytest.raises(ValueError):
        F.check_packets(Q.float(), P, S, a)
    with pytest.raises(ValueError):
        F.check_packets(Q, P, S, a.to(torch.complex64))
    with pytest.raises(ValueError):
        F.check_packets(Q, P, S, a[:-1])
    # mixed host kinds are one place (host); a mixed host/device set is refused on a GPU machine only


def test_other_entry_points(ctx):
    Q, P, S, a = packets(1, 8)
    u0 = np.zeros(64, np.complex128)
    with pytest.raises(ValueError):
        ctx.decompose(u0.astype(np.complex64), 1 / 64, (64,), 0.5, Q, P)
    with pytest.raises(ValueError):
        ctx.decompose(u0[:-1], 1 / 64, (64,), 0.5, Q, P)
    with pytest.raises(ValueError):
        ctx.decompose(u0, 1 / 64, (64,), 0.5, Q, P[:, :-1].copy())
    with pytest.raises(ValueError):
        ctx.decompose(u0, 1 / 64, (64,), 0.5, Q, P, out=np.zeros(7, np.complex128))
    with pytest.raises(ValueError):
        ctx.propagate(Q, P, S, a, F.potential(), 1e-3, 1, jac=np.zeros(5, np.complex128))
    with pytest.raises(ValueError):
        ctx.propagate(Q, P.astype(np.float32), S, a, F.potential(), 1e-3, 1)
    with pytest.raises(ValueError):
        ctx.fft(np.zeros(64, np.complex64), (64,), 1, -1, F.FP32)  # host memory
    with pytest.raises(ValueError):
        ctx.decompose_mesh(u0[:-1], 1 / 64, (64,), 0.5, [16], [0], [16], [0.1], [0], [4])


@pytest.mark.parametrize("bad", ["A0", "learned", "keep_idx", "new_idx"])
def test_learn_select_refuses_wrong_dtypes_and_sizes(ctx, bad):
    Nm = 12
    args = {"A0": np.zeros(Nm, np.complex128), "learned": np.zeros(Nm, np.uint8),
            "keep_idx": np.zeros(Nm, np.int64), "new_idx": np.zeros(Nm, np.int64)}
    wrong = {"A0": np.zeros(Nm, np.complex64), "learned": np.zeros(Nm, np.bool_),
             "keep_idx": np.zeros(Nm, np.int32), "new_idx": np.zeros(Nm - 1, np.int64)}
    args[bad] = wrong[bad]
    with pytest.raises(ValueError):
        ctx.learn_select(args["A0"], 1e-12, args["learned"], args["keep_idx"], args["new_idx"])
