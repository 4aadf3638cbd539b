"""Pins of the flow oracle (eq. 2.3-2.6, RK4) against closed forms and invariants.

- V = 0: Q = q + t p, S = t |p|^2 / 2, Z = (2 - i t) I and A = A0 (1 - i t/2)^{d/2}.
- Harmonic V = sum_k w_k x_k^2 / 2: the closed-form flow, action and
  Z_k = 2 cos(w t) - i (w + 1/w) sin(w t) per dimension (w = sqrt(w_k)).
- The paper's cosine and exponential potentials: energy |P|^2/2 + V(Q) is
  conserved, the real Jacobian of (q, p) -> (Q, P) is symplectic, and
  A^2 / A0^2 = det Z / det Z(0) (eq. 2.6 integrates to this).
"""
import math

import numpy as np
import pytest

from oracle import flow


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def start(d, N, seed, q_scale=0.8):
    rng = np.random.default_rng(seed)
    q = rng.uniform(-q_scale, q_scale, (d, N))
    p = 1.0 + 0.5 * rng.standard_normal((d, N))
    A0 = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return q, p, A0


@pytest.mark.parametrize("d", [1, 2])
def test_free_flow_closed_form(d):
    q, p, A0 = start(d, 50, 1)
    t, n = 0.8, 400
    Q, P, S, A, JQ, JP = flow.propagate(q, p, np.zeros(50), A0, flow.potential(), t / n, n)
    assert rel(Q, q + t * p) < 1e-13
    assert rel(P, p) == 0.0
    assert rel(S, t * np.sum(p * p, axis=0) / 2) < 1e-13
    assert rel(A, A0 * (1 - 0.5j * t) ** (d / 2)) < 1e-12
    eye = np.eye(d)[:, :, None]
    assert rel(JQ, (1 - 1j * t) * eye + 0 * JQ) < 1e-13
    assert rel(JP, -1j * eye + 0 * JP) < 1e-13


def test_harmonic_closed_form():
    d, N = 2, 40
    q, p, A0 = start(d, N, 2)
    wk = np.array([1.0, 2.25])
    om = np.sqrt(wk)[:, None]
    t, n = 0.8, 800
    Q, P, S, A, JQ, JP = flow.propagate(q, p, np.zeros(N), A0, flow.potential(w=wk), t / n, n)
    c, s = np.cos(om * t), np.sin(om * t)
    assert rel(Q, q * c + p / om * s) < 1e-12
    assert rel(P, p * c - q * om * s) < 1e-12
    S_ex = np.sum((p * p - om * om * q * q) * np.sin(2 * om * t) / (4 * om) - p * q * s * s, axis=0)
    assert rel(S, S_ex) < 1e-11
    Zk = 2 * c - 1j * (om + 1 / om) * s  # [d][1]
    assert rel(A, A0 * np.prod(np.sqrt(Zk / 2), axis=0)) < 1e-11
    Z = JQ + 1j * JP
    for k in range(d):
        assert np.allclose(Z[k, k], Zk[k, 0], rtol=1e-11, atol=0)
        assert np.allclose(Z[k, 1 - k], 0.0, atol=1e-14)


def real_jacobian(JQ, JP):
    """[[dQ/dq, dQ/dp], [dP/dq, dP/dp]] from dz = d_q - i d_p of real maps."""
    return np.block([[JQ.real.transpose(2, 0, 1), -JQ.imag.transpose(2, 0, 1)],
                     [JP.real.transpose(2, 0, 1), -JP.imag.transpose(2, 0, 1)]])


@pytest.mark.parametrize("d,V", [
    (1, flow.potential(c0=1.0, c1=-1.0, kappa=math.pi)),          # 1 - cos(pi x)
    # Example 2's V1 read as 1 - exp(-(x^2 + y^2)): the printed exp(+(x^2 + y^2))
    # pushes packets out to infinity in finite time
    (2, flow.potential(c0=1.0, c2=-1.0, c3=-1.0)),
    (2, flow.potential(c0=0.3, w=(0.5, 2.0), c1=0.2, kappa=2.0, c2=0.4, c3=-1.5)),
])
def test_invariants(d, V):
    N = 30
    q, p, A0 = start(d, N, 3 + d, q_scale=0.6)
    t, n = 0.8, 800
    Q, P, S, A, JQ, JP = flow.propagate(q, p, np.zeros(N), A0, V, t / n, n)
    H0 = 0.5 * np.sum(p * p, axis=0) + flow.v_grad_hess(V, q)[0]
    H1 = 0.5 * np.sum(P * P, axis=0) + flow.v_grad_hess(V, Q)[0]
    assert np.max(abs(H1 - H0) / (1 + abs(H0))) < 1e-9
    # the motion is not trivial
    assert np.max(abs(P - p)) > 0.05
    Mj = real_jacobian(JQ, JP)
    Om = np.block([[np.zeros((d, d)), np.eye(d)], [-np.eye(d), np.zeros((d, d))]])
    assert np.max(abs(np.einsum("nji,jk,nkl->nil", Mj, Om, Mj) - Om)) < 1e-9
    Z = (JQ + 1j * JP).transpose(2, 0, 1)
    detZ = np.linalg.det(Z)
    assert rel(A * A, A0 * A0 * detZ / 2 ** d) < 1e-9


def test_planted_errors_fail():
    """A wrong sign in the force or a missing 1/2 in (2.6) breaks the pins above."""
    V = flow.potential(c0=1.0, c1=-1.0, kappa=math.pi)
    q, p, A0 = start(1, 20, 9, q_scale=0.6)
    good = flow.propagate(q, p, np.zeros(20), A0, V, 1e-3, 800)
    orig = flow._rhs

    def bad_force(V_, Q, P, S, A, JQ, JP):
        r = list(orig(V_, Q, P, S, A, JQ, JP))
        r[1] = -r[1]
        return tuple(r)

    def bad_amp(V_, Q, P, S, A, JQ, JP):
        r = list(orig(V_, Q, P, S, A, JQ, JP))
        r[3] = 2 * r[3]
        return tuple(r)

    try:
        flow._rhs = bad_force
        Q, P = flow.propagate(q, p, np.zeros(20), A0, V, 1e-3, 800)[:2]
        H0 = 0.5 * p * p + flow.v_grad_hess(V, q)[0]
        H1 = 0.5 * P * P + flow.v_grad_hess(V, Q)[0]
        assert np.max(abs(H1 - H0)) > 1e-3
        flow._rhs = bad_amp
        A, JQ, JP = flow.propagate(q, p, np.zeros(20), A0, V, 1e-3, 800)[3:]
        detZ = (JQ + 1j * JP)[0, 0]
        assert rel(A * A, A0 * A0 * detZ / 2) > 1e-3
    finally:
        flow._rhs = orig
    assert rel(good[0], q) > 0.1


# --------------------------------------------------------------------------
# initial decomposition (2.7)
# --------------------------------------------------------------------------

def gaussian_transform(alpha, beta, eps, q, p):
    """u0^ of u0 = exp(-alpha y^2 + i beta y) in closed form (one dimension):
    int exp(-a y^2 + b y + c) dy = sqrt(pi / a) exp(b^2 / (4 a) + c)."""
    a = alpha + 1 / (2 * eps)
    b = 1j * beta - 1j * p / eps + q / eps
    c = 1j * p * q / eps - q * q / (2 * eps)
    return np.sqrt(np.pi / a) * np.exp(b * b / (4 * a) + c)


def test_decomposition_gaussian_closed_form():
    eps, M, alpha, beta = 1 / 64, 2048, 32.0, 64.0
    x = -math.pi + 2 * math.pi * np.arange(M) / M
    u0 = np.exp(-alpha * x * x + 1j * beta * x)
    rng = np.random.default_rng(4)
    q = rng.uniform(-0.4, 0.4, (1, 40))
    p = 1.0 + 0.3 * rng.standard_normal((1, 40))
    A = flow.decompose(u0, eps, [M], 8 * math.sqrt(eps), q, p)
    ref = math.sqrt(2) * gaussian_transform(alpha, beta, eps, q[0], p[0])
    assert rel(A, ref) < 1e-12
    # 2D: a product Gaussian decomposes into the product of 1D transforms (2^{d/2} = 2)
    M2 = 256
    x2 = -math.pi + 2 * math.pi * np.arange(M2) / M2
    eps2 = 1 / 16
    g1 = np.exp(-8.0 * x2 * x2 + 4j * x2)
    g2 = np.exp(-6.0 * x2 * x2 - 2j * x2)
    u2 = np.outer(g1, g2)
    q2 = rng.uniform(-0.3, 0.3, (2, 12))
    p2 = rng.uniform(-1, 1, (2, 12))
    A2 = flow.decompose(u2, eps2, [M2, M2], 3.0, q2, p2)
    ref2 = 2 * gaussian_transform(8.0, 4.0, eps2, q2[0], p2[0]) * gaussian_transform(6.0, -2.0, eps2, q2[1], p2[1])
    assert rel(A2, ref2) < 1e-10


def test_decomposition_reproduces_u0(orc):
    """Prop. 1 (eq. 2.9): the packets of (2.7) on the mesh dq = sqrt(eps)/2,
    dp = pi sqrt(eps)/8 sum back to u0 with weight (dq dp)/(2 pi eps)^{3/2}."""
    eps, M = 1 / 64, 1024
    x = -math.pi + 2 * math.pi * np.arange(M) / M
    u0 = (64 / math.pi) ** 0.25 * np.exp(-32 * x * x + 1j * x / eps)
    dq, dp = math.sqrt(eps) / 2, math.pi * math.sqrt(eps) / 8
    qs = np.arange(-1.0, 1.0 + 1e-12, dq)
    ps_ = 1.0 + np.arange(-1.0, 1.0 + 1e-12, dp)
    qq, pp = [g.ravel()[None, :] for g in np.meshgrid(qs, ps_, indexing="ij")]
    A = flow.decompose(u0, eps, [M], 8 * math.sqrt(eps), qq, pp)
    scale = dq * dp / (2 * math.pi * eps) ** 1.5
    u = orc.direct_sum(qq, pp, np.zeros(qq.shape[1]), A, eps, [M], 6 * math.sqrt(eps), scale)
    assert rel(u, u0) < 1e-7


# --------------------------------------------------------------------------
# the whole FGA chain (2.7) -> (2.3)-(2.6) -> (2.10) against a spectral reference
# --------------------------------------------------------------------------

def split_step(u0, Vx, eps, T, nsteps):
    """Strang splitting of i eps u_t = -eps^2/2 u_xx + V u on the periodic grid
    (a reference written for these tests; second order in dt, spectral in x)."""
    M = u0.size
    k = np.fft.fftfreq(M, d=1.0 / M)
    dt = T / nsteps
    half = np.exp(-1j * Vx * dt / (2 * eps))
    kin = np.exp(-1j * eps * k * k * dt / 2)
    u = u0.copy()
    for _ in range(nsteps):
        u = half * np.fft.ifft(kin * np.fft.fft(half * u))
    return u


def fga_chain(orc, eps, M, V, T, n):
    """Example 1's initial wave, decomposed on dq = sqrt(eps)/2, dp = pi sqrt(eps)/8,
    carried by RK4 and summed by the direct sum (R = 6 sqrt(eps))."""
    x = -math.pi + 2 * math.pi * np.arange(M) / M
    u0 = (64 / math.pi) ** 0.25 * np.exp(-32 * x * x + 1j * x / eps)
    dq, dp = math.sqrt(eps) / 2, math.pi * math.sqrt(eps) / 8
    qs = np.arange(-0.8, 0.8 + 1e-12, dq)
    ps_ = 1.0 + np.arange(-1.2, 1.2 + 1e-12, dp)
    qq, pp = [g.ravel()[None, :] for g in np.meshgrid(qs, ps_, indexing="ij")]
    A = flow.decompose(u0, eps, [M], 8 * math.sqrt(eps), qq, pp)
    Q, P, S, At, _, _ = flow.propagate(qq, pp, np.zeros(qq.shape[1]), A, V, T / n, n)
    scale = dq * dp / (2 * math.pi * eps) ** 1.5
    return x, u0, orc.direct_sum(Q, P, S, At, eps, [M], 6 * math.sqrt(eps), scale)


def test_fga_chain_exact_for_harmonic_potential(orc):
    """For a quadratic potential the FGA is exact: the chain meets the spectral
    solution to the reference's own time-step error."""
    eps, M, T = 1 / 64, 2048, 0.5
    x, u0, u = fga_chain(orc, eps, M, flow.potential(w=(1.0,)), T, 500)
    ref = split_step(u0, 0.5 * x * x, eps, T, 4000)
    assert rel(u, ref) < 5e-7


def test_fga_chain_first_order_in_eps(orc):
    """Example 1's potential 1 - cos(pi x): the FGA error is first order in eps
    (a factor ~4 per factor 4 in eps), far above the discretisation errors."""
    V = flow.potential(c0=1.0, c1=-1.0, kappa=math.pi)
    errs = []
    for eps, M in ((1 / 64, 2048), (1 / 256, 4096)):
        x, u0, u = fga_chain(orc, eps, M, V, 0.5, 500)
        errs.append(rel(u, split_step(u0, 1 - np.cos(math.pi * x), eps, 0.5, 4000)))
    assert 3e-3 < errs[0] < 3e-2
    assert 2.5 < errs[0] / errs[1] < 6


# --------------------------------------------------------------------------
# multi-step FGGC (Alg. 3)
# --------------------------------------------------------------------------

def multistep_setup():
    eps, M, Nq = 1 / 64, 512, 128
    x = -math.pi + 2 * math.pi * np.arange(M) / M
    u0 = (64 / math.pi) ** 0.25 * np.exp(-32 * x * x + 1j * x / eps)
    dq, dp = 2 * math.pi / Nq, math.pi * math.sqrt(eps) / 8
    qs = -math.pi + dq * np.arange(Nq)
    qs = qs[(qs > -1.0) & (qs < 1.8)]
    ps_ = dp * np.arange(int(np.floor(-0.3 / dp)), int(np.ceil(2.3 / dp)) + 1)
    qm, pm = [g.ravel()[None, :] for g in np.meshgrid(qs, ps_, indexing="ij")]
    return eps, M, Nq, dp, x, u0, qm, pm


def test_multistep_exact_for_harmonic_and_learns(orc):
    """Alg. 3 on the harmonic potential: every run's FGA is exact, so the
    composed result meets the spectral solution whatever the number of runs;
    later runs evolve only the mesh points not learned before."""
    eps, M, Nq, dp, x, u0, qm, pm = multistep_setup()
    ref = split_step(u0, 0.5 * x * x, eps, 0.5, 4000)
    for runs in (2, 4):
        u, ev = flow.multistep(orc, u0, eps, [M], qm, pm, flow.potential(w=(1.0,)), 1e-3, 500 // runs, runs,
                               [Nq], [dp], [-1, 0, 1, 2], [0, 1], 8 * math.sqrt(eps))
        assert rel(u, ref) < 2e-7
        assert all(e < 0.3 * ev[0] for e in ev[1:])


def test_multistep_error_accumulates_mildly(orc):
    """Example 1's potential: restarting the FGA at T/2 keeps the error of the
    same order (the paper reports growth by a small factor)."""
    eps, M, Nq, dp, x, u0, qm, pm = multistep_setup()
    V = flow.potential(c0=1.0, c1=-1.0, kappa=math.pi)
    ref = split_step(u0, 1 - np.cos(math.pi * x), eps, 0.5, 4000)
    errs = []
    for runs in (1, 2):
        u, _ = flow.multistep(orc, u0, eps, [M], qm, pm, V, 1e-3, 500 // runs, runs, [Nq], [dp],
                              [-1, 0, 1, 2], [0, 1], 8 * math.sqrt(eps))
        errs.append(rel(u, ref))
    assert 3e-3 < errs[0] < errs[1] < 3 * errs[0]


def test_decomposition_box_window():
    """The box window keeps every point of the ball and the corners beyond it:
    against the closed form both are exact once R is large (8 sqrt(eps)); with
    a small R they differ, the box being closer to the untruncated transform."""
    eps, M = 1 / 16, 256
    x2 = -math.pi + 2 * math.pi * np.arange(M) / M
    u2 = np.outer(np.exp(-8.0 * x2 * x2 + 4j * x2), np.exp(-6.0 * x2 * x2 - 2j * x2))
    rng = np.random.default_rng(6)
    q = rng.uniform(-0.3, 0.3, (2, 10))
    p = rng.uniform(-1, 1, (2, 10))
    exact = 2 * gaussian_transform(8.0, 4.0, eps, q[0], p[0]) * gaussian_transform(6.0, -2.0, eps, q[1], p[1])
    assert rel(flow.decompose(u2, eps, [M, M], 3.0, q, p, window="box"), exact) < 1e-10
    eb = rel(flow.decompose(u2, eps, [M, M], 0.4, q, p, window="box"), exact)
    ec = rel(flow.decompose(u2, eps, [M, M], 0.4, q, p), exact)
    assert 0 < eb < ec
