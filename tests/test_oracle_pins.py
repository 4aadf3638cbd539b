"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these tests retypes the oracle's formulas: each compares it with an
independent computation (quadrature, sampled least squares, a closed-form
solution, a brute-force sum, values printed in the paper) chosen so that a
dropped term, a wrong sign or a wrong conjugation fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
Q2 = [0, 1]
Q4 = [-1, 0, 1, 2]


def tensor1d(qs, ps):
    """1D tensor strategy: basis index a*len(ps) + b <-> (qs[a], ps[b])."""
    return [a for a in qs for b in ps], [b for a in qs for b in ps]


def packet(x, Q, P, eps):
    """G(x; Q, P) of eq. (2.16) on the real line (1D)."""
    return np.exp(1j * P * (x - Q) / eps - (x - Q) ** 2 / (2 * eps))


# --------------------------------------------------------------------------
# eq. (2.17): closed-form inner product against quadrature
# --------------------------------------------------------------------------

def test_inner_product_matches_quadrature(orc):
    rng = np.random.default_rng(17)
    eps = 1.0 / 64
    x = np.linspace(-6.0, 6.0, 240001)
    h = x[1] - x[0]
    for _ in range(6):
        Qa, Qb = rng.uniform(-0.4, 0.4, 2)
        Pa, Pb = rng.uniform(-1.0, 1.5, 2)
        num = np.sum(packet(x, Qa, Pa, eps) * np.conj(packet(x, Qb, Pb, eps))) * h
        assert abs(orc.inner(Qa, Pa, Qb, Pb, eps) - num) < 1e-12
    # d = 2: the integral factorises over dimensions
    Qa, Pa, Qb, Pb = rng.uniform(-0.4, 0.4, (4, 2))
    num = 1.0
    for k in range(2):
        num *= np.sum(packet(x, Qa[k], Pa[k], eps) * np.conj(packet(x, Qb[k], Pb[k], eps))) * h
    assert abs(orc.inner(Qa, Pa, Qb, Pb, eps) - num) < 1e-12


def test_gram_and_rhs_are_normalised_inner_products(orc):
    """eq. (3.22)-(3.23) equal eq. (2.17) / (pi eps)^{d/2} at any eps (Theorem 3's scaling)."""
    dq, dp = tensor1d(Q4, Q2)
    Cq, Cp = 0.5, math.pi / 8
    s, t = 0.31, 0.77
    A = orc.gram(dq, dp, Cq, Cp)
    f = orc.rhs(dq, dp, Cq, Cp, s, t)
    for eps in (1.0 / 64, 1.0 / 4096):
        Dq, Dp = Cq * math.sqrt(eps), Cp * math.sqrt(eps)
        for j in range(len(dq)):
            fj = orc.inner(dq[j] * Dq, dp[j] * Dp, s * Dq, t * Dp, eps) / math.sqrt(math.pi * eps)
            assert abs(fj - f[j]) < 1e-13
            for k in range(len(dq)):
                ajk = orc.inner(dq[j] * Dq, dp[j] * Dp, dq[k] * Dq, dp[k] * Dp, eps) / math.sqrt(math.pi * eps)
                assert abs(ajk - A[j, k]) < 1e-13
    assert np.allclose(A, A.conj().T, atol=1e-15)


# --------------------------------------------------------------------------
# Section 3.1 tables: M_LSA printed in the paper
# --------------------------------------------------------------------------

with open(os.path.join(HERE, "golden", "mlsa_tables.json")) as fh:
    MLSA = json.load(fh)

# Readings: the tables captioned "Q4P2" and "Q2P4" are reproduced by the
# shift sets with the q and p roles exchanged, and the paper's pseudo-inverse
# drops eigenvalues below 1e-10 of the largest.  One Q4P4 entry
# (dq = sqrt(eps), dp = pi sqrt(eps)/4, printed 1.385e-05) is not reproduced by
# any reading tried; every other entry is, within 2%.
TABLE_CASES = [
    ("Q2P2", (Q2, Q2), 0.0, set()),
    ("Q2P2", (Q2, Q2), 1e-10, set()),
    ("Q4P2", (Q2, Q4), 1e-10, set()),
    ("Q2P4", (Q4, Q2), 1e-10, set()),
    ("Q4P4", (Q4, Q4), 1e-10, {(1, 1)}),
]


@pytest.mark.parametrize("name,layout,rcond,unmatched", TABLE_CASES)
def test_mlsa_tables(orc, name, layout, rcond, unmatched):
    dq, dp = tensor1d(*layout)
    tab = MLSA["tables"][name]
    for i, cp in enumerate(MLSA["rows_dp_over_pi_sqrt_eps"]):
        for j, cq in enumerate(MLSA["columns_dq_over_sqrt_eps"]):
            sup, _, _ = orc.mlsa(dq, dp, cq, cp * math.pi, rcond=rcond, ns=21, nt=21)
            ratio = sup / tab[i][j]
            if (i, j) in unmatched:
                assert not (0.98 < ratio < 1.02)
            else:
                assert 0.98 < ratio < 1.02, (name, i, j, sup, tab[i][j])


def test_mlsa_recommended_strategy_values(orc):
    """Remark after the tables: at dq = sqrt(eps)/2, dp = pi sqrt(eps)/8, Q2P2 gives 6.859e-4."""
    dq, dp = tensor1d(Q2, Q2)
    sup, s_at, t_at = orc.mlsa(dq, dp, 0.5, math.pi / 8, ns=41, nt=41)
    assert abs(sup / 6.859e-4 - 1) < 2e-3
    # exact least squares of the build's default Q4P2 (dq {-1..2} x dp {0,1}) at C = pi/8
    dq, dp = tensor1d(Q4, Q2)
    sup, _, _ = orc.mlsa(dq, dp, math.pi / 8, math.pi / 8, ns=21, nt=21)
    assert 1e-7 < sup < 1e-6


with open(os.path.join(HERE, "golden", "mlsa1_table.json")) as fh:
    MLSA1 = json.load(fh)

# Reading: in the H^1 table the column "Q4P2" is the q-shift set of four
# (dq {-1, 0, 1, 2} x dp {0, 1}) and "Q2P4" the p-set of four -- the natural
# reading, unlike the L^2 tables above; the pseudo-inverse drops eigenvalues
# below 1e-10 of the largest, as there.
H1_LAYOUTS = {"Q2P2": (Q2, Q2), "Q4P2": (Q4, Q2), "Q2P4": (Q2, Q4), "Q4P4": (Q4, Q4)}


@pytest.mark.parametrize("name", ["Q2P2", "Q4P2", "Q2P4", "Q4P4"])
def test_mlsa_h1_reproduces_the_printed_table(orc, name):
    """The H^1 quantity (Sec. 3.1 remark, the sup after eq. 3.28) against every
    printed value of its column, eps = 2^-6 ... 2^-16 (4 printed digits)."""
    j = MLSA1["columns"].index(name)
    dq, dp = H1_LAYOUTS[name]
    for i, eps in enumerate(MLSA1["eps"]):
        sup, _, _ = orc.mlsa_h1(dq, dp, eps, 0.5, math.pi / 8, rcond=1e-10, ns=21, nt=21)
        want = MLSA1["values"][i][j]
        assert abs(sup / want - 1) < 1.5e-3, (name, eps, sup, want)


def test_mlsa_h1_vanishes_on_the_mesh_and_needs_the_cutoff_reading(orc):
    """A packet on a mesh point is its own basis function: with exact least
    squares its H^1 residual vanishes (to the conditioning of the Gram matrix;
    Q4P4's is singular at this mesh and is left out).  With the 1e-10 cutoff
    the larger shift sets lose a direction that the on-mesh packet itself
    needs, so their residual there is already the printed sup: the cutoff is
    part of the reading, as for the L^2 tables."""
    for name, bound in (("Q2P2", 1e-11), ("Q4P2", 1e-8), ("Q2P4", 1e-8)):
        dq, dp = H1_LAYOUTS[name]
        sup, _, _ = orc.mlsa_h1(dq, dp, 1 / 64, 0.5, math.pi / 8, rcond=0.0, ns=1, nt=1)
        assert sup < bound, (name, sup)
    for j, name in enumerate(MLSA1["columns"][1:], start=1):
        dq, dp = H1_LAYOUTS[name]
        sup, _, _ = orc.mlsa_h1(dq, dp, 1 / 64, 0.5, math.pi / 8, rcond=1e-10, ns=1, nt=1)
        assert abs(sup / MLSA1["values"][0][j] - 1) < 1.5e-3, (name, sup)


# --------------------------------------------------------------------------
# least squares: the oracle's coefficients are the L2-best ones
# --------------------------------------------------------------------------

@pytest.mark.parametrize("layout", [(Q2, Q2), (Q4, Q2), (Q2, Q4)])
def test_lsa_residual_orthogonal_and_E_by_quadrature(orc, layout):
    """E_LSA (eq. 3.4) by quadrature, and the normal-equation property <r, psi_j> = 0.

    The orthogonality of the residual is what fixes the conjugation: the
    coefficients of the printed system (the conjugates) fail it.
    """
    dq, dp = tensor1d(*layout)
    Cq, Cp = math.pi / 8, math.pi / 8
    x = np.linspace(-14.0, 14.0, 56001)
    h = x[1] - x[0]
    rng = np.random.default_rng(3)
    for s, t in [(0.5, 0.0), tuple(rng.uniform(0, 1, 2)), tuple(rng.uniform(0, 1, 2))]:
        c, E = orc.lsa(dq, dp, Cq, Cp, s, t)
        phi = packet(x, Cq * s, Cp * t, 1.0)
        psi = np.stack([packet(x, Cq * a, Cp * b, 1.0) for a, b in zip(dq, dp)])
        r = phi - c @ psi
        norm_phi = math.sqrt(np.sum(abs(phi) ** 2) * h)
        E_quad = math.sqrt(np.sum(abs(r) ** 2) * h) / norm_phi
        assert abs(E_quad - E) <= 1e-9 + 1e-6 * E
        proj = (psi.conj() @ r) * h / norm_phi
        assert np.max(abs(proj)) < 1e-10
        # sampled-basis least squares (an independent solver) agrees
        c_ls = np.linalg.lstsq(psi.T, phi, rcond=None)[0]
        assert np.max(abs(c_ls - c)) < 1e-6 * max(1.0, np.max(abs(c)))
        if t > 0.05:
            r_bad = phi - c.conj() @ psi
            assert np.max(abs(psi.conj() @ r_bad) * h / norm_phi) > 1e-3


def test_lsa_exact_on_grid_point(orc):
    """A packet on a mesh point (s = t = 0) is reproduced exactly by its own neighbour."""
    dq, dp = tensor1d(Q4, Q2)
    c, E = orc.lsa(dq, dp, math.pi / 8, math.pi / 8, 0.0, 0.0)
    e = np.zeros(len(dq), complex)
    k0 = [i for i, (a, b) in enumerate(zip(dq, dp)) if a == 0 and b == 0][0]
    e[k0] = 1
    assert np.max(abs(c - e)) < 1e-9
    assert E < 1e-9


def test_kronecker_factorisation_2d(orc):
    """For a tensor strategy the 2D least squares is the product of 1D ones (checked with Q2P2)."""
    q1, p1 = tensor1d(Q2, Q2)
    n1 = len(q1)
    dq2 = [[q1[a], q1[b]] for a in range(n1) for b in range(n1)]
    dp2 = [[p1[a], p1[b]] for a in range(n1) for b in range(n1)]
    Cq, Cp = [0.5, 0.39], [math.pi / 8, 0.45]
    s, t = [0.23, 0.81], [0.64, 0.12]
    c2, E2 = orc.lsa(dq2, dp2, Cq, Cp, s, t)
    c0, E0 = orc.lsa(q1, p1, Cq[0], Cp[0], s[0], t[0])
    c1, E1 = orc.lsa(q1, p1, Cq[1], Cp[1], s[1], t[1])
    assert np.max(abs(c2 - np.kron(c0, c1))) < 1e-11
    assert abs((1 - E2 ** 2) - (1 - E0 ** 2) * (1 - E1 ** 2)) < 1e-13


# --------------------------------------------------------------------------
# Theorems 2 and 3 through the cell array (physical units)
# --------------------------------------------------------------------------

def single_packet_cells(orc, Q, P, eps, Nq, dp, layout, rcond=0.0):
    cells, slo, sn = orc.fggc_cells(np.array([[Q]]), np.array([[P]]), np.array([0.0]),
                                    np.array([1.0 + 0j]), eps, [Nq], [dp], layout[0], layout[1],
                                    rcond=rcond)
    out = {}
    for l, i in zip(*np.nonzero(cells)):
        q = -math.pi + i * 2 * math.pi / Nq
        p = (slo[0] + l) * dp
        out[(round(q / (2 * math.pi / Nq)), int(slo[0] + l))] = (q, p, cells[l, i])
    return out


@pytest.mark.parametrize("layout", [(Q2, Q2), (Q4, Q2)])
def test_shift_of_coefficients_matches_direct_least_squares(orc, layout):
    """Theorem 2 / eq. (3.13) with the sign that goes with the conjugation.

    A packet far from the origin of phase space (ip ~ 25) is fitted directly,
    by least squares on sampled basis functions in physical units; the cell
    values the oracle scatters must be these coefficients.
    """
    eps = 1.0 / 64
    Nq = 128
    dq_m = 2 * math.pi / Nq
    dp_m = math.pi * math.sqrt(eps) / 8
    for Q, P in [(0.3712, 1.2345), (-0.61, -0.93)]:
        cells = single_packet_cells(orc, Q, P, eps, Nq, dp_m, layout)
        x = np.linspace(Q - 2.0, Q + 2.0, 40001)
        keys = sorted(cells)
        psi = np.stack([packet(x, cells[k][0], cells[k][1], eps) for k in keys])
        # the q index wraps at +-pi; these packets stay clear of it
        c_ls = np.linalg.lstsq(psi.T, packet(x, Q, P, eps), rcond=None)[0]
        c_or = np.array([cells[k][2] for k in keys])
        assert len(keys) == len(layout[0]) * len(layout[1])
        assert np.max(abs(c_ls - c_or)) < 1e-6


def test_lsa_error_independent_of_eps(orc):
    """Theorem 3: at fixed (s, t) and fixed C_q, C_p the fit error is the same for every eps."""
    dq, dp = tensor1d(Q4, Q2)
    Cq = Cp = math.pi / 8
    s, t = 0.37, 0.58
    _, E_ref = orc.lsa(dq, dp, Cq, Cp, s, t)
    for eps in (2.0 ** -6, 2.0 ** -10, 2.0 ** -14):
        Dq, Dp = Cq * math.sqrt(eps), Cp * math.sqrt(eps)
        iq, ip = 7, 40
        Q, P = (iq + s) * Dq, (ip + t) * Dp
        x = np.linspace(Q - 14 * math.sqrt(eps), Q + 14 * math.sqrt(eps), 60001)
        h = x[1] - x[0]
        psi = np.stack([packet(x, (iq + a) * Dq, (ip + b) * Dp, eps) for a, b in zip(dq, dp)])
        phi = packet(x, Q, P, eps)
        c_ls = np.linalg.lstsq(psi.T, phi, rcond=None)[0]
        E = math.sqrt(np.sum(abs(phi - c_ls @ psi) ** 2) / np.sum(abs(phi) ** 2))
        assert abs(E - E_ref) < 2e-3 * E_ref


# --------------------------------------------------------------------------
# direct sum: brute force and truncation bound
# --------------------------------------------------------------------------

def random_set(rng, d, N, pmean=0.5):
    Q = rng.uniform(-math.pi, math.pi, (d, N))
    P = pmean + 0.3 * rng.standard_normal((d, N))
    S = rng.uniform(0, 2 * math.pi, N)
    a = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return Q, P, S, a


@pytest.mark.parametrize("d,M", [(1, 96), (2, 24), (3, 12)])
def test_direct_sum_against_bruteforce(orc, d, M):
    rng = np.random.default_rng(5 + d)
    eps = 1.0 / 16
    Q, P, S, a = random_set(rng, d, 13)
    Mv = [M] * d
    ub = orc.direct_bruteforce(Q, P, S, a, eps, Mv, nimg=2, scale=0.7)
    # a window just under pi leaves only the far images out: exp(-pi^2 / (2 eps)) ~ 1e-34
    uw = orc.direct_sum(Q, P, S, a, eps, Mv, math.pi * (1 - 1e-9), scale=0.7)
    assert np.linalg.norm(uw - ub) <= 1e-13 * np.linalg.norm(ub)
    # R = 6 sqrt(eps): the cut tail of one Gaussian has relative L2 mass erfc-like ~ e^{-18}
    u6 = orc.direct_sum(Q, P, S, a, eps, Mv, 6 * math.sqrt(eps), scale=0.7)
    rel = np.linalg.norm(u6 - ub) / np.linalg.norm(ub)
    assert rel < {1: 1e-8, 2: 4e-8, 3: 1.5e-7}[d]
    # sampled points agree with the full evaluation bit for bit
    pts = rng.choice(M ** d, 7, replace=False)
    assert np.array_equal(orc.direct_sum(Q, P, S, a, eps, Mv, 6 * math.sqrt(eps), 0.7, pts=pts), u6[pts])


def test_direct_sum_box_window_against_definition(orc):
    """The box-window sum (every |y_k| <= R) against its definition, written out
    as plain loops over packets and points on a tiny 2D grid.  eps and R are
    large enough that the corners of the box (outside the ball of radius R)
    carry weight, so the window's shape is seen."""
    rng = np.random.default_rng(41)
    eps, R, M = 0.5, 1.3, (8, 6)
    Q, P, S, a = random_set(rng, 2, 7)
    ref = np.zeros(M, dtype=complex)
    for m0 in range(M[0]):
        for m1 in range(M[1]):
            x = (-math.pi + 2 * math.pi * m0 / M[0], -math.pi + 2 * math.pi * m1 / M[1])
            for j in range(Q.shape[1]):
                y = [(x[k] - Q[k, j] + math.pi) % (2 * math.pi) - math.pi for k in range(2)]
                if max(abs(y[0]), abs(y[1])) > R:
                    continue
                ph = (S[j] + P[0, j] * y[0] + P[1, j] * y[1]) / eps
                ref[m0, m1] += 0.9 * a[j] * np.exp(1j * ph - (y[0] ** 2 + y[1] ** 2) / (2 * eps))
    ub = orc.direct_sum(Q, P, S, a, eps, M, R, scale=0.9, window="box")
    assert np.linalg.norm(ub - ref.ravel()) <= 1e-13 * np.linalg.norm(ref)
    # the ball drops the corners: a visible difference here
    uc = orc.direct_sum(Q, P, S, a, eps, M, R, scale=0.9)
    assert np.linalg.norm(uc - ub) > 1e-3 * np.linalg.norm(ub)
    # in one dimension the box is the ball
    Q1, P1, S1, a1 = random_set(rng, 1, 9)
    assert np.array_equal(orc.direct_sum(Q1, P1, S1, a1, 1 / 16, [64], 0.9, window="box"),
                          orc.direct_sum(Q1, P1, S1, a1, 1 / 16, [64], 0.9))


def test_direct_sum_single_packet_on_grid_is_symmetric(orc):
    eps, M = 1.0 / 64, 256
    m0 = 100
    Q = np.array([[-math.pi + m0 * 2 * math.pi / M]])
    u = orc.direct_sum(Q, np.zeros((1, 1)), np.zeros(1), np.ones(1, complex), eps, [M], 0.75)
    k = np.arange(1, 20)
    assert np.allclose(u[m0 + k], u[m0 - k], rtol=0, atol=1e-13)
    assert abs(u[m0] - 1.0) < 1e-15


# --------------------------------------------------------------------------
# closed-form free-particle evolution (eq. 2.3-2.7, 2.10 with V = 0)
# --------------------------------------------------------------------------

def free_particle_packets(eps, t, q_half, p_half, nquad=8192):
    """FGA packets of u0 = (64/pi)^(1/4) exp(-32 x^2 + i x / eps) after free flow for time t.

    A(0, q, p) = 2^(1/2) u0^(q, p) by quadrature of eq. (2.7); with V = 0 the
    flow (2.3)-(2.6) gives Q = q + t p, P = p, S = t p^2 / 2 and
    Z = 2 - i t, so A(t) = A(0) (1 - i t / 2)^(1/2).
    """
    dq = math.sqrt(eps) / 2
    dp = math.pi * math.sqrt(eps) / 8
    q = np.arange(-q_half, q_half + 1e-12, dq)
    p = 1.0 + np.arange(-p_half, p_half + 1e-12, dp)
    qq, pp = [g.ravel() for g in np.meshgrid(q, p, indexing="ij")]
    y = -math.pi + 2 * math.pi * np.arange(nquad) / nquad
    u0 = (64 / math.pi) ** 0.25 * np.exp(-32 * y ** 2 + 1j * y / eps)
    yy = y[None, :] - qq[:, None]
    A0 = math.sqrt(2) * (np.exp(-1j * pp[:, None] * yy / eps - yy ** 2 / (2 * eps)) @ u0) * (2 * math.pi / nquad)
    Q = (qq + t * pp)[None, :]
    P = pp[None, :].copy()
    S = t * pp ** 2 / 2
    A = A0 * np.sqrt(1 - 0.5j * t)
    scale = dq * dp / (2 * math.pi * eps) ** 1.5
    return Q, P, S, A, scale, dp


def test_free_particle_closed_form(orc):
    eps, t, M = 1.0 / 64, 0.5, 1024
    x = -math.pi + 2 * math.pi * np.arange(M) / M
    k = np.fft.fftfreq(M, d=1.0 / M)
    u0 = (64 / math.pi) ** 0.25 * np.exp(-32 * x ** 2 + 1j * x / eps)
    u_exact = np.fft.ifft(np.fft.fft(u0) * np.exp(-1j * eps * k ** 2 * t / 2))
    Q, P, S, A, scale, dp = free_particle_packets(eps, t, 1.0, 1.0)
    u_fga = orc.direct_sum(Q, P, S, A, eps, [M], 6 * math.sqrt(eps), scale)
    err = np.linalg.norm(u_fga - u_exact) / np.linalg.norm(u_exact)
    assert err < 1e-8
    # FGGC with the recommended mesh (C_q = C_p = pi/8): error at the LSA level
    u_q4p2 = orc.fggc(Q, P, S, A * scale, eps, [M], [128], [dp], Q4, Q2)
    assert np.linalg.norm(u_q4p2 - u_exact) / np.linalg.norm(u_exact) < 1e-8
    u_q2p2 = orc.fggc(Q, P, S, A * scale, eps, [M], [128], [dp], Q2, Q2)
    e22 = np.linalg.norm(u_q2p2 - u_fga) / np.linalg.norm(u_fga)
    assert 1e-7 < e22 < 7e-4


def test_free_particle_closed_form_2d(orc):
    """The d-dimensional constants: (dq dp)^d / (2 pi eps)^{3d/2} and A(t) ~ (1 - i t/2)^{d/2}."""
    eps, t, M = 1.0 / 16, 0.5, 128
    Q1, P1, S1, A1, scale1, _ = free_particle_packets(eps, t, 1.5, 2.5, nquad=4096)
    n = A1.size
    ia, ib = [g.ravel() for g in np.meshgrid(np.arange(n), np.arange(n), indexing="ij")]
    Q = np.stack([Q1[0, ia], Q1[0, ib]])
    P = np.stack([P1[0, ia], P1[0, ib]])
    S = S1[ia] + S1[ib]
    A = A1[ia] * A1[ib]  # 2^(d/2) u0^ and (1 - i t/2)^(d/2) factor over dimensions
    x = -math.pi + 2 * math.pi * np.arange(M) / M
    k = np.fft.fftfreq(M, d=1.0 / M)
    u0 = (64 / math.pi) ** 0.25 * np.exp(-32 * x ** 2 + 1j * x / eps)
    u1 = np.fft.ifft(np.fft.fft(u0) * np.exp(-1j * eps * k ** 2 * t / 2))
    u_exact = np.outer(u1, u1).ravel()
    rng = np.random.default_rng(2)
    big = np.flatnonzero(abs(u_exact) > 0.1 * abs(u_exact).max())
    pts = np.concatenate([rng.choice(big, 40, replace=False), rng.choice(M * M, 24, replace=False)])
    u_fga = orc.direct_sum(Q, P, S, A, eps, [M, M], 6 * math.sqrt(eps), scale1 ** 2, pts=pts)
    assert np.max(abs(u_fga - u_exact[pts])) < 1e-5 * abs(u_exact).max()


# --------------------------------------------------------------------------
# FGGC against the direct sum on a random-phase set
# --------------------------------------------------------------------------

def test_fggc_error_matches_per_packet_prediction(orc):
    """With random phases the cross terms average out:
    rel-L2^2 ~ sum |alpha_j|^2 E_LSA(s_j, t_j)^2 / sum |alpha_j|^2."""
    rng = np.random.default_rng(11)
    eps, M, Nq = 1.0 / 64, 1024, 128
    N = 3000
    Q = rng.uniform(-math.pi, math.pi, (1, N))
    P = 0.5 + 0.25 * rng.standard_normal((1, N))
    S = rng.uniform(0, 2 * math.pi, N)
    a = np.exp(1j * rng.uniform(0, 2 * math.pi, N))
    dp = math.pi * math.sqrt(eps) / 8
    Cq = (2 * math.pi / Nq) / math.sqrt(eps)
    Cp = dp / math.sqrt(eps)
    u_dir = orc.direct_sum(Q, P, S, a, eps, [M], 8 * math.sqrt(eps))
    dq1, dp1 = tensor1d(Q2, Q2)
    u_fg = orc.fggc(Q, P, S, a, eps, [M], [Nq], [dp], Q2, Q2)
    meas = np.linalg.norm(u_fg - u_dir) / np.linalg.norm(u_dir)
    Es = []
    for j in range(N):
        v, w = Q[0, j] / (2 * math.pi / Nq), P[0, j] / dp
        Es.append(orc.lsa(dq1, dp1, Cq, Cp, v - math.floor(v), w - math.floor(w))[1])
    pred = math.sqrt(np.mean(np.square(Es)))
    assert 0.6 < meas / pred < 1.6


@pytest.mark.parametrize("d,eps,M,Nq", [(2, 1.0 / 64, 128, 128), (3, 1.0 / 16, 32, 32)])
def test_fggc_error_matches_prediction_multidim(orc, d, eps, M, Nq):
    """d >= 2: the cell layout, the Kronecker product and eq. (2.24) over slices.

    Per packet 1 - E_d^2 = prod_k (1 - E_k^2) (tensor strategy), and with random
    phases the FGGC-vs-direct error follows the per-packet prediction.
    """
    rng = np.random.default_rng(21 + d)
    N = 300
    Q = rng.uniform(-math.pi, math.pi, (d, N))
    P = 0.5 + 0.1 * rng.standard_normal((d, N))
    S = rng.uniform(0, 2 * math.pi, N)
    a = np.exp(1j * rng.uniform(0, 2 * math.pi, N))
    dp = math.pi * math.sqrt(eps) / 8
    Cq = (2 * math.pi / Nq) / math.sqrt(eps)
    Cp = dp / math.sqrt(eps)
    pts = rng.choice(M ** d, 48, replace=False)
    u_dir = orc.direct_sum(Q, P, S, a, eps, [M] * d, 8 * math.sqrt(eps), pts=pts)
    u_fg = orc.fggc(Q, P, S, a, eps, [M] * d, [Nq] * d, [dp] * d, Q2, Q2, pts=pts)
    meas = np.linalg.norm(u_fg - u_dir) / np.linalg.norm(u_dir)
    dq1, dp1 = tensor1d(Q2, Q2)
    E2 = []
    for j in range(N):
        keep = 1.0
        for k in range(d):
            v, w = Q[k, j] / (2 * math.pi / Nq), P[k, j] / dp
            keep *= 1 - orc.lsa(dq1, dp1, Cq, Cp, v - math.floor(v), w - math.floor(w))[1] ** 2
        E2.append(1 - keep)
    pred = math.sqrt(np.mean(E2))
    assert 0.4 < meas / pred < 2.5


@pytest.mark.parametrize("d,eps,M,Nq,shifts", [(2, 1.0 / 64, 96, 64, (Q4, Q2)), (3, 1.0 / 16, 24, 32, (Q2, Q2)),
                                              (3, 1.0 / 32, 20, 48, (Q2, Q4))])
def test_fggc_points_equals_dense_cells(orc, d, eps, M, Nq, shifts):
    """The sampled-point form keeps only the cells within Ro of the points; it must
    give the dense cell array's evaluation to rounding, for any batch size (a
    tiny byte budget forces one point per batch), with packets on the periodic
    seam, negative momenta, and points on the seam."""
    rng = np.random.default_rng(40 + d)
    N = 400
    Q = rng.uniform(-math.pi, math.pi, (d, N))
    Q[:, :20] = -math.pi  # on the seam
    P = 0.3 + 0.03 * rng.standard_normal((d, N))
    P[0, 20:40] *= -1.0  # negative momenta
    S = rng.uniform(0, 2 * math.pi, N)
    a = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    dp = math.pi * math.sqrt(eps) / 8
    seam = np.ravel_multi_index(tuple(np.zeros((d, 3), dtype=np.int64) + np.array([0, M - 1, M // 2])),
                                (M,) * d)
    pts = np.unique(np.concatenate([rng.choice(M ** d, 30, replace=False), seam]))
    args = (Q, P, S, a, eps, [M] * d, [Nq] * d, [dp] * d, shifts[0], shifts[1])
    dense = orc.fggc(*args, pts=pts, sparse=False, scale=0.7)
    assert np.max(np.abs(dense)) > 0
    for budget in (4e9, 1.0):
        sp = orc.fggc_points(*args, pts, scale=0.7, max_bytes=budget)
        e = np.linalg.norm(sp - dense) / np.linalg.norm(dense)
        assert e <= 1e-14, (budget, e)
        assert np.max(np.abs(sp - dense)) <= 1e-14 * np.max(np.abs(dense))
