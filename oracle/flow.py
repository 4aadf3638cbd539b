"""Plain FP64 oracle for the steps either side of the reconstruction, in numpy:
the initial decomposition (2.7) and the packet flow of eq. (2.3)-(2.6).

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
package.  It shares no code with the HIP path.

The flow of one packet, after Sec. 2.1:
- (2.3) dQ/dt = P;  (2.4) dP/dt = -grad V(Q);  (2.5) dS/dt = |P|^2/2 - V(Q);
- (2.6) dA/dt = (A/2) tr(Z^{-1} dZ/dt), with Z = dz(Q + iP) and dz = d_q - i d_p.

Z needs the derivatives of the flow with respect to its starting point
(q, p).  Differentiating (2.3)-(2.4) along dz gives the variational system
    d(dz Q)/dt = dz P,   d(dz P)/dt = -Hess V(Q) dz Q,
started at dz Q = I, dz P = -i I (so Z(0) = 2 I).  This is a reading: the
paper defines Z through the flow and leaves these equations implicit.

The potential family covers the paper's examples:
    V(x) = c0 + sum_k w_k x_k^2 / 2 + c1 sum_k cos(kappa x_k) + c2 exp(c3 |x|^2).

The time stepping is the classical fourth-order Runge-Kutta scheme (the
paper's choice, Sec. 4), written plainly: four stage derivatives k1..k4 and
y + dt (k1 + 2 k2 + 2 k3 + k4) / 6.
"""
from __future__ import annotations

import numpy as np


def potential(c0=0.0, w=(0.0, 0.0, 0.0), c1=0.0, kappa=0.0, c2=0.0, c3=0.0) -> dict:
    return {"c0": float(c0), "w": tuple(float(x) for x in (list(w) + [0.0, 0.0, 0.0])[:3]),
            "c1": float(c1), "kappa": float(kappa), "c2": float(c2), "c3": float(c3)}


def v_grad_hess(V: dict, Q: np.ndarray):
    """V, grad V and Hess V at Q ([d][N]); returns ([N], [d][N], [d][d][N])."""
    d, N = Q.shape
    w = np.array(V["w"][:d])[:, None]
    r2 = np.sum(Q * Q, axis=0)
    E = V["c2"] * np.exp(V["c3"] * r2)
    kap = V["kappa"]
    val = V["c0"] + 0.5 * np.sum(w * Q * Q, axis=0) + V["c1"] * np.sum(np.cos(kap * Q), axis=0) + E
    grad = w * Q - V["c1"] * kap * np.sin(kap * Q) + 2 * V["c3"] * Q * E[None, :]
    hess = np.zeros((d, d, N))
    for k in range(d):
        hess[k, k] = V["w"][k] - V["c1"] * kap * kap * np.cos(kap * Q[k]) + 2 * V["c3"] * E
        for m in range(d):
            hess[k, m] += 4 * V["c3"] ** 2 * Q[k] * Q[m] * E
    return val, grad, hess


def _rhs(V, Q, P, S, A, JQ, JP):
    """Time derivatives of (Q, P, S, A, JQ, JP); JQ, JP are [d][d][N] complex."""
    val, grad, hess = v_grad_hess(V, Q)
    dQ = P
    dP = -grad
    dS = 0.5 * np.sum(P * P, axis=0) - val
    dJQ = JP
    dJP = -np.einsum("kmn,mln->kln", hess, JQ)
    Z = JQ + 1j * JP
    dZ = dJQ + 1j * dJP
    # tr(Z^{-1} dZ) per packet
    Zt = np.moveaxis(Z, -1, 0)
    dZt = np.moveaxis(dZ, -1, 0)
    tr = np.trace(np.linalg.solve(Zt, dZt), axis1=1, axis2=2)
    dA = 0.5 * A * tr
    return dQ, dP, dS, dA, dJQ, dJP


def propagate(Q, P, S, A, V: dict, dt: float, nsteps: int, JQ=None, JP=None):
    """RK4 for (2.3)-(2.6) from (Q, P, S, A) at t = 0 over nsteps steps of dt.

    Q, P: [d][N]; S: [N]; A: [N] complex.  JQ, JP default to I and -i I.
    Returns (Q, P, S, A, JQ, JP) at t = nsteps dt.
    """
    Q = np.array(Q, dtype=np.float64)
    P = np.array(P, dtype=np.float64)
    S = np.array(S, dtype=np.float64)
    A = np.array(A, dtype=np.complex128)
    d, N = Q.shape
    if JQ is None:
        JQ = np.repeat(np.eye(d, dtype=np.complex128)[:, :, None], N, axis=2)
    if JP is None:
        JP = -1j * np.repeat(np.eye(d, dtype=np.complex128)[:, :, None], N, axis=2)
    y = [Q, P, S, A, np.array(JQ, dtype=np.complex128), np.array(JP, dtype=np.complex128)]
    for _ in range(int(nsteps)):
        k1 = _rhs(V, *y)
        k2 = _rhs(V, *[a + 0.5 * dt * b for a, b in zip(y, k1)])
        k3 = _rhs(V, *[a + 0.5 * dt * b for a, b in zip(y, k2)])
        k4 = _rhs(V, *[a + dt * b for a, b in zip(y, k3)])
        y = [a + dt / 6.0 * (b1 + 2 * b2 + 2 * b3 + b4) for a, b1, b2, b3, b4 in zip(y, k1, k2, k3, k4)]
    return tuple(y)


def decompose(u0, eps, M, R, q, p, window="ball"):
    """A(0, q, p) = 2^{d/2} u0^(q, p) of eq. (2.6)-(2.7) by quadrature on the grid.

    u0^(q, p) = int u0(y) exp(-i p.(y - q)/eps - |y - q|^2/(2 eps)) dy, with u0
    sampled on the periodic grid x_m = -pi + m 2 pi / M (row-major, [prod M]),
    y - q taken as the minimum image and the integrand kept for |y - q| <= R
    (window "ball", that of the direct sum) or for every |y_k - q_k| <= R
    (window "box"); weight prod_k 2 pi / M_k.  q, p: [d][N].
    """
    M = [int(m) for m in np.atleast_1d(M)]
    d = len(M)
    axes = [-np.pi + 2 * np.pi * np.arange(m) / m for m in M]
    X = np.stack([g.ravel() for g in np.meshgrid(*axes, indexing="ij")])  # [d][npts]
    u = np.asarray(u0, dtype=np.complex128).ravel()
    w = np.prod([2 * np.pi / m for m in M])
    q = np.asarray(q, dtype=np.float64).reshape(d, -1)
    p = np.asarray(p, dtype=np.float64).reshape(d, -1)
    out = np.zeros(q.shape[1], dtype=np.complex128)
    for j in range(q.shape[1]):
        y = X - q[:, j:j + 1]
        y = y - 2 * np.pi * np.floor((y + np.pi) / (2 * np.pi))
        r2 = np.sum(y * y, axis=0)
        keep = r2 <= R * R if window == "ball" else np.all(np.abs(y) <= R, axis=0)
        ph = -np.sum(p[:, j:j + 1] * y[:, keep], axis=0) / eps
        out[j] = np.sum(u[keep] * np.exp(1j * ph - r2[keep] / (2 * eps))) * w
    return 2 ** (d / 2) * out


def multistep(orc, u0, eps, M, qm, pm, V: dict, dt: float, steps: int, runs: int, Nq, dp, dq_off, dp_off,
              R_dec: float, prune: float = 1e-12, rcond: float = 0.0):
    """Multi-step FGGC (Alg. 3): `runs` times (Step 1) decompose the current u on
    the fixed mesh (qm, pm) ([d][Nm]), (Step 2) evolve over steps * dt the mesh
    points not learned yet and keep what the flow maps them to, (Step 3)
    reconstruct u by FGGC (eq. 2.23-2.25) with the oracle's plain evaluation.

    The flow is linear in A, so a learned point is stored as its final
    (Q, P, S) and the ratio A(T_evo) / A(0) (the flow of A(0) = 1).  Mesh
    points whose |A(0)| is below prune * max are dropped in that run.
    Returns the final u ([prod M]) and the number of points evolved per run.
    """
    M = [int(m) for m in np.atleast_1d(M)]
    d = len(M)
    qm = np.asarray(qm, dtype=np.float64).reshape(d, -1)
    pm = np.asarray(pm, dtype=np.float64).reshape(d, -1)
    Nm = qm.shape[1]
    learned = np.zeros(Nm, dtype=bool)
    Qf, Pf = np.zeros((d, Nm)), np.zeros((d, Nm))
    Sf, ratio = np.zeros(Nm), np.zeros(Nm, dtype=np.complex128)
    dq = 2 * np.pi / np.asarray(Nq, dtype=np.float64)
    scale = float(np.prod(dq * np.asarray(dp, dtype=np.float64))) / (2 * np.pi * eps) ** (1.5 * d)
    u = np.asarray(u0, dtype=np.complex128).ravel()
    evolved = []
    for _ in range(int(runs)):
        A0 = decompose(u, eps, M, R_dec, qm, pm)
        keep = np.abs(A0) > prune * np.abs(A0).max()
        new = np.flatnonzero(keep & ~learned)
        if new.size:
            Q, P, S, A, _, _ = propagate(qm[:, new], pm[:, new], np.zeros(new.size),
                                         np.ones(new.size, dtype=np.complex128), V, dt, steps)
            Qf[:, new], Pf[:, new], Sf[new], ratio[new] = Q, P, S, A
            learned[new] = True
        evolved.append(int(new.size))
        k = np.flatnonzero(keep)
        u = orc.fggc(Qf[:, k], Pf[:, k], Sf[k], A0[k] * ratio[k], eps, M, Nq, dp, dq_off, dp_off,
                     rcond=rcond, scale=scale)
    return u, evolved
