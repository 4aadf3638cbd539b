"""ctypes wrapper around the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, obviously correct
implementation of what the reconstruction path computes; it is imported by
the test suite, by the smoke check and by the CPU-baseline leg of the
benchmark, never by the product package.  See oracle.c for the equations each
function follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, strict IEEE)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.oracle_num_threads.restype = ctypes.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _cplx(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops; returns the previous count."""
    return int(_load().oracle_set_threads(ctypes.c_int(int(n))))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with code {rc}")


def direct_sum(Q, P, S, a, eps, M, R, scale=1.0, pts=None, window="ball"):
    """Windowed direct sum of eq. (2.10) at grid points `pts` (flat indices; None = all).

    window: "ball" (|y| <= R) or "box" (every |y_k| <= R).
    """
    Q = _f64(Q); P = _f64(P); S = _f64(S); a = _cplx(a)
    d, N = Q.shape
    M = _i64(M)
    pts_a = None if pts is None else _i64(pts)
    npts = int(np.prod(M)) if pts_a is None else pts_a.size
    u = np.zeros(npts, dtype=np.complex128)
    if window not in ("ball", "box"):
        raise ValueError(f"unknown window {window!r}")
    fn = _load().oracle_direct_sum if window == "ball" else _load().oracle_direct_sum_boxwin
    rc = fn(ctypes.c_int(d), ctypes.c_int64(N), _p(Q), _p(P), _p(S), _p(a), ctypes.c_double(eps),
            _p(M), ctypes.c_double(R), ctypes.c_double(scale), ctypes.c_int64(npts), _p(pts_a), _p(u))
    _check(rc, "oracle_direct_sum" if window == "ball" else "oracle_direct_sum_boxwin")
    return u


def direct_bruteforce(Q, P, S, a, eps, M, nimg=2, scale=1.0):
    """Untruncated sum over all packets and periodic images (tiny inputs only)."""
    Q = _f64(Q); P = _f64(P); S = _f64(S); a = _cplx(a)
    d, N = Q.shape
    M = _i64(M)
    u = np.zeros(int(np.prod(M)), dtype=np.complex128)
    rc = _load().oracle_direct_bruteforce(ctypes.c_int(d), ctypes.c_int64(N), _p(Q), _p(P), _p(S),
                                          _p(a), ctypes.c_double(eps), _p(M), ctypes.c_int(nimg),
                                          ctypes.c_double(scale), _p(u))
    _check(rc, "oracle_direct_bruteforce")
    return u


def inner(Qa, Pa, Qb, Pb, eps):
    """Closed-form packet inner product, eq. (2.17)."""
    Qa = _f64(np.atleast_1d(Qa)); Pa = _f64(np.atleast_1d(Pa))
    Qb = _f64(np.atleast_1d(Qb)); Pb = _f64(np.atleast_1d(Pb))
    out = np.zeros(1, dtype=np.complex128)
    rc = _load().oracle_inner(ctypes.c_int(Qa.size), _p(Qa), _p(Pa), _p(Qb), _p(Pb),
                              ctypes.c_double(eps), _p(out))
    _check(rc, "oracle_inner")
    return out[0]


def _shifts(dq, dp):
    dq = np.ascontiguousarray(np.asarray(dq, dtype=np.int32))
    dp = np.ascontiguousarray(np.asarray(dp, dtype=np.int32))
    if dq.ndim == 1:
        dq = dq[:, None]
        dp = dp[:, None]
    return dq, dp


def gram(dq, dp, Cq, Cp):
    """Gram matrix A~ of eq. (3.22); dq, dp are [n] or [n][d] integer shifts."""
    dq, dp = _shifts(dq, dp)
    n, d = dq.shape
    Cq = _f64(np.broadcast_to(Cq, (d,))); Cp = _f64(np.broadcast_to(Cp, (d,)))
    out = np.zeros((n, n), dtype=np.complex128)
    _check(_load().oracle_gram(ctypes.c_int(d), ctypes.c_int(n), _p(dq), _p(dp), _p(Cq), _p(Cp),
                               _p(out)), "oracle_gram")
    return out


def rhs(dq, dp, Cq, Cp, s, t):
    """Right-hand side f~ of eq. (3.23)."""
    dq, dp = _shifts(dq, dp)
    n, d = dq.shape
    Cq = _f64(np.broadcast_to(Cq, (d,))); Cp = _f64(np.broadcast_to(Cp, (d,)))
    s = _f64(np.broadcast_to(s, (d,))); t = _f64(np.broadcast_to(t, (d,)))
    out = np.zeros(n, dtype=np.complex128)
    _check(_load().oracle_rhs(ctypes.c_int(d), ctypes.c_int(n), _p(dq), _p(dp), _p(Cq), _p(Cp),
                              _p(s), _p(t), _p(out)), "oracle_rhs")
    return out


def lsa(dq, dp, Cq, Cp, s, t, rcond=0.0):
    """L2-best coefficients c~ and E_LSA for the fractional problem (Theorem 2/3 form)."""
    dq, dp = _shifts(dq, dp)
    n, d = dq.shape
    Cq = _f64(np.broadcast_to(Cq, (d,))); Cp = _f64(np.broadcast_to(Cp, (d,)))
    s = _f64(np.broadcast_to(s, (d,))); t = _f64(np.broadcast_to(t, (d,)))
    c = np.zeros(n, dtype=np.complex128)
    E = ctypes.c_double(0.0)
    _check(_load().oracle_lsa(ctypes.c_int(d), ctypes.c_int(n), _p(dq), _p(dp), _p(Cq), _p(Cp),
                              ctypes.c_double(rcond), _p(s), _p(t), _p(c), ctypes.byref(E)),
           "oracle_lsa")
    return c, E.value


def mlsa(dq, dp, Cq, Cp, rcond=0.0, ns=41, nt=41):
    """M_LSA of eq. (3.25) for a 1D strategy, sampled on an ns x nt grid of the unit cell."""
    dq, dp = _shifts(dq, dp)
    n = dq.shape[0]
    sup = ctypes.c_double(0); sa = ctypes.c_double(0); ta = ctypes.c_double(0)
    _check(_load().oracle_mlsa(ctypes.c_int(n), _p(np.ascontiguousarray(dq[:, 0])),
                               _p(np.ascontiguousarray(dp[:, 0])), ctypes.c_double(Cq),
                               ctypes.c_double(Cp), ctypes.c_double(rcond), ctypes.c_int(ns),
                               ctypes.c_int(nt), ctypes.byref(sup), ctypes.byref(sa),
                               ctypes.byref(ta)), "oracle_mlsa")
    return sup.value, sa.value, ta.value


def mlsa_h1(dq, dp, eps, Cq, Cp, rcond=0.0, ns=41, nt=41, nx=2001):
    """The H^1 quantity of the remark in Sec. 3.1 (the sup after eq. 3.28), d = 1:

        sup over (Q, P) in [0, dq_mesh] x [0, dp_mesh] of
            || dG/dx - sum_k c_k dG_k/dx ||_{L^2} / || G ||_{H^1},

    with G(x) = exp(i P (x - Q) / eps - (x - Q)^2 / (2 eps)), the basis
    G_k = G(x; dq_k dq_mesh, dp_k dp_mesh), dq_mesh = Cq sqrt(eps),
    dp_mesh = Cp sqrt(eps), and c the L^2 least-squares coefficients of G on the
    basis (normal equations A c = f, A_jk = <G_k, G_j>, f_j = <G, G_j>, solved
    through the eigenpairs of A with eigenvalues below rcond * max dropped).
    Every integral is a trapezoidal sum over x in [-16 sqrt(eps), 16 sqrt(eps)]
    (nx points; the integrands are Gaussians centred within a few mesh steps of
    0, so the sum converges spectrally), and the derivative of a packet is
    taken analytically: dG/dx = (i P / eps - (x - Q) / eps) G.  The sup is taken
    over an ns x nt grid of the cell, edges included.  Returns (sup, s, t) with
    (s, t) = (Q / dq_mesh, P / dp_mesh) where it is reached."""
    dq = np.asarray(dq, dtype=np.float64).ravel()
    dp = np.asarray(dp, dtype=np.float64).ravel()
    se = math.sqrt(eps)
    Dq, Dp = Cq * se, Cp * se
    x = np.linspace(-16.0 * se, 16.0 * se, nx)
    w = np.full(nx, x[1] - x[0])
    w[0] = w[-1] = 0.5 * (x[1] - x[0])

    def packet(q, p):
        g = np.exp(1j * p * (x - q) / eps - (x - q) ** 2 / (2.0 * eps))
        return g, (1j * p / eps - (x - q) / eps) * g

    basis = [packet(a * Dq, b * Dp) for a in dq for b in dp]
    B = np.stack([g for g, _ in basis], axis=1)
    dB = np.stack([h for _, h in basis], axis=1)
    A = (B.conj().T * w) @ B
    lam, V = np.linalg.eigh(A)
    kept = lam > rcond * lam.max() if rcond > 0 else lam > 0
    best = (-1.0, 0.0, 0.0)
    for s in np.linspace(0.0, 1.0, ns):
        for t in np.linspace(0.0, 1.0, nt):
            g, h = packet(s * Dq, t * Dp)
            f = (B.conj().T * w) @ g
            c = V[:, kept] @ ((V[:, kept].conj().T @ f) / lam[kept])
            r = h - dB @ c
            num = math.sqrt(float(np.sum(w * np.abs(r) ** 2)))
            den = math.sqrt(float(np.sum(w * (np.abs(g) ** 2 + np.abs(h) ** 2))))
            if num / den > best[0]:
                best = (num / den, float(s), float(t))
    return best


def pcell_bounds(P, dp):
    P = _f64(P)
    d, N = P.shape
    dp = _f64(np.broadcast_to(dp, (d,)))
    lo = np.zeros(d, dtype=np.int64); hi = np.zeros(d, dtype=np.int64)
    _check(_load().oracle_pcell_bounds(ctypes.c_int(d), ctypes.c_int64(N), _p(P), _p(dp), _p(lo),
                                       _p(hi)), "oracle_pcell_bounds")
    return lo, hi


def fggc_cells(Q, P, S, a, eps, Nq, dp, dq_off, dp_off, rcond=0.0, scale=1.0):
    """Dense on-grid cells A~ (eq. 2.25) over the occupied p-cell box.

    Returns (cells[prod sn][prod Nq] complex, slo[d], sn[d]).
    """
    Q = _f64(Q); P = _f64(P); S = _f64(S); a = _cplx(a)
    d, N = Q.shape
    Nq = _i64(np.broadcast_to(Nq, (d,))); dp = _f64(np.broadcast_to(dp, (d,)))
    dq_off = np.ascontiguousarray(np.asarray(dq_off, dtype=np.int32))
    dp_off = np.ascontiguousarray(np.asarray(dp_off, dtype=np.int32))
    lo, hi = pcell_bounds(P, dp)
    slo = _i64(lo + dp_off.min())
    sn = _i64(hi + dp_off.max() - slo + 1)
    cells = np.zeros((int(np.prod(sn)), int(np.prod(Nq))), dtype=np.complex128)
    rc = _load().oracle_fggc_cells(ctypes.c_int(d), ctypes.c_int64(N), _p(Q), _p(P), _p(S), _p(a),
                                   ctypes.c_double(eps), _p(Nq), _p(dp), ctypes.c_int(dq_off.size),
                                   _p(dq_off), ctypes.c_int(dp_off.size), _p(dp_off),
                                   ctypes.c_double(rcond), ctypes.c_double(scale), _p(slo), _p(sn),
                                   _p(cells))
    _check(rc, "oracle_fggc_cells")
    return cells, slo, sn


def eval_cells(cells, slo, sn, Nq, dp, eps, M, Ro, pts=None):
    """Evaluate eq. (2.24) directly over the cells at grid points `pts` (None = all)."""
    cells = _cplx(cells)
    d = len(sn)
    slo = _i64(slo); sn = _i64(sn)
    Nq = _i64(np.broadcast_to(Nq, (d,))); dp = _f64(np.broadcast_to(dp, (d,)))
    M = _i64(M)
    pts_a = None if pts is None else _i64(pts)
    npts = int(np.prod(M)) if pts_a is None else pts_a.size
    u = np.zeros(npts, dtype=np.complex128)
    rc = _load().oracle_eval_cells(ctypes.c_int(d), _p(cells), _p(slo), _p(sn), _p(Nq), _p(dp),
                                   ctypes.c_double(eps), _p(M), ctypes.c_double(Ro),
                                   ctypes.c_int64(npts), _p(pts_a), _p(u))
    _check(rc, "oracle_eval_cells")
    return u


def fggc_points(Q, P, S, a, eps, M, Nq, dp, dq_off, dp_off, pts, rcond=0.0, scale=1.0, Ro=None,
                max_bytes=4e9):
    """FGGC at grid points `pts` keeping only the cells within Ro of them (no dense cell array).

    The same scatter (eq. 2.23-2.25) and the same plain evaluation of eq. (2.24)
    as fggc_cells + eval_cells; points are processed in batches whose kept cells
    fit in max_bytes."""
    if Ro is None:
        Ro = 8.0 * np.sqrt(eps)
    Q = _f64(Q); P = _f64(P); S = _f64(S); a = _cplx(a)
    d, N = Q.shape
    Nq = _i64(np.broadcast_to(Nq, (d,))); dp = _f64(np.broadcast_to(dp, (d,)))
    dq_off = np.ascontiguousarray(np.asarray(dq_off, dtype=np.int32))
    dp_off = np.ascontiguousarray(np.asarray(dp_off, dtype=np.int32))
    M = _i64(M)
    pts_a = _i64(pts)
    u = np.zeros(pts_a.size, dtype=np.complex128)
    if pts_a.size == 0:
        return u
    if N == 0:
        return u
    lo, hi = pcell_bounds(P, dp)
    slo = _i64(lo + dp_off.min())
    sn = _i64(hi + dp_off.max() - slo + 1)
    rc = _load().oracle_fggc_points(ctypes.c_int(d), ctypes.c_int64(N), _p(Q), _p(P), _p(S), _p(a),
                                    ctypes.c_double(eps), _p(Nq), _p(dp), ctypes.c_int(dq_off.size),
                                    _p(dq_off), ctypes.c_int(dp_off.size), _p(dp_off),
                                    ctypes.c_double(rcond), ctypes.c_double(scale), _p(slo), _p(sn), _p(M),
                                    ctypes.c_double(Ro), ctypes.c_int64(pts_a.size), _p(pts_a),
                                    ctypes.c_double(max_bytes), _p(u))
    _check(rc, "oracle_fggc_points")
    return u


def fggc(Q, P, S, a, eps, M, Nq, dp, dq_off, dp_off, rcond=0.0, scale=1.0, Ro=None, pts=None,
         sparse=None):
    """Whole FGGC reconstruction: cells (eq. 2.25) then eq. (2.24) over cells, window Ro = 8 sqrt(eps).

    With grid points `pts`, only the cells within Ro of them are kept (fggc_points)
    unless sparse=False, which builds the dense cell array as for the whole grid."""
    if Ro is None:
        Ro = 8.0 * np.sqrt(eps)
    if pts is not None and sparse is not False:
        return fggc_points(Q, P, S, a, eps, M, Nq, dp, dq_off, dp_off, pts, rcond, scale, Ro)
    cells, slo, sn = fggc_cells(Q, P, S, a, eps, Nq, dp, dq_off, dp_off, rcond, scale)
    return eval_cells(cells, slo, sn, Nq, dp, eps, M, Ro, pts)
