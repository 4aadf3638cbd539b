"""Seeded synthetic packet sets.

This module holds no reconstruction arithmetic: it only draws the inputs
(Q, P, S, a) that both the GPU library and the CPU oracle are fed.  Random
numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: output i of the stream seeded with s is mix(s + (i + 1) * gamma).
Uniforms in [0, 1) take the top 53 bits; normals use the Box-Muller transform.

The packet sets mirror the shape of the paper's workloads: packets start on a
(q, p) phase-space mesh (q uniform over the periodic box [-pi, pi)^d), are
carried by free flow Q = q + t p, P = p (eq. 2.3-2.4 with V = 0), carry a
uniform random action S and a Gaussian-in-q amplitude with a uniform random
phase.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
BASE_SEED = 2504217850

_TWO_PI = 2.0 * math.pi


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset+1 .. offset+n of the SplitMix64 sequence started at `seed` (uint64)."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        return z ^ (z >> np.uint64(31))


def substream_seed(seed: int, stream: int) -> int:
    """Seed of an independent sub-stream: output `stream` of the master sequence."""
    return int(splitmix64(seed, 1, offset=stream)[0])


def uniform(seed: int, stream: int, n: int) -> np.ndarray:
    """n uniforms in [0, 1) from sub-stream `stream` of `seed` (53-bit resolution)."""
    z = splitmix64(substream_seed(seed, stream), n)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """n standard normals (Box-Muller, cosine branch) from sub-stream `stream`."""
    u = uniform(seed, stream, 2 * n)
    u1, u2 = u[0::2], u[1::2]
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(_TWO_PI * u2)


def wrap(y: np.ndarray) -> np.ndarray:
    """Map onto the periodic box [-pi, pi)."""
    return y - _TWO_PI * np.floor((y + math.pi) / _TWO_PI)


@dataclasses.dataclass
class PacketSet:
    """A packet set and the grid it is reconstructed on.

    Q, P: [d][N] float64 (structure of arrays); S: [N] float64; a: [N] complex128.
    """
    name: str
    d: int
    eps: float
    M: tuple
    Q: np.ndarray
    P: np.ndarray
    S: np.ndarray
    a: np.ndarray
    R: float

    @property
    def N(self) -> int:
        return int(self.S.shape[0])


def gen_1d(n_q: int, n_p: int, eps: float, M: int, seed: int, t: float = 0.5,
           p_mean: float = 0.5, p_std: float = 0.25, amp: float = 25.0, name: str = "1d") -> PacketSet:
    """1D set: q on an n_q-point mesh of [-pi, pi), n_p packets per q with p = mean + std N(0,1).

    Packet j = i * n_p + r.  Q = wrap(q + t p), P = p, S and theta uniform on
    [0, 2 pi), a = exp(-amp q^2) exp(i theta).
    """
    q = -math.pi + _TWO_PI * np.arange(n_q, dtype=np.float64) / n_q
    qj = np.repeat(q, n_p)
    N = n_q * n_p
    p = p_mean + p_std * normal(seed, 1, N)
    S = _TWO_PI * uniform(seed, 2, N)
    theta = _TWO_PI * uniform(seed, 3, N)
    Q = wrap(qj + t * p)[None, :]
    P = p[None, :].copy()
    a = np.exp(-amp * qj * qj) * np.exp(1j * theta)
    return PacketSet(name, 1, eps, (M,), np.ascontiguousarray(Q), np.ascontiguousarray(P), S, a,
                     6.0 * math.sqrt(eps))


def gen_mesh(d: int, n_q: int, n_p: int, p_width: float, p_center, eps: float, M: int, seed: int,
             t: float = 0.5, amp: float = 10.0, name: str = "nd") -> PacketSet:
    """d-dimensional set: q on an n_q^d mesh of [-pi, pi)^d, p on an n_p^d mesh.

    The p mesh is endpoint-inclusive, p_center +- p_width/2 per dimension.
    Packet order: q index major, p index minor (row-major in each).
    Q = wrap(q + t p), P = p, S and theta uniform, a = exp(-amp |q|^2) e^{i theta}.
    """
    q1 = -math.pi + _TWO_PI * np.arange(n_q, dtype=np.float64) / n_q
    pc = np.broadcast_to(np.asarray(p_center, dtype=np.float64), (d,))
    qg = np.stack([g.ravel() for g in np.meshgrid(*([q1] * d), indexing="ij")])  # [d][n_q^d]
    pg = np.stack([g.ravel() for g in np.meshgrid(
        *[np.linspace(pc[k] - p_width / 2, pc[k] + p_width / 2, n_p) for k in range(d)],
        indexing="ij")])  # [d][n_p^d]
    nqd, npd = qg.shape[1], pg.shape[1]
    N = nqd * npd
    qj = np.repeat(qg, npd, axis=1)
    pj = np.tile(pg, (1, nqd))
    S = _TWO_PI * uniform(seed, 2, N)
    theta = _TWO_PI * uniform(seed, 3, N)
    Q = wrap(qj + t * pj)
    a = np.exp(-amp * np.sum(qj * qj, axis=0)) * np.exp(1j * theta)
    return PacketSet(name, d, eps, (M,) * d, np.ascontiguousarray(Q), np.ascontiguousarray(pj), S,
                     a, 6.0 * math.sqrt(eps))


CONFIG_NAMES = {
    0: "1D direct sum, eps=1/64, N=65536 (256x256 (q,p)), M=1024, complex128",
    1: "1D FGGC vs direct sum, eps=1/1024, N=2^20 (1024x1024 (q,p)), M=16384, complex64",
    2: "2D FGGC vs direct sum, eps=1/256, N=2^22 (64^2 q x 32^2 p), M=1024^2, complex64",
    3: "3D FGGC, eps=1/128, N=2^24 (32^3 q x 8^3 p), M=256^3, complex64",
    4: "serving stream: mixed 1D/2D requests, N log-uniform in 2^12..2^22, eps in {1/64,1/256,1/1024}, "
       "M 2^10..2^14 (1D) or 256^2..1024^2 (2D), FGGC Q4P2, Poisson arrivals",
}


def config(k: int, seed: int | None = None) -> PacketSet:
    """The synthetic packet sets of the four benchmark workloads (seed = 2504217850 + k)."""
    if seed is None:
        seed = BASE_SEED + k
    if k == 0:
        return gen_1d(256, 256, 1.0 / 64, 1024, seed, name="cfg0")
    if k == 1:
        return gen_1d(1024, 1024, 1.0 / 1024, 16384, seed, name="cfg1")
    if k == 2:
        return gen_mesh(2, 64, 32, 0.5, (0.5, 0.3), 1.0 / 256, 1024, seed, name="cfg2")
    if k == 3:
        return gen_mesh(3, 32, 8, 0.5, (0.5, 0.3, 0.3), 1.0 / 128, 256, seed, name="cfg3")
    raise ValueError(f"no workload {k}")


def serving_request(r: int, seed: int | None = None) -> PacketSet:
    """Request r of the serving stream: mixed 1D/2D, N log-uniform in 2^12..2^22.

    d in {1, 2}; eps in {1/64, 1/256, 1/1024}; grid 2^10..2^14 (1D) or
    256^2, 512^2, 1024^2 (2D); q uniform on the box, p uniform in c +- 0.25
    (c = 0.5 in 1D, (0.5, 0.3) in 2D); t = 0.5; S, theta uniform;
    a = exp(-25 q^2) e^{i theta} (1D) or exp(-10 |q|^2) e^{i theta} (2D).
    """
    if seed is None:
        seed = BASE_SEED * 1000 + r
    u = uniform(seed, 10, 4)
    d = 1 if u[0] < 0.5 else 2
    N = int(math.floor(2.0 ** (12 + 10 * u[1])))
    eps = (1.0 / 64, 1.0 / 256, 1.0 / 1024)[min(int(u[2] * 3), 2)]
    if d == 1:
        M = (1024, 2048, 4096, 8192, 16384)[min(int(u[3] * 5), 4)]
        c = np.array([0.5])
        amp = 25.0
    else:
        M = (256, 512, 1024)[min(int(u[3] * 3), 2)]
        c = np.array([0.5, 0.3])
        amp = 10.0
    q = -math.pi + _TWO_PI * uniform(seed, 11, d * N).reshape(d, N)
    p = c[:, None] - 0.25 + 0.5 * uniform(seed, 12, d * N).reshape(d, N)
    S = _TWO_PI * uniform(seed, 13, N)
    theta = _TWO_PI * uniform(seed, 14, N)
    Q = wrap(q + 0.5 * p)
    a = np.exp(-amp * np.sum(q * q, axis=0)) * np.exp(1j * theta)
    return PacketSet(f"req{r}", d, eps, (M,) * d, np.ascontiguousarray(Q), np.ascontiguousarray(p),
                     S, a, 6.0 * math.sqrt(eps))
