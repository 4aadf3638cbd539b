"""The seeded input generator (shared by the oracle and the GPU path)."""
import math

import numpy as np
import pytest

from paper_2504_21785_amd import workloads as w


def test_splitmix64_reference_vector():
    # first outputs of SplitMix64 seeded with 1234567, as published with the
    # generator's reference implementation
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [int(v) for v in w.splitmix64(1234567, 5)] == ref
    # counter-based: any window of the stream is the same sequence
    assert [int(v) for v in w.splitmix64(1234567, 3, offset=2)] == ref[2:5]


def test_uniform_and_normal_moments():
    u = w.uniform(7, 1, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 3e-3
    z = w.normal(7, 2, 200000)
    assert abs(z.mean()) < 1e-2 and abs(z.std() - 1) < 1e-2
    assert not np.array_equal(w.uniform(7, 1, 10), w.uniform(7, 2, 10))


def test_configs_shapes_and_determinism():
    c0 = w.config(0)
    assert c0.d == 1 and c0.N == 65536 and c0.M == (1024,)
    assert c0.Q.shape == (1, 65536) and c0.a.dtype == np.complex128
    assert np.all(c0.Q >= -math.pi) and np.all(c0.Q < math.pi)
    assert abs(c0.R - 0.75) < 1e-15
    again = w.config(0)
    assert np.array_equal(c0.Q, again.Q) and np.array_equal(c0.a, again.a)
    g = w.gen_mesh(2, 8, 4, 0.5, (0.5, 0.3), 1.0 / 256, 64, seed=3)
    assert g.N == 8 * 8 * 4 * 4 and g.Q.shape == (2, g.N)
    assert np.isclose(g.P[0].min(), 0.25) and np.isclose(g.P[0].max(), 0.75)
    assert np.isclose(g.P[1].min(), 0.05) and np.isclose(g.P[1].max(), 0.55)


def test_serving_requests_cover_the_mix():
    ds, epss = set(), set()
    for r in range(40):
        req = w.serving_request(r)
        ds.add(req.d)
        epss.add(req.eps)
        assert 2 ** 12 <= req.N < 2 ** 22
        assert req.Q.shape == (req.d, req.N)
    assert ds == {1, 2} and len(epss) == 3


@pytest.mark.parametrize("k", [0, 1, 2])
def test_native_generator_matches(k):
    """fggc_gen_config (C ABI, host) draws the same packets as the Python generator:
    uniform-derived values bit for bit, Box-Muller normals to the last ulp or two
    (the two sides call different cos / log1p implementations)."""
    from paper_2504_21785_amd import fggc as F
    ps = w.config(k)
    info = F.config_info(k)
    assert (info["d"], info["N"], info["M"]) == (ps.d, ps.N, tuple(ps.M))
    assert info["eps"] == ps.eps and abs(info["R"] - ps.R) <= 1e-15
    Q, P, S, a = F.gen_config(k)
    assert np.array_equal(S, ps.S)
    if k >= 2:  # mesh momenta: no normals involved
        assert np.array_equal(P, ps.P) and np.array_equal(Q, ps.Q)
    assert np.max(np.abs(P - ps.P)) <= 4e-16 * np.max(np.abs(ps.P))
    assert np.max(np.abs(Q - ps.Q)) <= 1e-15
    assert np.max(np.abs(a - ps.a)) <= 1e-15
    # another seed gives other values, and the same ones on both sides
    Q2, _, S2, _ = F.gen_config(k, seed=12345)
    assert not np.array_equal(S2, S)
    assert np.array_equal(S2, w.config(k, seed=12345).S)
