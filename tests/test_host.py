"""Host-side logic of libfggc that runs without a GPU.

- the shared library loads and exports every function include/fggc.h declares;
- argument errors come back as status codes (no GPU touched);
- the default strategy and mesh choice;
- the host eigen-decomposition of the eps-free Gram matrix (3.22) against
  numpy's eigh of the oracle's Gram matrix;
- the serving policy (admission under a budget, packet-count buckets, box
  alignment), compiled from its header with g++ and driven from here.
"""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fggc.h")
CSRC = os.path.join(ROOT, "paper_2504_21785_amd", "csrc")

from paper_2504_21785_amd import fggc as F  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fggc_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20, names
    L = ctypes.CDLL(F.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert F.lib().fggc_version().decode().startswith("fggc")


def test_null_arguments_are_rejected_without_a_device():
    L = F.lib()
    g = F.Grid()
    g.d = 1
    g.n[0] = 64
    assert L.fggc_direct_sum(None, None, 0.01, ctypes.byref(g), 0.5, 1.0, 0, None, None) == F.FGGC_EINVAL
    assert "NULL" in F.last_error()
    st = F.default_strategy(1, 1 / 64)
    assert L.fggc_reconstruct(None, None, 0.01, ctypes.byref(g), ctypes.byref(st), 1.0, 0, None,
                              None) == F.FGGC_EINVAL
    assert L.fggc_server_wait(None, 1, 0.0) == F.FGGC_EINVAL
    assert L.fggc_server_submit(None, None, 0.01, None, None, 1.0, 0, None, None) == F.FGGC_EINVAL
    s = F.Strategy()
    assert L.fggc_default_strategy(4, 0.01, b"Q4P2", ctypes.byref(s)) == F.FGGC_EINVAL
    assert L.fggc_default_strategy(1, -1.0, b"Q4P2", ctypes.byref(s)) == F.FGGC_EINVAL
    assert L.fggc_default_strategy(1, 0.01, b"Q3P3", ctypes.byref(s)) == F.FGGC_EINVAL


@pytest.mark.parametrize("eps,nq", [(2.0 ** -6, 128), (2.0 ** -7, 128), (2.0 ** -8, 256),
                                    (2.0 ** -10, 512)])
def test_default_strategy_mesh(eps, nq):
    # Nq = the power of two nearest (in ratio) 4 pi / sqrt(eps); dp = pi sqrt(eps) / 8
    d = 2
    st = F.default_strategy(d, eps, "Q4P2").describe()
    assert st["Nq"][:d] == [nq] * d and st["Nq"][d] == 1
    assert st["dp"][0] == pytest.approx(math.pi * math.sqrt(eps) / 8, rel=1e-15)
    assert st["dq_off"] == [-1, 0, 1, 2] and st["dp_off"] == [0, 1]
    Cq = 2 * math.pi / nq / math.sqrt(eps)
    assert 0.35 < Cq < 0.6
    q2p4 = F.default_strategy(1, eps, "Q2P4").describe()
    assert q2p4["dq_off"] == [0, 1] and q2p4["dp_off"] == [-1, 0, 1, 2]


@pytest.mark.parametrize("name,Cq,Cp", [("Q4P2", math.pi / 8, math.pi / 8), ("Q2P2", 0.5554, 0.3927),
                                        ("Q4P4", 0.4, 0.7)])
def test_plan_gram_eigenpairs(orc, name, Cq, Cp):
    st = F.default_strategy(1, 1 / 64, name).describe()
    dq, dp = st["dq_off"], st["dp_off"]
    w, V = F.plan_gram(dq, dp, Cq, Cp)
    n = len(dq) * len(dp)
    # the oracle's (3.22) Gram matrix over the basis (dq[a], dp[b]), index a * np + b
    bq = [x for x in dq for _ in dp]
    bp = [y for _ in dq for y in dp]
    A = orc.gram(bq, bp, Cq, Cp)
    assert A.shape == (n, n)
    wr = np.linalg.eigvalsh(A)
    assert np.allclose(w, wr, rtol=1e-12, atol=1e-15 * wr.max())
    assert np.all(np.diff(w) >= 0)
    # V diag(w) V^H reproduces A and V is unitary
    assert np.allclose(V @ np.diag(w) @ V.conj().T, A, atol=1e-13)
    assert np.allclose(V.conj().T @ V, np.eye(n), atol=1e-13)


DRIVER = r"""
#include "admission.h"
#include <cstdio>
#include <cstdlib>
#include <cstring>
using namespace fggc;
int main(int argc, char **argv) {
  if (!strcmp(argv[1], "pad")) {
    for (int i = 2; i < argc; ++i) printf("%lld\n", (long long)padded_count(atoll(argv[i])));
  } else if (!strcmp(argv[1], "box")) {
    long long lo = atoll(argv[2]), n = atoll(argv[3]), a = atoll(argv[4]);
    int64_t L = lo, N = n;
    align_box(L, N, a);
    printf("%lld %lld\n", (long long)L, (long long)N);
  } else {  // admit budget need cap0 busy0 cap1 busy1 ...
    size_t budget = strtoull(argv[2], 0, 10), need = strtoull(argv[3], 0, 10);
    std::vector<SlotState> s;
    for (int i = 4; i + 1 < argc; i += 2) s.push_back({(size_t)strtoull(argv[i], 0, 10), atoi(argv[i + 1]) != 0});
    Admission a = plan_admission(s, need, budget);
    printf("%d %zu", a.slot, a.limit);
    for (int j : a.release) printf(" %d", j);
    printf("\n");
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def policy(tmp_path_factory):
    d = tmp_path_factory.mktemp("policy")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)

    def run(*args):
        return subprocess.run([str(exe)] + [str(a) for a in args], check=True, capture_output=True,
                              text=True).stdout.split("\n")[0].split()
    return run


def test_padded_count(policy):
    Ns = [1, 63, 64, 65, 100, 4095, 4096, 4097, 5000, 123457, 2 ** 22 - 1, 2 ** 22, 2 ** 22 + 1, 2 ** 30]
    out = [int(x) for x in subprocess_lines(policy, "pad", Ns)]
    for N, p in zip(Ns, out):
        assert p >= N and p >= 64
        assert p <= max(64, 1.25 * N)
        # p = m 2^e with m in 4..8
        e = 0
        while p % (2 ** (e + 1)) == 0 and p // 2 ** (e + 1) >= 4:
            e += 1
        assert 4 <= p // 2 ** e <= 8, (N, p)
    # buckets are monotone and idempotent
    assert out == sorted(out)
    assert [int(x) for x in subprocess_lines(policy, "pad", out)] == out


def subprocess_lines(policy, cmd, args):
    return [policy(cmd, a)[0] for a in args]


@pytest.mark.parametrize("lo,n", [(0, 1), (1, 1), (-3, 5), (20, 41), (-1, 2), (7, 7)])
def test_align_box(policy, lo, n):
    L, N = (int(x) for x in policy("box", lo, n, 2))
    assert L <= lo and L + N >= lo + n and L % 2 == 0 and (L + N) % 2 == 0
    assert L > lo - 2 and L + N < lo + n + 2


def test_admission_prefers_a_slot_that_already_fits(policy):
    # slots: cap 100 idle, cap 50 idle, cap 10 busy; need 40 -> the smallest idle that fits (1)
    out = policy("admit", 1000, 40, 100, 0, 50, 0, 10, 1)
    assert out == ["1", "50"]


def test_admission_grows_within_budget(policy):
    # nothing idle fits 300: the largest idle slot grows; limit = budget - others
    out = policy("admit", 1000, 300, 100, 0, 50, 0, 10, 1)
    assert out[0] == "0" and int(out[1]) == 1000 - 60 and len(out) == 2


def test_admission_releases_idle_memory(policy):
    # budget 500, need 400: slot 0 (cap 100) grows only if idle slot 1 (cap 300) is freed
    out = policy("admit", 500, 400, 100, 0, 300, 0, 0, 1)
    assert out[0] == "1"  # the largest idle slot is the one that grows
    out = policy("admit", 500, 450, 300, 0, 100, 0, 0, 1)
    assert out[0] == "0" and out[2:] == ["1"] and int(out[1]) == 500


def test_admission_waits_for_busy_memory(policy):
    # busy slots hold 400 of 500: a 200-byte request must wait
    out = policy("admit", 500, 200, 400, 1, 0, 0)
    assert out[0] == "-1"
    # no idle slot at all
    assert policy("admit", 10 ** 9, 1, 5, 1, 5, 1)[0] == "-1"
