"""ctypes binding of libfggc (argument marshalling only).

Every step of the reconstruction runs in the HIP library; this module only
turns torch tensors (device memory and streams) or numpy arrays (host memory)
into the pointers and sizes of the C ABI declared in include/fggc.h, with the
same names.  It raises when the library has not been built -- there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfggc.so")

FGGC_OK = 0
FGGC_EINVAL = -1
FGGC_ENOMEM = -2
FGGC_EBUDGET = -3
FGGC_EUNSUPPORTED = -4
FGGC_EDEVICE = -5
FGGC_ECANCELLED = -6
FGGC_ETIMEOUT = -7
NOALLOC_SCRATCH_BYTES = 256 << 20  # FGGC_NOALLOC_SCRATCH_BYTES
FP32 = 0
FP64 = 1

_STATUS = {0: "FGGC_OK", -1: "FGGC_EINVAL", -2: "FGGC_ENOMEM", -3: "FGGC_EBUDGET",
           -4: "FGGC_EUNSUPPORTED", -5: "FGGC_EDEVICE", -6: "FGGC_ECANCELLED", -7: "FGGC_ETIMEOUT"}


class FggcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", ctypes.c_int64 * 3)]


class Packets(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("N", ctypes.c_int64), ("Q", ctypes.c_void_p),
                ("P", ctypes.c_void_p), ("S", ctypes.c_void_p), ("a", ctypes.c_void_p)]


class Strategy(ctypes.Structure):
    _fields_ = [("Nq", ctypes.c_int64 * 3), ("dp", ctypes.c_double * 3), ("nq", ctypes.c_int32),
                ("np", ctypes.c_int32), ("dq_off", ctypes.c_int32 * 8),
                ("dp_off", ctypes.c_int32 * 8), ("cutoff", ctypes.c_double)]

    def describe(self) -> dict:
        return {"Nq": list(self.Nq), "dp": list(self.dp), "dq_off": list(self.dq_off[:self.nq]),
                "dp_off": list(self.dp_off[:self.np]), "cutoff": self.cutoff}


class Potential(ctypes.Structure):
    """V(x) = c0 + sum_k w_k x_k^2 / 2 + c1 sum_k cos(kappa x_k) + c2 exp(c3 |x|^2)."""
    _fields_ = [("c0", ctypes.c_double), ("w", ctypes.c_double * 3), ("c1", ctypes.c_double),
                ("kappa", ctypes.c_double), ("c2", ctypes.c_double), ("c3", ctypes.c_double)]


def potential(c0=0.0, w=(0.0, 0.0, 0.0), c1=0.0, kappa=0.0, c2=0.0, c3=0.0) -> Potential:
    V = Potential()
    V.c0, V.c1, V.kappa, V.c2, V.c3 = float(c0), float(c1), float(kappa), float(c2), float(c3)
    for k, v in enumerate((list(w) + [0.0, 0.0, 0.0])[:3]):
        V.w[k] = float(v)
    return V


_lib = None

# (name, restype, argtypes) of every function in include/fggc.h
_VP, _I, _D, _I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
_SIGS = [
    ("fggc_create", _I, [ctypes.POINTER(_VP), _I, ctypes.c_size_t]),
    ("fggc_destroy", None, [_VP]),
    ("fggc_last_error", ctypes.c_char_p, []),
    ("fggc_version", ctypes.c_char_p, []),
    ("fggc_direct_sum", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Grid), _D, _D, _I, _VP, _VP]),
    ("fggc_direct_sum_noalloc", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Grid), _D, _D, _I, _VP,
                                     _VP]),
    ("fggc_direct_sum_box", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Grid),
                                 ctypes.POINTER(_I64), ctypes.POINTER(_I64), _D, _D, _I, _VP, _VP]),
    ("fggc_direct_sum_separable", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Grid), _D, _D, _I,
                                       _VP, _VP]),
    ("fggc_reconstruct", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Grid),
                              ctypes.POINTER(Strategy), _D, _I, _VP, _VP]),
    ("fggc_decompose", _I, [_VP, ctypes.POINTER(Grid), _VP, _D, _D, _I64, _VP, _VP, _VP, _VP]),
    ("fggc_decompose_mesh", _I, [_VP, ctypes.POINTER(Grid), _VP, _D, _D, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                 ctypes.POINTER(_I64), ctypes.POINTER(_D), ctypes.POINTER(_I64),
                                 ctypes.POINTER(_I64), _VP, _VP]),
    ("fggc_propagate", _I, [_VP, ctypes.c_int32, _I64, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(Potential), _D,
                            _I64, _VP]),
    ("fggc_coefficients", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Strategy), _D, _VP, _VP, _VP]),
    ("fggc_learn_select", _I, [_VP, _I64, _VP, _D, _VP, _VP, _VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                               _VP]),
    ("fggc_learn_start", _I, [_VP, ctypes.c_int32, _I64, _I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("fggc_learn_store", _I, [_VP, ctypes.c_int32, _I64, _I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                              _VP]),
    ("fggc_learn_packets", _I, [_VP, ctypes.c_int32, _I64, _I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                _VP, _VP]),
    ("fggc_default_strategy", _I, [_I, _D, ctypes.c_char_p, ctypes.POINTER(Strategy)]),
    ("fggc_config_info", _I, [_I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_I64), ctypes.POINTER(_D),
                              ctypes.POINTER(Grid), ctypes.POINTER(_D)]),
    ("fggc_gen_config", _I, [_I, ctypes.c_uint64, ctypes.POINTER(Packets)]),
    ("fggc_cell_box", _I, [_VP, ctypes.POINTER(Packets), ctypes.POINTER(Strategy),
                           ctypes.POINTER(_I64), ctypes.POINTER(_I64), _VP]),
    ("fggc_cells", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Strategy), _D, _I,
                        ctypes.POINTER(_I64), ctypes.POINTER(_I64), _VP, ctypes.c_size_t, _VP]),
    ("fggc_fft", _I, [_VP, _I, ctypes.POINTER(_I64), _I64, _I, _I, _VP, _VP]),
    ("fggc_plan_gram", _I, [_I, ctypes.POINTER(ctypes.c_int32), _I, ctypes.POINTER(ctypes.c_int32),
                            _D, _D, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    ("fggc_profile", _I, [_VP, _I]),
    ("fggc_stage_time", _I, [_VP, ctypes.c_char_p, ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    ("fggc_server_create", _I, [_VP, _I, ctypes.POINTER(_VP)]),
    ("fggc_server_submit", _I, [_VP, ctypes.POINTER(Packets), _D, ctypes.POINTER(Grid),
                                ctypes.POINTER(Strategy), _D, _I, _VP, ctypes.POINTER(_I64)]),
    ("fggc_server_wait", _I, [_VP, _I64, _D]),
    ("fggc_server_stats", _I, [_VP, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D),
                               ctypes.POINTER(_I64)]),
    ("fggc_server_counters", _I, [_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                              ctypes.POINTER(_I64)]),
    ("fggc_server_reset_stats", _I, [_VP]),
    ("fggc_server_destroy", None, [_VP]),
]


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libfggc.so not found at {LIB_PATH}: build it with "
                               "`python -m paper_2504_21785_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().fggc_last_error().decode()


def _check(rc: int):
    if rc != FGGC_OK:
        raise FggcError(rc, last_error())


def default_strategy(d: int, eps: float, name: str = "Q4P2") -> Strategy:
    st = Strategy()
    _check(lib().fggc_default_strategy(d, eps, name.encode(), ctypes.byref(st)))
    return st


def config_info(config_id: int) -> dict:
    """fggc_config_info: d, N, eps, grid and window radius of a synthetic workload (0-3)."""
    d, N, eps, R = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    g = Grid()
    _check(lib().fggc_config_info(int(config_id), ctypes.byref(d), ctypes.byref(N), ctypes.byref(eps),
                                  ctypes.byref(g), ctypes.byref(R)))
    return {"d": d.value, "N": N.value, "eps": eps.value, "M": tuple(g.n[:d.value]), "R": R.value}


def gen_config(config_id: int, seed: int = 0):
    """fggc_gen_config: the workload's packets as numpy arrays (Q, P [d][N], S [N], a [N] complex)."""
    info = config_info(config_id)
    d, N = info["d"], info["N"]
    Q, P = np.empty((d, N)), np.empty((d, N))
    S, a = np.empty(N), np.empty(N, dtype=np.complex128)
    pk = Packets()
    pk.d, pk.N = d, N
    pk.Q, pk.P, pk.S, pk.a = Q.ctypes.data, P.ctypes.data, S.ctypes.data, a.ctypes.data
    _check(lib().fggc_gen_config(int(config_id), ctypes.c_uint64(seed), ctypes.byref(pk)))
    return Q, P, S, a


def make_strategy(d: int, Nq: Sequence[int], dp: Sequence[float], dq_off: Sequence[int],
                  dp_off: Sequence[int], cutoff: float = 0.0) -> Strategy:
    st = Strategy()
    for k in range(3):
        st.Nq[k] = int(Nq[k]) if k < d else 1
        st.dp[k] = float(dp[k]) if k < d else 1.0
    st.nq, st.np = len(dq_off), len(dp_off)
    for i, v in enumerate(dq_off):
        st.dq_off[i] = int(v)
    for i, v in enumerate(dp_off):
        st.dp_off[i] = int(v)
    st.cutoff = cutoff
    return st


def plan_gram(dq_off, dp_off, Cq: float, Cp: float):
    """Eigenpairs of the one-dimensional Gram matrix (3.22) used by the plan."""
    dq = (ctypes.c_int32 * len(dq_off))(*dq_off)
    dpv = (ctypes.c_int32 * len(dp_off))(*dp_off)
    n1 = len(dq_off) * len(dp_off)
    ev = np.zeros(n1)
    V = np.zeros((n1, n1), dtype=np.complex128)
    _check(lib().fggc_plan_gram(len(dq_off), dq, len(dp_off), dpv, Cq, Cp,
                                ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                V.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return ev, V


def _grid(d: int, M) -> Grid:
    g = Grid()
    g.d = d
    M = list(M) if hasattr(M, "__len__") else [int(M)] * d
    for k in range(3):
        g.n[k] = int(M[k]) if k < d else 1
    return g


def _ptr(x) -> int:
    """Address of a torch tensor (any device) or a numpy array (host)."""
    if x is None:
        return 0
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous:
            raise ValueError("arrays must be C-contiguous")
        return x.ctypes.data
    raise TypeError(f"unsupported buffer type {type(x)}")


# -- argument checks (before any library call: a wrong dtype, shape or
# device would make the kernels read or write outside the buffers) ---------

def _dtype(x) -> str:
    return str(x.dtype).replace("torch.", "")


def _where(x):
    """'host' for numpy arrays and CPU tensors, ('cuda', index) for device tensors."""
    if hasattr(x, "is_cuda") and x.is_cuda:
        return ("cuda", x.device.index)
    if hasattr(x, "data_ptr") or isinstance(x, np.ndarray):
        return "host"
    raise TypeError(f"unsupported buffer type {type(x)}")


def _need(x, name: str, dtype: str, shape=None):
    if x is None:
        raise ValueError(f"{name} is missing")
    if _dtype(x) != dtype:
        raise ValueError(f"{name} must be {dtype}, got {_dtype(x)}")
    if shape is not None and tuple(int(v) for v in x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(int(v) for v in x.shape)}")
    _ptr(x)  # contiguity


def _same_place(*xs):
    places = {_where(x) for x in xs if x is not None}
    if len(places) > 1:
        raise ValueError(f"buffers must all be on the host or all on one device, got {sorted(map(str, places))}")


def check_packets(Q, P, S, a) -> tuple:
    """Q, P: [d][N] float64; S: [N] float64; a: [N] complex128, all in one place; returns (d, N)."""
    for x, n in ((Q, "Q"), (P, "P"), (S, "S"), (a, "a")):
        if x is None:
            raise ValueError(f"{n} is missing")
    if len(Q.shape) != 2:
        raise ValueError(f"Q must be [d][N], got shape {tuple(Q.shape)}")
    d, N = int(Q.shape[0]), int(Q.shape[1])
    if d < 1 or d > 3:
        raise ValueError(f"d must be 1, 2 or 3, got {d}")
    _need(Q, "Q", "float64", (d, N))
    _need(P, "P", "float64", (d, N))
    _need(S, "S", "float64", (N,))
    _need(a, "a", "complex128", (N,))
    _same_place(Q, P, S, a)
    return d, N


def _check_grid(d: int, M):
    n = list(M) if hasattr(M, "__len__") else [int(M)] * d
    if len(n) != d:
        raise ValueError(f"grid has {len(n)} sizes for d = {d}")
    return n


def _check_out(out, npts: int, precision: int, what: str = "out"):
    if out is None:
        return
    want = "complex128" if precision == FP64 else "complex64"
    if _dtype(out) != want:
        raise ValueError(f"{what} must be {want} for this precision, got {_dtype(out)}")
    numel = int(np.prod([int(v) for v in out.shape])) if len(out.shape) else 1
    if numel != npts:
        raise ValueError(f"{what} must hold {npts} values, has {numel}")
    _ptr(out)


def _packets(Q, P, S, a) -> Packets:
    d, N = check_packets(Q, P, S, a)
    pk = Packets()
    pk.d = d
    pk.N = N
    pk.Q, pk.P, pk.S, pk.a = _ptr(Q), _ptr(P), _ptr(S), _ptr(a)
    return pk


def _npts(g: Grid) -> int:
    return int(np.prod([int(g.n[k]) for k in range(g.d)]))


def _check_out_for(out, like, npts: int, precision: int):
    """A caller's output: the precision's dtype, one value per point, and (for a
    device tensor) the device of the inputs when those are on a device."""
    if precision not in (FP32, FP64):
        raise ValueError(f"precision must be FP32 ({FP32}) or FP64 ({FP64})")
    if out is None:
        return
    _check_out(out, npts, precision)
    wo, wi = _where(out), _where(like)
    if wo != "host" and wi != "host" and wo != wi:
        raise ValueError(f"out is on {wo}, the packets on {wi}")


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


class Context:
    """A libfggc context on one HIP device (fggc_create / fggc_destroy)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(lib().fggc_create(ctypes.byref(h), device, hbm_budget_bytes))
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().fggc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- reconstruction -----------------------------------------------------
    def direct_sum(self, Q, P, S, a, eps: float, M, window_radius: float, scale: float = 1.0,
                   precision: int = FP32, out=None, stream=None):
        """fggc_direct_sum.  Q, P: [d][N] float64; S: [N] float64; a: [N] complex128.

        Buffers are torch tensors (on the GPU: device path, stream-ordered on
        the current stream) or numpy arrays (host path, synchronous).  Returns
        `out` (allocated like Q when None), shape = grid.
        """
        d, _ = check_packets(Q, P, S, a)
        g = _grid(d, _check_grid(d, M))
        _check_out_for(out, Q, _npts(g), precision)
        out = self._alloc_out(Q, g, precision, out)
        pk = _packets(Q, P, S, a)
        _check(lib().fggc_direct_sum(self.h, ctypes.byref(pk), float(eps), ctypes.byref(g),
                                     float(window_radius), float(scale), int(precision),
                                     _ptr(out), _stream_ptr(stream) if _on_device(Q) else None))
        return out

    def direct_sum_noalloc(self, Q, P, S, a, eps: float, M, window_radius: float, out, scale: float = 1.0,
                           precision: int = FP32, stream=None):
        """fggc_direct_sum_noalloc: fggc_direct_sum with the library's fixed
        per-GPU scratch and no allocation; packets and `out` are device tensors."""
        d, _ = check_packets(Q, P, S, a)
        g = _grid(d, _check_grid(d, M))
        if out is None:
            raise ValueError("direct_sum_noalloc writes into a caller-supplied `out`")
        _check_out_for(out, Q, _npts(g), precision)
        pk = _packets(Q, P, S, a)
        _check(lib().fggc_direct_sum_noalloc(self.h, ctypes.byref(pk), float(eps), ctypes.byref(g),
                                             float(window_radius), float(scale), int(precision),
                                             _ptr(out), _stream_ptr(stream)))
        return out

    def direct_sum_box(self, Q, P, S, a, eps: float, M, box_lo, box_n, window_radius: float,
                       scale: float = 1.0, precision: int = FP32, out=None, stream=None):
        """fggc_direct_sum_box: the direct sum at the points of a box of the grid."""
        d, _ = check_packets(Q, P, S, a)
        g = _grid(d, _check_grid(d, M))
        if len(list(box_lo)) != d or len(list(box_n)) != d:
            raise ValueError("box_lo and box_n need one entry per dimension")
        _check_out_for(out, Q, int(np.prod([int(v) for v in box_n])), precision)
        lo = (ctypes.c_int64 * 3)(*[int(v) for v in list(box_lo) + [0] * (3 - d)])
        n = (ctypes.c_int64 * 3)(*[int(v) for v in list(box_n) + [1] * (3 - d)])
        if out is None:
            bg = _grid(d, list(box_n))
            out = self._alloc_out(Q, bg, precision, None)
        pk = _packets(Q, P, S, a)
        _check(lib().fggc_direct_sum_box(self.h, ctypes.byref(pk), float(eps), ctypes.byref(g), lo, n,
                                         float(window_radius), float(scale), int(precision),
                                         _ptr(out), _stream_ptr(stream) if _on_device(Q) else None))
        return out

    def direct_sum_separable(self, Q, P, S, a, eps: float, M, window_half_width: float, scale: float = 1.0,
                             precision: int = FP32, out=None, stream=None):
        """fggc_direct_sum_separable: the box-window direct sum on the matrix cores (d = 2, FP32)."""
        d, _ = check_packets(Q, P, S, a)
        g = _grid(d, _check_grid(d, M))
        _check_out_for(out, Q, _npts(g), precision)
        out = self._alloc_out(Q, g, precision, out)
        pk = _packets(Q, P, S, a)
        _check(lib().fggc_direct_sum_separable(self.h, ctypes.byref(pk), float(eps), ctypes.byref(g),
                                               float(window_half_width), float(scale), int(precision),
                                               _ptr(out), _stream_ptr(stream) if _on_device(Q) else None))
        return out

    def decompose(self, u0, eps: float, M, window_radius: float, q, p, out=None, stream=None):
        """fggc_decompose: A(0, q, p) of eq. (2.7) for the [d][N] points (q, p) from u0 on the grid.

        u0: complex128 grid values (torch on the GPU, or numpy).  Returns A
        ([N] complex128, allocated like q when out is None).
        """
        if len(q.shape) != 2:
            raise ValueError(f"q must be [d][N], got shape {tuple(q.shape)}")
        d, N = int(q.shape[0]), int(q.shape[1])
        g = _grid(d, _check_grid(d, M))
        _need(q, "q", "float64", (d, N))
        _need(p, "p", "float64", (d, N))
        _need(u0, "u0", "complex128")
        if int(np.prod([int(v) for v in u0.shape])) != _npts(g):
            raise ValueError(f"u0 must hold {_npts(g)} grid values")
        _same_place(u0, q, p)
        if out is not None:
            _need(out, "out", "complex128")
            if int(np.prod([int(v) for v in out.shape])) != N:
                raise ValueError(f"out must hold {N} values")
            _same_place(q, out)
        if out is None:
            if hasattr(q, "device"):
                import torch
                out = torch.empty(N, dtype=torch.complex128, device=q.device)
            else:
                out = np.empty(N, dtype=np.complex128)
        _check(lib().fggc_decompose(self.h, ctypes.byref(g), _ptr(u0), float(eps), float(window_radius), N,
                                    _ptr(q), _ptr(p), _ptr(out), _stream_ptr(stream) if _on_device(q) else None))
        return out

    def decompose_mesh(self, u0, eps: float, M, window_half_width: float, Nq, q_lo, q_n, dp, p_lo, p_n,
                       out=None, stream=None):
        """fggc_decompose_mesh: A(0, q, p) of eq. (2.7) on the product mesh
        q_k = -pi + (q_lo[k] + i) 2 pi / Nq[k], p_k = (p_lo[k] + j) dp[k] (box window).

        Returns [prod q_n * prod p_n] complex128, q-major (allocated like u0 when out is None).
        """
        M = list(M) if hasattr(M, "__len__") else [int(M)]
        d = len(M)
        g = _grid(d, M)
        _need(u0, "u0", "complex128")
        if int(np.prod([int(v) for v in u0.shape])) != _npts(g):
            raise ValueError(f"u0 must hold {_npts(g)} grid values")
        for v, n in ((Nq, "Nq"), (q_lo, "q_lo"), (q_n, "q_n"), (dp, "dp"), (p_lo, "p_lo"), (p_n, "p_n")):
            if len(list(v)) != d:
                raise ValueError(f"{n} needs one entry per dimension")
        arr = lambda v, t: (t * 3)(*[(float(x) if t is _D else int(x)) for x in (list(v) + [0] * (3 - d))])
        total = int(np.prod(list(q_n))) * int(np.prod(list(p_n)))
        if out is not None:
            _need(out, "out", "complex128")
            if int(np.prod([int(v) for v in out.shape])) != total:
                raise ValueError(f"out must hold {total} values")
            _same_place(u0, out)
        if out is None:
            if hasattr(u0, "device"):
                import torch
                out = torch.empty(total, dtype=torch.complex128, device=u0.device)
            else:
                out = np.empty(total, dtype=np.complex128)
        _check(lib().fggc_decompose_mesh(self.h, ctypes.byref(g), _ptr(u0), float(eps), float(window_half_width),
                                         arr(Nq, _I64), arr(q_lo, _I64), arr(q_n, _I64), arr(dp, _D), arr(p_lo, _I64),
                                         arr(p_n, _I64), _ptr(out),
                                         _stream_ptr(stream) if _on_device(u0) else None))
        return out

    def propagate(self, Q, P, S, a, V: Potential, dt: float, nsteps: int, jac=None, stream=None):
        """fggc_propagate: RK4 for eq. (2.3)-(2.6), in place on Q, P, S, a (and jac).

        Q, P: [d][N] float64; S: [N] float64; a: [N] complex128; jac: None or
        [N][2][d][d] complex128.  Torch tensors on the GPU run stream-ordered;
        numpy arrays are staged (synchronous).
        """
        d, N = check_packets(Q, P, S, a)
        if jac is not None:
            _need(jac, "jac", "complex128")
            if int(np.prod([int(v) for v in jac.shape])) != N * 2 * d * d:
                raise ValueError(f"jac must hold [N][2][d][d] = {N * 2 * d * d} values")
            _same_place(Q, jac)
        for x in (Q, P, S, a) + ((jac,) if jac is not None else ()):
            if hasattr(x, "is_contiguous") and not x.is_contiguous():
                raise ValueError("propagate works in place: arrays must be contiguous")
            if isinstance(x, np.ndarray) and not x.flags["C_CONTIGUOUS"]:
                raise ValueError("propagate works in place: arrays must be contiguous")
        _check(lib().fggc_propagate(self.h, d, N, _ptr(Q), _ptr(P), _ptr(S), _ptr(a),
                                    _ptr(jac) if jac is not None else None, ctypes.byref(V), float(dt),
                                    int(nsteps), _stream_ptr(stream) if _on_device(Q) else None))
        return Q, P, S, a

    def coefficients(self, Q, P, S, a, eps: float, strategy: Strategy, scale: float = 1.0, stream=None):
        """fggc_coefficients: per-packet least-squares coefficients (device tensors).

        Returns (c [N][(nq np)^d] complex128, cells [N][2][d] int32) on the
        packets' device."""
        import torch
        d, N = check_packets(Q, P, S, a)
        if not _on_device(Q):
            raise ValueError("coefficients takes device tensors")
        n1 = int(strategy.nq) * int(strategy.np)
        c = torch.empty((N, n1 ** d), dtype=torch.complex128, device=Q.device)
        cells = torch.empty((N, 2, d), dtype=torch.int32, device=Q.device)
        pk = _packets(Q, P, S, a)
        _check(lib().fggc_coefficients(self.h, ctypes.byref(pk), float(eps), ctypes.byref(strategy), float(scale),
                                       _ptr(c), _ptr(cells), _stream_ptr(stream)))
        return c, cells

    # -- multi-step FGGC bookkeeping (Alg. 3); device tensors only ----------
    def learn_select(self, A0, prune: float, learned, keep_idx, new_idx, stream=None):
        """fggc_learn_select: fills keep_idx / new_idx (int64 [Nm]) and marks the
        new points in learned (uint8 [Nm]); returns (n_keep, n_new)."""
        Nm = int(A0.shape[0])
        for x, nm, dt in ((A0, "A0", "complex128"), (learned, "learned", "uint8"), (keep_idx, "keep_idx", "int64"),
                          (new_idx, "new_idx", "int64")):
            _need(x, nm, dt)
            if int(np.prod([int(v) for v in x.shape])) != Nm:
                raise ValueError(f"{nm} must hold {Nm} values")
        nk, nn = _I64(), _I64()
        _check(lib().fggc_learn_select(self.h, Nm, _ptr(A0), float(prune), _ptr(learned), _ptr(keep_idx),
                                       _ptr(new_idx), ctypes.byref(nk), ctypes.byref(nn), _stream_ptr(stream)))
        return int(nk.value), int(nn.value)

    def learn_start(self, idx, n: int, qm, pm, Q, P, S, A, stream=None):
        """fggc_learn_start: packets at mesh points idx[:n] with S = 0 and A = 1."""
        d, Nm = int(qm.shape[0]), int(qm.shape[1])
        _check(lib().fggc_learn_start(self.h, d, Nm, int(n), _ptr(idx), _ptr(qm), _ptr(pm), _ptr(Q), _ptr(P),
                                      _ptr(S), _ptr(A), _stream_ptr(stream)))

    def learn_store(self, idx, n: int, Q, P, S, A, Qf, Pf, Sf, ratio, stream=None):
        """fggc_learn_store: evolved packets into the per-point tables at idx[:n]."""
        d, Nm = int(Qf.shape[0]), int(Qf.shape[1])
        _check(lib().fggc_learn_store(self.h, d, Nm, int(n), _ptr(idx), _ptr(Q), _ptr(P), _ptr(S), _ptr(A),
                                      _ptr(Qf), _ptr(Pf), _ptr(Sf), _ptr(ratio), _stream_ptr(stream)))

    def learn_packets(self, idx, n: int, Qf, Pf, Sf, ratio, A0, Q, P, S, a, stream=None):
        """fggc_learn_packets: the kept points' learned packets, a = A0 * ratio."""
        d, Nm = int(Qf.shape[0]), int(Qf.shape[1])
        _check(lib().fggc_learn_packets(self.h, d, Nm, int(n), _ptr(idx), _ptr(Qf), _ptr(Pf), _ptr(Sf),
                                        _ptr(ratio), _ptr(A0), _ptr(Q), _ptr(P), _ptr(S), _ptr(a),
                                        _stream_ptr(stream)))

    def reconstruct(self, Q, P, S, a, eps: float, M, strategy: Strategy, scale: float = 1.0,
                    precision: int = FP32, out=None, stream=None):
        """fggc_reconstruct (FGGC); same buffer conventions as direct_sum."""
        d, _ = check_packets(Q, P, S, a)
        g = _grid(d, _check_grid(d, M))
        _check_out_for(out, Q, _npts(g), precision)
        out = self._alloc_out(Q, g, precision, out)
        pk = _packets(Q, P, S, a)
        _check(lib().fggc_reconstruct(self.h, ctypes.byref(pk), float(eps), ctypes.byref(g),
                                      ctypes.byref(strategy), float(scale), int(precision),
                                      _ptr(out), _stream_ptr(stream) if _on_device(Q) else None))
        return out

    def cell_box(self, Q, P, S, a, strategy: Strategy, stream=None):
        d, _ = check_packets(Q, P, S, a)
        pk = _packets(Q, P, S, a)
        lo = (ctypes.c_int64 * 3)()
        n = (ctypes.c_int64 * 3)()
        _check(lib().fggc_cell_box(self.h, ctypes.byref(pk), ctypes.byref(strategy), lo, n,
                                   _stream_ptr(stream) if _on_device(Q) else None))
        return np.array(lo[:d]), np.array(n[:d])

    def cells(self, Q, P, S, a, eps: float, strategy: Strategy, scale: float = 1.0,
              precision: int = FP32, box=None, stream=None):
        """fggc_cells: the dense cell array of eq. (2.25) as a numpy array [slices][q]."""
        d, _ = check_packets(Q, P, S, a)
        if precision not in (FP32, FP64):
            raise ValueError(f"precision must be FP32 ({FP32}) or FP64 ({FP64})")
        if box is None:
            box = self.cell_box(Q, P, S, a, strategy, stream)
        lo, n = box
        nq = int(np.prod([strategy.Nq[k] for k in range(d)]))
        ns = int(np.prod(n))
        dt = np.complex128 if precision == FP64 else np.complex64
        out = np.zeros((ns, nq), dtype=dt)
        pk = _packets(Q, P, S, a)
        lo_c = (ctypes.c_int64 * 3)(*[int(v) for v in lo])
        n_c = (ctypes.c_int64 * 3)(*[int(v) for v in n])
        _check(lib().fggc_cells(self.h, ctypes.byref(pk), float(eps), ctypes.byref(strategy),
                                float(scale), int(precision), lo_c, n_c, out.ctypes.data,
                                out.nbytes, _stream_ptr(stream) if _on_device(Q) else None))
        return out, np.asarray(lo), np.asarray(n)

    def fft(self, data, dims: Sequence[int], batch: int, direction: int, precision: int = FP32,
            stream=None):
        """fggc_fft in place on a torch complex tensor on the device."""
        if not (1 <= len(list(dims)) <= 3):
            raise ValueError("dims must have 1 to 3 entries")
        _need(data, "data", "complex128" if precision == FP64 else "complex64")
        if _where(data) == "host":
            raise ValueError("fggc_fft transforms device memory: pass a GPU tensor")
        want = int(batch) * int(np.prod([int(v) for v in dims]))
        if int(np.prod([int(v) for v in data.shape])) != want:
            raise ValueError(f"data must hold batch * prod(dims) = {want} values")
        nd = (ctypes.c_int64 * 3)(*[int(v) for v in list(dims) + [1] * (3 - len(dims))])
        _check(lib().fggc_fft(self.h, len(dims), nd, int(batch), int(direction), int(precision),
                              _ptr(data), _stream_ptr(stream)))
        return data

    def profile(self, enable: bool):
        """fggc_profile: start (True) or stop (False) per-stage event timing; resets totals."""
        _check(lib().fggc_profile(self.h, 1 if enable else 0))

    def stage_time(self, stage: str):
        """fggc_stage_time: (total milliseconds, launches) recorded for one stage."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().fggc_stage_time(self.h, stage.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    @staticmethod
    def _alloc_out(like, g: Grid, precision: int, out):
        shape = tuple(g.n[k] for k in range(g.d))
        if out is not None:
            return out
        if hasattr(like, "is_cuda"):  # a torch tensor (numpy arrays have .device too)
            import torch
            dt = torch.complex128 if precision == FP64 else torch.complex64
            return torch.empty(shape, dtype=dt, device=like.device)
        return np.empty(shape, dtype=np.complex128 if precision == FP64 else np.complex64)


def _on_device(x) -> bool:
    return hasattr(x, "is_cuda") and x.is_cuda


class Server:
    """fggc_server_*: continuous-batching reconstruction service on one context."""

    def __init__(self, ctx: Context, n_streams: int = 4):
        h = ctypes.c_void_p()
        _check(lib().fggc_server_create(ctx.h, n_streams, ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self._keep = {}

    def submit(self, Q, P, S, a, eps: float, M, strategy: Optional[Strategy] = None,
               scale: float = 1.0, precision: int = FP32, out=None):
        """Submit packets (numpy arrays, or device tensors kept alive until wait);
        returns (ticket, output) -- output is filled when the ticket completes.
        out defaults to a numpy array for host packets and a device tensor otherwise."""
        d, _ = check_packets(Q, P, S, a)
        g = _grid(d, _check_grid(d, M))
        _check_out_for(out, Q, _npts(g), precision)
        shape = tuple(g.n[k] for k in range(d))
        if out is None:
            if _on_device(Q):
                import torch
                out = torch.empty(shape, dtype=torch.complex128 if precision == FP64 else torch.complex64,
                                  device=Q.device)
            else:
                out = np.zeros(shape, dtype=np.complex128 if precision == FP64 else np.complex64)
        if _on_device(Q):
            import torch
            torch.cuda.current_stream().synchronize()  # packets must be written before submit
        pk = _packets(Q, P, S, a)
        t = ctypes.c_int64()
        _check(lib().fggc_server_submit(self.h, ctypes.byref(pk), float(eps), ctypes.byref(g),
                                        ctypes.byref(strategy) if strategy is not None else None,
                                        float(scale), int(precision), _ptr(out),
                                        ctypes.byref(t)))
        self._keep[t.value] = (out, Q, P, S, a)
        return t.value, out

    def wait(self, ticket: int, timeout_s: float = -1.0) -> int:
        rc = lib().fggc_server_wait(self.h, ticket, float(timeout_s))
        if rc != FGGC_ETIMEOUT:
            self._keep.pop(ticket, None)
        return rc

    def stats(self):
        p50, p99, pps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().fggc_server_stats(self.h, ctypes.byref(p50), ctypes.byref(p99),
                                       ctypes.byref(pps), ctypes.byref(n)))
        return {"p50_s": p50.value, "p99_s": p99.value, "packets_per_s": pps.value,
                "completed": n.value}

    def counters(self):
        e, c, r = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fggc_server_counters(self.h, ctypes.byref(e), ctypes.byref(c), ctypes.byref(r)))
        return {"eager": e.value, "captured": c.value, "replayed": r.value}

    def reset_stats(self):
        _check(lib().fggc_server_reset_stats(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().fggc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
