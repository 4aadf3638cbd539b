"""Parity bound used by the GPU tests: relative L2 and max-abs, on every result.

rel-L2  = ||u - ref||_2 / ||ref||_2 over the compared points;
max-abs = max |u - ref| / max |ref| over the same points.
Both must be within the stated tolerance (max_tol defaults to tol), so that
an error confined to a few points (a seam, one p-slice) cannot hide inside a
norm taken over a large grid.
"""
import sys

import numpy as np


def errors(u, ref):
    u = np.asarray(u).reshape(-1).astype(np.complex128)
    ref = np.asarray(ref).reshape(-1).astype(np.complex128)
    if u.shape != ref.shape:
        raise AssertionError(f"shape mismatch {u.shape} vs {ref.shape}")
    nr = float(np.linalg.norm(ref))
    mr = float(np.max(np.abs(ref))) if ref.size else 0.0
    e = float(np.linalg.norm(u - ref)) / nr if nr > 0 else float(np.linalg.norm(u))
    m = float(np.max(np.abs(u - ref))) / mr if mr > 0 else (float(np.max(np.abs(u))) if u.size else 0.0)
    return e, m


def check(u, ref, tol, what="", max_tol=None):
    """Assert rel-L2 <= tol and max-abs / max|ref| <= max_tol (default tol); returns both."""
    mt = tol if max_tol is None else max_tol
    e, m = errors(u, ref)
    print(f"{what}: rel-L2 {e:.3e} (<= {tol:.1e}), max-abs/max|ref| {m:.3e} (<= {mt:.1e})", flush=True)
    sys.stdout.flush()
    assert np.isfinite(e) and np.isfinite(m), (what, e, m)
    assert e <= tol, (what, "rel-L2", e, tol)
    assert m <= mt, (what, "max-abs", m, mt)
    return e, m
