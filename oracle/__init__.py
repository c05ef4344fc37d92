"""ctypes view of the CPU oracle (``oracle/rotvote_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It is independent of
the HIP library (no shared source, no shared helpers).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "rotvote_oracle.c"
LIB = HERE / "liborc.so"

# -ffp-contract=off: no implicit fused multiply-adds; no fast-math, so '/' and
# sqrtf stay correctly rounded and denormals are kept.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra"]


def build(src: Path = SRC, out: Path = LIB, extra: list | None = None) -> Path:
    """Compile the oracle with gcc (host only)."""
    cmd = ["gcc", *CFLAGS, *(extra or []), "-o", str(out), str(src), "-lm"]
    subprocess.run(cmd, check=True)
    return out


_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


class Oracle:
    """Numpy-friendly wrapper around one compiled oracle library."""

    def __init__(self, path: Path | str = LIB):
        path = Path(path)
        if not path.exists():
            build(out=path)
        self.path = path
        L = self.lib = ct.CDLL(str(path))
        L.orc_tables.argtypes = [ct.c_int32, _f32p, _f32p]
        L.orc_tables.restype = None
        L.orc_residual_bound.argtypes = [ct.c_float]
        L.orc_residual_bound.restype = ct.c_float
        L.orc_normalise.argtypes = [_f32p, _f32p]
        L.orc_normalise.restype = ct.c_int32
        L.orc_normalise_pairs.argtypes = [_f32p, _f32p, ct.c_int64, _f32p, _f32p, _u8p]
        L.orc_normalise_pairs.restype = None
        L.orc_circle_basis.argtypes = [_f32p, _f32p, _f32p, _f32p]
        L.orc_circle_basis.restype = ct.c_int32
        L.orc_cell_of.argtypes = [_f32p, ct.c_int32, _f32p, _f32p, _i32p]
        L.orc_cell_of.restype = ct.c_int32
        L.orc_circle_cells.argtypes = [_f32p, _f32p, ct.c_int32, ct.c_int32, _i32p]
        L.orc_circle_cells.restype = ct.c_int32
        L.orc_histogram.argtypes = [_f32p, _f32p, ct.c_int64, ct.c_int32, ct.c_int32, _i32p,
                                    ct.c_int32]
        L.orc_histogram.restype = None
        L.orc_topk.argtypes = [_i32p, ct.c_int32, ct.c_int32, _i32p, _i32p]
        L.orc_topk.restype = ct.c_int32
        L.orc_decode.argtypes = [ct.c_int32, ct.c_int32, _f32p]
        L.orc_decode.restype = None
        L.orc_residual.argtypes = [_f32p, _f32p, _f32p]
        L.orc_residual.restype = ct.c_float
        L.orc_rescore.argtypes = [_f32p, _f32p, ct.c_int64, _f32p, ct.c_float, ct.c_void_p]
        L.orc_rescore.restype = ct.c_int64
        L.orc_solve.argtypes = [_f32p, _f32p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_float,
                                ct.c_int32, ct.c_int32, _i32p, _i32p, _i32p, _i64p, _f32p,
                                ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32), ct.c_void_p]
        L.orc_solve.restype = ct.c_int32

    # ---- per-step views ------------------------------------------------
    def tables(self, J: int):
        C = np.empty(J, np.float32)
        S = np.empty(J, np.float32)
        self.lib.orc_tables(J, C, S)
        return C, S

    def residual_bound(self, eps_rad: float) -> np.float32:
        return np.float32(self.lib.orc_residual_bound(float(np.float32(eps_rad))))

    def normalise(self, v):
        out = np.zeros(3, np.float32)
        ok = self.lib.orc_normalise(np.ascontiguousarray(v, np.float32), out)
        return bool(ok), out

    def normalise_pairs(self, x, y):
        """Step 1 for SoA [3, n] arrays: (a, b, ok) with a, b float32 [3, n]."""
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        n = x.shape[1]
        a = np.empty((3, n), np.float32)
        b = np.empty((3, n), np.float32)
        ok = np.empty(n, np.uint8)
        self.lib.orc_normalise_pairs(x, y, n, a, b, ok)
        return a, b, ok.astype(bool)

    def circle_basis(self, a, b):
        u = np.empty(4, np.float32)
        v = np.empty(4, np.float32)
        k = self.lib.orc_circle_basis(np.ascontiguousarray(a, np.float32),
                                      np.ascontiguousarray(b, np.float32), u, v)
        return u, v, int(k)

    def cell_of(self, q, G: int):
        qc = np.empty(4, np.float32)
        t = np.empty(3, np.float32)
        ic = np.empty(3, np.int32)
        idx = self.lib.orc_cell_of(np.ascontiguousarray(q, np.float32), G, qc, t, ic)
        return int(idx), qc, t, ic

    def circle_cells(self, x3, y3, G: int, J: int):
        cells = np.empty(J, np.int32)
        ok = self.lib.orc_circle_cells(np.ascontiguousarray(x3, np.float32),
                                       np.ascontiguousarray(y3, np.float32), G, J, cells)
        return cells if ok else None

    def histogram(self, x, y, G: int, J: int, nthreads: int = 1):
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        n = x.shape[1]
        hist = np.empty(G * G * G, np.int32)
        self.lib.orc_histogram(x, y, n, G, J, hist, nthreads)
        return hist

    def topk(self, hist, G: int, K: int):
        counts = np.zeros(K, np.int32)
        idx = np.zeros(K, np.int32)
        m = self.lib.orc_topk(np.ascontiguousarray(hist, np.int32), G, K, counts, idx)
        return counts[:m].copy(), idx[:m].copy()

    def decode(self, idx: int, G: int):
        q = np.empty(4, np.float32)
        self.lib.orc_decode(int(idx), G, q)
        return q

    def residual(self, x3, y3, q):
        return float(self.lib.orc_residual(np.ascontiguousarray(x3, np.float32),
                                           np.ascontiguousarray(y3, np.float32),
                                           np.ascontiguousarray(q, np.float32)))

    def rescore(self, x, y, q, T2, want_mask: bool = False):
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        n = x.shape[1]
        mask = np.zeros(n, np.uint8) if want_mask else None
        c = self.lib.orc_rescore(x, y, n, np.ascontiguousarray(q, np.float32),
                                 float(np.float32(T2)),
                                 mask.ctypes.data_as(ct.c_void_p) if want_mask else None)
        return (int(c), mask) if want_mask else int(c)

    def solve(self, x, y, G: int, J: int, eps_rad: float, K: int, nthreads: int = 1):
        """Whole solve; returns a dict with every intermediate."""
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        n = x.shape[1]
        hist = np.empty(G * G * G, np.int32)
        tc = np.zeros(max(K, 1), np.int32)
        ti = np.zeros(max(K, 1), np.int32)
        cc = np.zeros(max(K, 1), np.int64)
        q = np.empty(4, np.float32)
        cnt = ct.c_int64()
        win = ct.c_int32()
        mask = np.zeros(max(n, 1), np.uint8)
        m = self.lib.orc_solve(x, y, n, G, J, float(np.float32(eps_rad)), K, nthreads, hist,
                               tc, ti, cc, q, ct.byref(cnt), ct.byref(win),
                               mask.ctypes.data_as(ct.c_void_p))
        return dict(hist=hist, top_counts=tc[:m].copy(), top_idx=ti[:m].copy(),
                    cand_counts=cc[:m].copy(), q=q, count=int(cnt.value),
                    winner=int(win.value), mask=mask[:n].astype(bool))


_default = None


def get() -> Oracle:
    """The oracle built from ``rotvote_oracle.c`` (built on first use)."""
    global _default
    if _default is None:
        _default = Oracle(LIB)
    return _default


def threads() -> int:
    """Threads the oracle may use here (affinity-aware)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)
