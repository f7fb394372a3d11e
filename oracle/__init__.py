"""CPU oracle for ray intersection through hybrid voxel formats.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library. It builds formats in the paper's
own word layout (Sec. 3.3) with its own parser and builder (Sec. 4.1), traces them with
a plain recursive per-level tracer (Sec. 4.2), and offers two independent companions
(a flat DDA on a dense grid and a brute-force scan of every occupied voxel).

Every function's numerics: fp32, correctly rounded reciprocal, plane time
T(p) = (float(p) - o) * inv, fixed-form min/max, half-open visit intervals. See the
header of oracle.cpp for the full statement and the paper sections each part follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")


def build(force: bool = False) -> str:
    """Compile oracle.cpp (g++ -O2 -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_parse.restype = i32
        L.orc_parse.argtypes = [ctypes.c_char_p, vp]
        L.orc_build.restype = vp
        L.orc_build.argtypes = [ctypes.c_char_p, vp, i64]
        L.orc_free.argtypes = [vp]
        L.orc_num_words.restype = i64
        L.orc_num_words.argtypes = [vp]
        L.orc_copy_words.argtypes = [vp, vp]
        L.orc_split_buffers.restype = i32
        L.orc_split_buffers.argtypes = [vp]
        L.orc_num_levels.restype = i32
        L.orc_num_levels.argtypes = [vp]
        L.orc_node_counts.argtypes = [vp, vp]
        L.orc_trace.argtypes = [vp, vp, i64, vp, i32]
        L.orc_decode.restype = i64
        L.orc_decode.argtypes = [vp, vp, i64]
        L.orc_flat_dda.argtypes = [vp, vp, vp, i64, vp]
        L.orc_brute.argtypes = [vp, i64, vp, vp, i64, vp, vp]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def parse(spec: str):
    """Return (number of levels, per-axis log2 extents) or raise OracleError."""
    ext = np.zeros(3, dtype=np.int32)
    n = lib().orc_parse(spec.encode(), ext.ctypes.data)
    if n < 0:
        raise OracleError(lib().orc_last_error().decode())
    return n, tuple(int(e) for e in ext)


def _rays(rays):
    r = np.ascontiguousarray(rays, dtype=np.float32)
    assert r.ndim == 2 and r.shape[1] == 8
    return r


class Volume:
    """A hybrid format built in the paper's layout."""

    def __init__(self, spec: str, codes: np.ndarray):
        codes = np.ascontiguousarray(codes, dtype=np.uint64)
        self.spec = spec
        self.levels, self.ext = parse(spec)
        self._codes = codes
        h = lib().orc_build(spec.encode(), codes.ctypes.data, len(codes))
        if not h:
            raise OracleError(lib().orc_last_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    @property
    def num_words(self) -> int:
        return int(lib().orc_num_words(self._h))

    def split_buffers(self) -> bool:
        """One buffer per level (--depth-buffers, or past 2^32 words)."""
        return bool(lib().orc_split_buffers(self._h))

    def words(self) -> np.ndarray:
        out = np.empty(self.num_words, dtype=np.uint32)
        lib().orc_copy_words(self._h, out.ctypes.data)
        return out

    def node_counts(self) -> np.ndarray:
        out = np.zeros(self.levels, dtype=np.int64)
        lib().orc_node_counts(self._h, out.ctypes.data)
        return out

    def decode(self) -> np.ndarray:
        n = lib().orc_decode(self._h, None, 0)
        out = np.empty(n, dtype=np.uint64)
        lib().orc_decode(self._h, out.ctypes.data, n)
        return out

    def trace(self, rays, nthreads: int = 1) -> np.ndarray:
        """int32 [n, 4] hits: x, y, z and the float32 bits of t (miss: -1,-1,-1,+inf)."""
        r = _rays(rays)
        hits = np.empty((len(r), 4), dtype=np.int32)
        lib().orc_trace(self._h, r.ctypes.data, len(r), hits.ctypes.data, int(nthreads))
        return hits


def flat_dda(occ_dense: np.ndarray, ext, rays) -> np.ndarray:
    """First hit on a dense grid: occ_dense[z, y, x] (uint8/bool) of extents 2^ext."""
    occ = np.ascontiguousarray(occ_dense, dtype=np.uint8)
    ex = np.asarray(ext, dtype=np.int32)
    assert occ.size == 1 << int(ex.sum())
    r = _rays(rays)
    hits = np.empty((len(r), 4), dtype=np.int32)
    lib().orc_flat_dda(occ.ctypes.data, ex.ctypes.data, r.ctypes.data, len(r), hits.ctypes.data)
    return hits


def brute(codes: np.ndarray, ext, rays, return_ties: bool = False):
    """The plain definition over every occupied voxel (tiny volumes only)."""
    c = np.ascontiguousarray(codes, dtype=np.uint64)
    ex = np.asarray(ext, dtype=np.int32)
    r = _rays(rays)
    hits = np.empty((len(r), 4), dtype=np.int32)
    ties = np.zeros(len(r), dtype=np.int32)
    lib().orc_brute(c.ctypes.data, len(c), ex.ctypes.data, r.ctypes.data, len(r), hits.ctypes.data,
                    ties.ctypes.data)
    return (hits, ties) if return_ties else hits
