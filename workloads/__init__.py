"""Seeded synthetic workloads: occupancy scenes (ascending Morton codes) and ray arrays.

Inputs only. Nothing here intersects a ray with a volume; the CPU oracle and the GPU
library both consume these arrays and share no code with this module or each other.

Ray layout (32 B): float32 [ox, oy, oz, tmin, dx, dy, dz, tmax], grid units.
Hit layout (16 B): int32 [x, y, z] + float32 t (a miss is x = y = z = -1, t = +inf).

Scene recipes (all seeded; see the module docstring of gen.cpp):
  * ``solid_noise``  solid spheres OR i.i.d. Bernoulli noise (the small 64^3 case)
  * ``shell``        1-voxel shell of a union of spheres and tori (surface volumes)
  * ``bernoulli``    i.i.d. occupancy on a possibly non-cubic grid (tiny test volumes)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libhvfgen.so")
_SRC = os.path.join(_HERE, "gen.cpp")

RAY_DTYPE = np.float32
RAY_FIELDS = 8
HIT_FIELDS = 4


def build(force: bool = False) -> str:
    """Compile gen.cpp into libhvfgen.so (plain g++, no fast-math, no contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                               "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        u64, i64, i32, dbl, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.wl_morton_encode.restype = u64
        L.wl_morton_encode.argtypes = [ctypes.c_uint32] * 3
        L.wl_morton_encode_many.argtypes = [vp, i64, vp]
        L.wl_morton_decode_many.argtypes = [vp, i64, vp]
        L.wl_rng_u64.restype = u64
        L.wl_rng_u64.argtypes = [u64, u64, u64]
        L.wl_result_size.restype = i64
        L.wl_result_size.argtypes = [vp]
        L.wl_result_copy.argtypes = [vp, vp]
        L.wl_result_free.argtypes = [vp]
        L.wl_scene_shell.restype = vp
        L.wl_scene_shell.argtypes = [u64, i32, i32, i32, dbl, i32]
        L.wl_scene_solid_noise.restype = vp
        L.wl_scene_solid_noise.argtypes = [u64, i32, i32, dbl, dbl, dbl]
        L.wl_scene_bernoulli.restype = vp
        L.wl_scene_bernoulli.argtypes = [u64, i32, i32, i32, dbl]
        L.wl_camera_rays.argtypes = [u64, u64, i32, i32, i32, i32, i32, dbl, dbl, dbl, vp]
        L.wl_random_rays.argtypes = [u64, i32, i32, i32, i64, vp]
        L.wl_bounce_rays.restype = i64
        L.wl_bounce_rays.argtypes = [u64, vp, vp, i64, vp, vp]
        _lib = L
    return _lib


def _take(h) -> np.ndarray:
    L = lib()
    n = L.wl_result_size(h)
    out = np.empty(n, dtype=np.uint64)
    if n:
        L.wl_result_copy(h, out.ctypes.data)
    L.wl_result_free(h)
    return out


def _ptr(a: np.ndarray):
    return a.ctypes.data


# --------------------------------------------------------------------------- Morton codes
def morton_encode(xyz: np.ndarray) -> np.ndarray:
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    out = np.empty(len(xyz), dtype=np.uint64)
    lib().wl_morton_encode_many(_ptr(xyz), len(xyz), _ptr(out))
    return out


def morton_decode(codes: np.ndarray) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    out = np.empty((len(codes), 3), dtype=np.int32)
    lib().wl_morton_decode_many(_ptr(codes), len(codes), _ptr(out))
    return out


# --------------------------------------------------------------------------- scenes
def scene_shell(seed: int, log2n: int, n_sph: int, n_tor: int, scale: float = 1.0,
                nthreads: int | None = None) -> np.ndarray:
    """1-voxel shell of a seeded union of spheres and tori in a 2^log2n cube.

    Sphere centres U[0.15N, 0.85N]^3, radii U[0.04, 0.12]*N*scale; torus major radius
    U[0.05, 0.12]*N*scale, minor U[0.01, 0.03]*N*scale, axis uniform on the sphere.
    A voxel is occupied iff the union SDF at its centre is <= 0 and some 6-neighbour
    centre has SDF > 0.
    """
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    return _take(lib().wl_scene_shell(seed, log2n, n_sph, n_tor, float(scale), int(nthreads)))


def scene_solid_noise(seed: int, log2n: int = 6, n_sph: int = 8, rmin: float = 4.0, rmax: float = 16.0,
                      noise: float = 0.05) -> np.ndarray:
    """Solid union of n_sph spheres (centres U[N/4, 3N/4]^3, radii U[rmin, rmax]*N/64)
    OR-ed with i.i.d. Bernoulli(noise) voxels."""
    return _take(lib().wl_scene_solid_noise(seed, log2n, n_sph, rmin, rmax, noise))


def scene_bernoulli(seed: int, ex: int, ey: int, ez: int, p: float) -> np.ndarray:
    return _take(lib().wl_scene_bernoulli(seed, ex, ey, ez, float(p)))


# --------------------------------------------------------------------------- rays
def camera_rays(seed: int, view: int, extent, width: int, height: int, fov_deg: float = 50.0,
                rmin: float = 1.2, rmax: float = 2.0) -> np.ndarray:
    nx, ny, nz = extent
    out = np.empty((height * width, RAY_FIELDS), dtype=RAY_DTYPE)
    lib().wl_camera_rays(seed, view, nx, ny, nz, width, height, float(fov_deg), float(rmin), float(rmax),
                         _ptr(out))
    return out


def random_rays(seed: int, extent, n: int) -> np.ndarray:
    nx, ny, nz = extent
    out = np.empty((n, RAY_FIELDS), dtype=RAY_DTYPE)
    lib().wl_random_rays(seed, nx, ny, nz, n, _ptr(out))
    return out


def bounce_rays(seed: int, rays: np.ndarray, hits: np.ndarray):
    """One cosine-weighted bounce per primary hit. Returns (rays, source_index)."""
    rays = np.ascontiguousarray(rays, dtype=np.float32)
    hits = np.ascontiguousarray(hits)
    assert hits.dtype.itemsize == 4 and hits.shape == (len(rays), 4)
    out = np.empty_like(rays)
    src = np.empty(len(rays), dtype=np.int64)
    m = lib().wl_bounce_rays(seed, _ptr(rays), _ptr(hits), len(rays), _ptr(out), _ptr(src))
    return out[:m].copy(), src[:m].copy()


def hits_view(hits_i32: np.ndarray):
    """Split an int32 [n, 4] hit array into (xyz int32 [n, 3], t float32 [n])."""
    h = np.ascontiguousarray(hits_i32)
    return h[:, :3], h[:, 3].view(np.float32)
