"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no lattice Boltzmann arithmetic: it produces solid masks,
velocity fields and request parameters only.  The equilibrium PDFs that
follow from a velocity field are computed by each side on its own.

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014),
which is counter based: draw k (k = 0, 1, ...) of a stream seeded with s is
mix(s + (k + 1) * gamma) with gamma = 0x9E3779B97F4A7C15, so long streams
vectorise in numpy.  ``spheres.c`` holds the same generator for the sphere
packs.

Workloads (all periodic unless stated):
  * channel: cells z = 0 and z = nz-1 are solid walls, periodic in x and y;
  * sphere pack: overlapping spheres of radius r added until the porosity
    reaches a target (stands in for the packed bed of spheres the paper
    benchmarks, whose geometry file is not available);
  * velocity noise: u_a = (2U - 1) * amplitude per cell and component, cells
    in lexicographic order (x fastest), components in the order x, y, z.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spheres.c")
_LIB_PATH = os.path.join(_HERE, "libspheres.so")
_lib = None

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.sm_next.argtypes = [u64p]
        lib.sm_next.restype = ctypes.c_uint64
        lib.sm_fill.argtypes = [u64p, u64p, ctypes.c_long]
        lib.sphere_pack.argtypes = [ctypes.POINTER(ctypes.c_uint8), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_double, u64p, ctypes.c_long,
                                    ctypes.POINTER(ctypes.c_long)]
        lib.sphere_pack.restype = ctypes.c_long
        _lib = lib
    return _lib


def _mix(z):
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Draws start .. start+n-1 of the SplitMix64 stream seeded with `seed` (uint64[n])."""
    k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GAMMA
    return _mix(state)


def uniform01(seed: int, n: int, start: int = 0) -> np.ndarray:
    """U = (draw >> 11) * 2^-53, in [0, 1)."""
    return (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class SplitMix64:
    """Sequential SplitMix64 stream (host-side sampling of small parameter sets)."""

    def __init__(self, seed: int):
        self.state = ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)

    def next(self) -> int:
        return int(_load().sm_next(ctypes.byref(self.state)))

    def uniform(self) -> float:
        return (self.next() >> 11) * (2.0 ** -53)


def channel_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """uint8[nz, ny, nx]: solid wall planes z = 0 and z = nz-1."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[0] = 1
    m[nz - 1] = 1
    return m


def velocity_noise(shape, amplitude: float = 1e-3, seed: int = 1) -> np.ndarray:
    """float64[3, nz, ny, nx] with u_a = (2U - 1) * amplitude, draws ordered cell-major then x, y, z."""
    nz, ny, nx = shape
    n = nx * ny * nz
    U = uniform01(seed, 3 * n).reshape(n, 3)
    u = (2.0 * U - 1.0) * amplitude
    return np.ascontiguousarray(u.T.reshape(3, nz, ny, nx))


def rho_u_field(shape, u=None) -> np.ndarray:
    """float64[4, nz, ny, nx]: rho = 1 and the given velocity (zeros if None)."""
    out = np.zeros((4,) + tuple(shape))
    out[0] = 1.0
    if u is not None:
        out[1:] = u
    return out


def sphere_pack(n, radius: int, porosity: float, seed: int, max_spheres: int = 1 << 40, rng=None):
    """Periodic sphere pack in an (nx, ny, nz) box (or an n^3 box for an int n).

    Returns (mask uint8[nz, ny, nx], number of spheres).  Pass `rng` (a
    SplitMix64) to continue an existing stream instead of seeding a new one.
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    lib = _load()
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    state = rng.state if rng is not None else ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)
    ns = ctypes.c_long(0)
    count = lib.sphere_pack(mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), nx, ny, nz, int(radius),
                            float(porosity), ctypes.byref(state), int(max_spheres), ctypes.byref(ns))
    assert int(ns.value) == int(mask.sum(dtype=np.int64))
    return mask, int(count)


def sphere_pack_reference(n, radius: int, porosity: float, seed: int):
    """Slow pure-Python pack from the minimum-image definition (tiny boxes only)."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    st = SplitMix64(seed)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    ncell = nx * ny * nz
    count = 0
    while (ncell - int(mask.sum())) / ncell > porosity:
        cx = (st.next() >> 32) % nx
        cy = (st.next() >> 32) % ny
        cz = (st.next() >> 32) % nz
        for z in range(nz):
            dz = min(abs(z - cz), nz - abs(z - cz))
            for y in range(ny):
                dy = min(abs(y - cy), ny - abs(y - cy))
                for x in range(nx):
                    dx = min(abs(x - cx), nx - abs(x - cx))
                    if dx * dx + dy * dy + dz * dz <= radius * radius:
                        mask[z, y, x] = 1
        count += 1
    return mask, count


def serving_request(seed: int):
    """Parameters of one porous permeability solve, drawn from SplitMix64(seed).

    Returns dict(edge, radius, porosity, rng) where rng continues the same
    stream for the sphere centres: edge = 32 + 16 * (draw mod 11),
    radius = 3 + (draw mod 8), porosity = 0.3 + 0.5 * U.
    """
    st = SplitMix64(seed)
    edge = 32 + 16 * ((st.next() >> 32) % 11)
    radius = 3 + ((st.next() >> 32) % 8)
    porosity = 0.3 + 0.5 * st.uniform()
    return {"edge": int(edge), "radius": int(radius), "porosity": float(porosity), "rng": st}


def serving_geometry(seed: int):
    """(mask, params) of serving request `seed`."""
    p = serving_request(seed)
    mask, count = sphere_pack(p["edge"], p["radius"], p["porosity"], seed=0, rng=p["rng"])
    p = dict(p)
    p.pop("rng")
    p["spheres"] = count
    return mask, p
