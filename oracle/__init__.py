"""FP64 CPU oracle of the D3Q19 node update -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product package.

The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, the two-step
two-grid algorithm of Sec. 2 with pull propagation, Sec. 3 / Fig. 1(c)).
This module only marshals numpy arrays into it and adds the host-side
derived quantities (velocity field, permeability) that follow from the
moments by plain definitions.

Array conventions: PDFs are ``float64[19, nz, ny, nx]`` (x fastest, the
lexicographic cell order); the solid mask is ``uint8[nz, ny, nx]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

Q = 19


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP over z-planes)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.ora_tables.argtypes = [ip, dp, ip]
    lib.ora_equilibrium.argtypes = [ctypes.c_double, dp, dp]
    lib.ora_guo_source.argtypes = [ctypes.c_double, dp, ctypes.c_double, dp, dp]
    lib.ora_collide_node.argtypes = [dp, ctypes.c_double, dp, ctypes.c_int, dp]
    lib.ora_round_half.argtypes = [ctypes.c_double]
    lib.ora_round_half.restype = ctypes.c_double
    lib.ora_round_half_array.argtypes = [dp, dp, ctypes.c_long]
    lib.ora_quantize_field.argtypes = [dp, u8p, ip, ctypes.c_int, ctypes.c_double]
    lib.ora_collide.argtypes = [dp, dp, u8p, ip, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.ora_collide_node_trt.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.ora_stream.argtypes = [dp, dp, u8p, ip, ip, dp, ctypes.c_int]
    lib.ora_run_ts.argtypes = [dp, dp, u8p, ip, ip, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int,
                               ctypes.c_int, ctypes.c_double, dp, ctypes.c_long, ctypes.c_int]
    lib.ora_moments.argtypes = [dp, u8p, ip, dp]
    lib.ora_macroscopic.argtypes = [dp, u8p, ip, dp, dp]
    lib.ora_init_equilibrium.argtypes = [dp, u8p, ip, dp]
    lib.ora_build_idx.argtypes = [u8p, ip, ip, i32p, i32p, ctypes.c_long]
    lib.ora_build_idx.restype = ctypes.c_long
    lib.ora_build_idx_brick.argtypes = [u8p, ip, ip, ip, i32p, i32p, ctypes.c_long]
    lib.ora_build_idx_brick.restype = ctypes.c_long
    lib.ora_num_threads.argtypes = [ctypes.c_int]
    lib.ora_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dims(solid):
    nz, ny, nx = solid.shape
    return (ctypes.c_int * 3)(nx, ny, nz)


def _per(periodic):
    return (ctypes.c_int * 3)(*[int(bool(p)) for p in periodic])


def _vec3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


QUANT = {None: 0, "f64": 0, "f32": 1, "f16s": 2, "f32s": 3}
COLLIDER = {"identity": 0, "bgk": 1, "trt": 2}


def tables():
    """(c[19,3] int, w[19] float64, opp[19] int) as the oracle holds them."""
    lib = _load()
    c = np.zeros(57, dtype=np.intc)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.intc)
    lib.ora_tables(_p(c, ctypes.c_int), _p(w, ctypes.c_double), _p(opp, ctypes.c_int))
    return c.reshape(19, 3).astype(np.int64), w, opp.astype(np.int64)


def equilibrium(rho, u):
    lib = _load()
    out = np.zeros(19)
    lib.ora_equilibrium(float(rho), _vec3(u), _p(out, ctypes.c_double))
    return out


def guo_source(rho, u, omega, g):
    lib = _load()
    out = np.zeros(19)
    lib.ora_guo_source(float(rho), _vec3(u), float(omega), _vec3(g), _p(out, ctypes.c_double))
    return out


def collide_node(f, omega, g, collider="bgk", omega_minus=None):
    """One node's collision; collider 'trt' relaxes odd moments with omega_minus."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(19)
    if collider == "trt":
        lib.ora_collide_node_trt(_p(f, ctypes.c_double), float(omega), float(omega_minus), _vec3(g),
                                 _p(out, ctypes.c_double))
    else:
        lib.ora_collide_node(_p(f, ctypes.c_double), float(omega), _vec3(g), COLLIDER[collider],
                             _p(out, ctypes.c_double))
    return out


def trt_omega_minus(omega, lam):
    """w- from w+ = omega and Lambda = (1/w+ - 1/2)(1/w- - 1/2)."""
    return 1.0 / (lam / (1.0 / omega - 0.5) + 0.5)


def round_half(v):
    """Nearest IEEE binary16 value of each element (as float64)."""
    lib = _load()
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(v)
    lib.ora_round_half_array(_p(v, ctypes.c_double), _p(out, ctypes.c_double), v.size)
    return out


def quantize(f, solid, precision, sigma=1.0):
    """Round the stored values of the fluid cells to a storage precision."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    lib.ora_quantize_field(_p(f, ctypes.c_double), _p(solid, ctypes.c_uint8), _dims(solid),
                           QUANT[precision], float(sigma))
    return f


def init_equilibrium(rho_u, solid):
    """f = f^eq(rho, u) per fluid cell; rho_u is float64[4, nz, ny, nx]."""
    lib = _load()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    rho_u = np.ascontiguousarray(rho_u, dtype=np.float64)
    f = np.zeros((19,) + solid.shape)
    lib.ora_init_equilibrium(_p(rho_u, ctypes.c_double), _p(solid, ctypes.c_uint8), _dims(solid),
                             _p(f, ctypes.c_double))
    return f


def collide(f, solid, omega, g, collider="bgk", precision=None, sigma=1.0, threads=0, omega_minus=None):
    """Collision loop alone (post-collision state at the same cells)."""
    lib = _load()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    A = np.ascontiguousarray(f, dtype=np.float64)
    B = np.zeros_like(A)
    lib.ora_collide(_p(A, ctypes.c_double), _p(B, ctypes.c_double), _p(solid, ctypes.c_uint8),
                    _dims(solid), float(omega), float(omega if omega_minus is None else omega_minus), _vec3(g),
                    COLLIDER[collider], QUANT[precision], float(sigma), int(threads))
    return B


BC_KIND = {"wall": 0, "velocity": 1, "pressure": 2}


def _bc_table(bc):
    """Boundary classes {class 1..4: (kind, rho, (ux, uy, uz))} as the flat [4][5] table, or NULL."""
    if not bc:
        return None
    t = np.zeros((4, 5))
    for cls, (kind, rho, u) in bc.items():
        assert 1 <= cls <= 4
        t[cls - 1] = (BC_KIND[kind], rho, u[0], u[1], u[2])
    return t


def stream(fpost, solid, periodic=(1, 1, 1), threads=0, bc=None):
    """Propagation loop alone: pull with half-way bounce-back (and open boundaries, see run_ts)."""
    lib = _load()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    B = np.ascontiguousarray(fpost, dtype=np.float64)
    A = np.zeros_like(B)
    t = _bc_table(bc)
    lib.ora_stream(_p(B, ctypes.c_double), _p(A, ctypes.c_double), _p(solid, ctypes.c_uint8),
                   _dims(solid), _per(periodic), None if t is None else _p(t, ctypes.c_double), int(threads))
    return A


def run_ts(f, solid, steps, omega, g, periodic=(1, 1, 1), collider="bgk", precision=None,
           sigma=1.0, threads=0, omega_minus=None, bc=None):
    """`steps` time steps of the two-step two-grid algorithm; returns f(t+steps).

    collider: 'bgk', 'identity', or 'trt' (odd moments relaxed with omega_minus).
    bc: open boundaries {class: (kind, rho, u)} for mask cells of value class + 1;
    kind 'wall' (bounce-back), 'velocity' (moving wall) or 'pressure' (anti-bounce-back).
    """
    lib = _load()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    A = np.array(f, dtype=np.float64, order="C", copy=True)
    B = np.zeros_like(A)
    t = _bc_table(bc)
    lib.ora_run_ts(_p(A, ctypes.c_double), _p(B, ctypes.c_double), _p(solid, ctypes.c_uint8),
                   _dims(solid), _per(periodic), float(omega), float(omega if omega_minus is None else omega_minus),
                   _vec3(g), COLLIDER[collider], QUANT[precision], float(sigma),
                   None if t is None else _p(t, ctypes.c_double), int(steps), int(threads))
    return A


def moments(f, solid):
    """(M, Jx, Jy, Jz): total mass and raw momentum sum_i c_i f_i over fluid cells."""
    lib = _load()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    A = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(4)
    lib.ora_moments(_p(A, ctypes.c_double), _p(solid, ctypes.c_uint8), _dims(solid), _p(out, ctypes.c_double))
    return out


def macroscopic(f, solid, g):
    """(rho[nz,ny,nx], u[3,nz,ny,nx]) with u = (j + rho g/2)/rho; zeros on solids."""
    lib = _load()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    A = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros((4,) + solid.shape)
    lib.ora_macroscopic(_p(A, ctypes.c_double), _p(solid, ctypes.c_uint8), _dims(solid), _vec3(g),
                        _p(out, ctypes.c_double))
    return out[0], out[1:]


def build_idx(solid, periodic=(1, 1, 1), with_idx=True, brick=None):
    """(cellmap int32[nz,ny,nx], idx int32[18, N_f] or None, N_f).

    brick = (bx, by, bz) numbers the fluid cells brick by brick (bricks in
    lexicographic order, cells inside a brick likewise); None = lexicographic.
    """
    lib = _load()
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    cellmap = np.zeros(solid.shape, dtype=np.int32)
    nf = int((solid == 0).sum())
    idx = np.zeros((18, max(nf, 1)), dtype=np.int32) if with_idx else None
    b = (ctypes.c_int * 3)(*(brick if brick is not None else (0, 0, 0)))
    got = lib.ora_build_idx_brick(_p(solid, ctypes.c_uint8), _dims(solid), _per(periodic), b,
                                  _p(cellmap, ctypes.c_int32),
                                  _p(idx, ctypes.c_int32) if with_idx else None, max(nf, 1))
    assert got == nf
    return cellmap, (idx[:, :nf] if with_idx else None), nf


def node_order(cellmap):
    """Flat cell index of each fluid id (inverse of the cellmap)."""
    flat = cellmap.reshape(-1)
    order = np.empty(int((flat >= 0).sum()), dtype=np.int64)
    order[flat[flat >= 0]] = np.flatnonzero(flat >= 0)
    return order


def ordered_view(f, order):
    """PDFs of the fluid cells in fluid-id order, float64[19, N_f]."""
    return np.ascontiguousarray(f.reshape(19, -1)[:, order])


def num_threads(threads=0):
    return int(_load().ora_num_threads(int(threads)))


def fluid_view(f, solid):
    """PDFs of the fluid cells only, float64[19, N_f] in lexicographic order."""
    return np.ascontiguousarray(f.reshape(19, -1)[:, solid.reshape(-1) == 0])


def mean_velocity(mom, g):
    """Mass-weighted mean velocity U = (J + M g/2) / M from a moments 4-vector."""
    M = mom[0]
    return (np.asarray(mom[1:4]) + 0.5 * M * np.asarray(g, dtype=np.float64)) / M


def permeability(mom, g, omega, porosity):
    """Darcy permeability k = nu * phi * U_x / |g| (lattice units^2), nu = (1/omega - 1/2)/3."""
    nu = (1.0 / omega - 0.5) / 3.0
    U = mean_velocity(mom, g)
    return nu * porosity * U[0] / float(np.linalg.norm(g))
