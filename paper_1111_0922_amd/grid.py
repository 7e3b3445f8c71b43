"""Python binding of the C ABI: argument marshalling only.

torch owns every device buffer (allocated here with the sizes the library
reports) and supplies the stream; every step of the node update runs in the
HIP kernels of liblbm355.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def lattice():
    """(c[19,3], w[19], opp[19]) as the library holds them (no GPU needed)."""
    lib = L.load()
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    o = np.zeros(19, dtype=np.int32)
    L.check(lib.lbm_lattice(c.ctypes.data, w.ctypes.data, o.ctypes.data))
    return c.reshape(19, 3), w, o


def model_bytes(scheme, addressing="direct", precision="f64", model="gpu"):
    """Bytes per lattice-node update of the transfer model: 'paper' (Tables 1-6), 'gpu' (this library
    with IDX) or 'gpu_rank' (neighbour ids looked up by rank)."""
    lib = L.load()
    return lib.lbm_model_bytes(L.SCHEMES[scheme], L.ADDRESSING[addressing], L.PRECISIONS[precision],
                               {"paper": 0, "gpu": 1, "gpu_rank": 2}[model])


def stream_copy(src: torch.Tensor, dst: torch.Tensor, nbytes: int | None = None):
    lib = L.load()
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    L.check(lib.lbm_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(src.device)))


def _alloc(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Grid:
    """One lattice on one GPU: geometry, index, bound buffers of one scheme."""

    def __init__(self, nx, ny, nz, *, addressing="direct", layout="soa", precision="f64", wall_z=False,
                 et_ghosts=False, omega=1.0, g=(0.0, 0.0, 0.0), f16_scale=1.0, brick=None, trt_lambda=3.0 / 16.0, device=None):
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        d = L.GridDesc()
        d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
        d.addressing = L.ADDRESSING[addressing]
        d.layout = L.LAYOUTS[layout]
        d.precision = L.PRECISIONS[precision]
        d.wall_z = int(bool(wall_z))
        d.et_ghosts = int(bool(et_ghosts))
        d.omega = float(omega)
        for k in range(3):
            d.g[k] = float(g[k])
        d.f16_scale = float(f16_scale)
        for k in range(3):
            d.brick[k] = int(brick[k]) if brick is not None else 0
        d.trt_lambda = float(trt_lambda)
        self.desc = d
        self.shape = (int(nz), int(ny), int(nx))
        self.addressing, self.layout, self.precision = addressing, layout, precision
        self._h = ctypes.c_void_p()
        L.check(self.lib.lbm_create_grid(ctypes.byref(d), ctypes.byref(self._h)))
        self.scheme = None
        self.buffers = {}
        self.cellmap = None
        self.idx = None
        self.et = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.lbm_destroy_grid(h)
            self._h = None

    # ---------------------------------------------------------- queries
    def sizes(self, scheme="aa") -> L.Sizes:
        s = L.Sizes()
        L.check(self.lib.lbm_query_sizes(self._h, L.SCHEMES[scheme], ctypes.byref(s)))
        return s

    @property
    def n_nodes(self) -> int:
        return int(self.sizes("aa").n_nodes)

    @property
    def t(self) -> int:
        return int(self.lib.lbm_time(self._h))

    def set_params(self, omega, g):
        arr = (ctypes.c_double * 3)(*[float(v) for v in g])
        L.check(self.lib.lbm_set_params(self._h, float(omega), arr))

    def set_boundary(self, cls: int, kind: str, rho: float = 1.0, u=(0.0, 0.0, 0.0)):
        """Open boundary class `cls` (mask value cls + 1): 'wall', 'velocity' (moving wall) or 'pressure'."""
        arr = (ctypes.c_double * 3)(*[float(v) for v in u])
        L.check(self.lib.lbm_set_boundary(self._h, int(cls), L.BC_KINDS[kind], float(rho), arr))

    @property
    def rank_lookup(self) -> bool:
        """Whether the bound grid's neighbour-reading kernels look ids up by rank (LBM_OPT_RANK_LOOKUP)."""
        rc = self.lib.lbm_rank_lookup_active(self._h)
        L.check(min(rc, 0))
        return bool(rc & 1)

    @property
    def lattice_block(self) -> int:
        """Nodes per block of the bound SoA lattices (LBM_OPT_SOA_BLOCK), 0 for plain SoA or AoS."""
        rc = self.lib.lbm_lattice_block(self._h)
        L.check(min(rc, 0))
        return rc

    @property
    def et_rank_lookup(self) -> bool:
        """Whether the esoteric twist takes its storage addresses from the rank words."""
        rc = self.lib.lbm_rank_lookup_active(self._h)
        L.check(min(rc, 0))
        return bool(rc & 2)

    def set_option(self, option, value):
        L.check(self.lib.lbm_set_option(self._h, int(option), int(value)))

    def set_block_order(self, order: torch.Tensor | None):
        """Indirect grids: workgroup b of the update kernels takes node block order[b] (int32/uint32
        device tensor, a permutation of the ceil(N_f / 256) blocks), or the natural order for None."""
        if order is None:
            L.check(self.lib.lbm_set_block_order(self._h, None, 0))
            self._order = None
            return
        assert order.dtype in (torch.int32,) and order.is_contiguous() and order.device.type == "cuda"
        self._order = order   # the library keeps the pointer
        L.check(self.lib.lbm_set_block_order(self._h, _ptr(order), order.numel()))

    # ---------------------------------------------------------- setup
    def build_idx(self, mask: torch.Tensor) -> int:
        """Indirect grids: cellmap, IDX (and the ET table) from a uint8 solid mask [nz, ny, nx]."""
        assert mask.dtype == torch.uint8 and tuple(mask.shape) == self.shape and mask.is_contiguous()
        mask = mask.to(self.device)
        s0 = self.sizes()
        self.cellmap = _alloc(s0.cellmap_bytes, self.device).view(torch.int32)
        scratch = _alloc(s0.build_scratch_bytes, self.device)
        nf = ctypes.c_int64(0)
        st = _stream(self.device)
        L.check(self.lib.lbm_build_idx(self._h, _ptr(mask), _ptr(self.cellmap), None, None, _ptr(scratch),
                                       ctypes.byref(nf), st))
        s1 = self.sizes("et" if self.desc.et_ghosts else "aa")
        self.idx = _alloc(s1.idx_bytes, self.device).view(torch.int32)
        self.et = _alloc(s1.aux_bytes, self.device).view(torch.int32) if self.desc.et_ghosts else None
        L.check(self.lib.lbm_build_idx(self._h, _ptr(mask), _ptr(self.cellmap), _ptr(self.idx), _ptr(self.et),
                                       _ptr(scratch), ctypes.byref(nf), st))
        self._mask = mask
        return int(nf.value)

    def bind(self, scheme: str):
        s = self.sizes(scheme)
        b = {"pdf0": _alloc(s.pdf_bytes, self.device),
             "pdf1": _alloc(s.pdf1_bytes, self.device) if s.pdf1_bytes else None,
             "scratch": _alloc(s.scratch_bytes, self.device)}
        self.buffers = b
        L.check(self.lib.lbm_bind(self._h, L.SCHEMES[scheme], _ptr(b["pdf0"]), _ptr(b["pdf1"]), _ptr(self.idx),
                                  _ptr(self.et) if scheme == "et" else None, _ptr(b["scratch"])))
        self.scheme = scheme
        return self

    # ---------------------------------------------------------- state
    def set_pdfs(self, canon: torch.Tensor):
        canon = canon.to(self.device, torch.float64).contiguous()
        assert canon.shape == (19, self.n_nodes)
        self._keep = canon  # alive until the asynchronous upload has run
        L.check(self.lib.lbm_set_pdfs(self._h, _ptr(canon), _stream(self.device)))

    def get_pdfs(self) -> torch.Tensor:
        out = torch.empty((19, self.n_nodes), dtype=torch.float64, device=self.device)
        L.check(self.lib.lbm_get_pdfs(self._h, _ptr(out), _stream(self.device)))
        return out

    def init_equilibrium(self, rho_u: torch.Tensor | None = None):
        if rho_u is not None:
            rho_u = rho_u.to(self.device, torch.float64).contiguous()
            assert rho_u.shape == (4, self.n_nodes)
            self._keep = rho_u
        L.check(self.lib.lbm_init_equilibrium(self._h, _ptr(rho_u), _stream(self.device)))

    def step(self, n: int = 1, collider: str = "bgk"):
        L.check(self.lib.lbm_step(self._h, L.SCHEMES[self.scheme], L.COLLIDERS[collider], int(n),
                                  _stream(self.device)))

    def moments(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """Device float64[4] = (M, Jx, Jy, Jz) of the current state (asynchronous)."""
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=self.device)
        L.check(self.lib.lbm_reduce_moments(self._h, _ptr(out), _stream(self.device)))
        return out

    def moments_noalloc(self, out: torch.Tensor) -> torch.Tensor:
        """As moments(), into a caller-given float64[4] device tensor, through the entry point that
        allocates nothing (its partials live in a static device array of the library)."""
        assert out.dtype == torch.float64 and out.numel() >= 4 and out.is_contiguous()
        L.check(self.lib.lbm_reduce_moments_noalloc(self._h, _ptr(out), _stream(self.device)))
        return out
