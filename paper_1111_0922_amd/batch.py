"""Python binding of the batch executor (lbm_batch_*): marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .grid import _ptr, _stream


class Batch:
    """Up to `max_slots` indirect AA lattices advanced together by one batched kernel."""

    MODES = {"launches": 0, "graph": 1, "cooperative": 2}

    def __init__(self, max_slots: int, max_tiles: int, precision: str = "f32", use_graph: bool = True,
                 device=None, mode: str | None = None):
        """mode: 'graph' (default with use_graph), 'launches', or 'cooperative' (one launch per run)."""
        self.lib = L.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        nbytes = ctypes.c_int64(0)
        L.check(self.lib.lbm_batch_workspace_bytes(int(max_slots), int(max_tiles), ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        L.check(self.lib.lbm_batch_create(int(max_slots), int(max_tiles), L.PRECISIONS[precision],
                                          _ptr(self.workspace), ctypes.byref(self._h)))
        self.max_slots = int(max_slots)
        self.mode = self.MODES[mode if mode is not None else ("graph" if use_graph else "launches")]
        self.moments_host = torch.zeros((self.max_slots, 4), dtype=torch.float64, pin_memory=True)
        self.grids = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.lbm_batch_destroy(h)
            self._h = None

    def add(self, grid) -> int:
        slot = ctypes.c_int32(-1)
        L.check(self.lib.lbm_batch_add(self._h, grid._h, ctypes.byref(slot)))
        self.grids[int(slot.value)] = grid
        return int(slot.value)

    def remove(self, slot: int):
        L.check(self.lib.lbm_batch_remove(self._h, int(slot)))
        self.grids.pop(int(slot), None)

    def run_async(self, k_steps: int):
        """Enqueue k_steps for every slot plus the per-slot moments (copied to `moments_host`)."""
        L.check(self.lib.lbm_batch_run(self._h, int(k_steps), ctypes.c_void_p(self.moments_host.data_ptr()),
                                       self.mode, _stream(self.device)))

    def sync(self) -> np.ndarray:
        """Waits for the batch's work on the current stream; returns int32[max_slots], 1 for each slot
        of the last run whose moments are not finite (a diverged lattice), else 0."""
        status = np.zeros(self.max_slots, dtype=np.int32)
        rc = self.lib.lbm_batch_sync(self._h, ctypes.c_void_p(status.ctypes.data), _stream(self.device))
        if rc not in (L.LBM_OK, L.LBM_E_DIVERGED):
            L.check(rc)
        return status

    def run(self, k_steps: int) -> np.ndarray:
        """k_steps for every slot; returns float64[max_slots, 4] moments after synchronising
        (rows of diverged slots are not finite; see sync())."""
        self.run_async(k_steps)
        self.last_status = self.sync()
        return self.moments_host.numpy().copy()
