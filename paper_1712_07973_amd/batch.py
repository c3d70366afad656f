"""Batches of independent systems (exx_batch_* of the C ABI)."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .api import MODES, PRECISIONS, Grid, _check_tensor, _stream_ptr


class Batch:
    """Evaluates many systems (mixed grids and orbital counts) per call.

    With ``use_graph`` the first call captures the whole evaluation into a HIP
    graph and later calls with the same tensors replay it.  With
    ``complex_orbitals`` every system's psi is complex128.  The two spin
    channels of a spin-polarized system are a batch of two systems.  With
    ``merge`` (FP32) systems on one grid share their launches (EXX_BATCH_MERGE:
    "kpsi" and "energy_kpsi" modes).
    """

    def __init__(self, grids: list[Grid], n_orb: list[int], precision: str = "fp32",
                 use_graph: bool = True, device: torch.device | None = None,
                 complex_orbitals: bool = False, merge: bool = False):
        if len(grids) != len(n_orb) or not grids:
            raise ValueError("grids and n_orb must be non-empty lists of equal length")
        self.grids = list(grids)
        self.n_orb = [int(x) for x in n_orb]
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.dtype = torch.complex128 if complex_orbitals else torch.float64
        flags = ((L.BATCH_GRAPH if use_graph else 0) | (L.BATCH_COMPLEX if complex_orbitals else 0)
                 | (L.BATCH_MERGE if merge else 0))
        arr = (L.ExxGrid * len(grids))(*[g.to_c() for g in grids])
        na = (C.c_int * len(grids))(*self.n_orb)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().exx_batch_create(C.byref(h), arr, na, len(grids),
                                             PRECISIONS[precision], flags),
                    "exx_batch_create")
        self._h = h
        size = C.c_size_t()
        L.check(L.lib().exx_batch_workspace_bytes(h, C.byref(size)), "exx_batch_workspace_bytes")
        self.ws = torch.empty(max(int(size.value), 256), dtype=torch.uint8, device=self.device)
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.lib().exx_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def _systems(self, psis, occs, outputs, m):
        S = len(self.grids)
        sysarr = (L.ExxSystem * S)()
        for s in range(S):
            n = self.grids[s].n
            _check_tensor("psi", psis[s], (self.n_orb[s], n, n, n), self.device, self.dtype)
            _check_tensor("occ", occs[s], (self.n_orb[s],), self.device)
            ex, kp = outputs[s]
            sysarr[s].psi = psis[s].data_ptr()
            sysarr[s].occ = occs[s].data_ptr()
            sysarr[s].ex_out = ex.data_ptr() if (m & L.MODE_ENERGY) else None
            sysarr[s].kpsi = kp.data_ptr() if kp is not None else None
            sysarr[s].pair_e = None
        return sysarr

    def autotune(self, psis, occs, budget_ms: int = 20000, cache_path: str | None = None) -> list:
        """exx_batch_autotune: picks the tuning per grid class on the given inputs
        (K psi buffers of the right shape serve as scratch); returns the tunings."""
        outputs = [(torch.empty((), dtype=torch.float64, device=self.device), torch.empty_like(p))
                   for p in psis]
        sysarr = self._systems(psis, occs, outputs, L.MODE_ENERGY_KPSI)
        with torch.cuda.device(self.device):
            rc = L.lib().exx_batch_autotune(self._h, sysarr, self.ws.data_ptr(), self.ws.numel(),
                                            _stream_ptr(self.device), int(budget_ms),
                                            cache_path.encode() if cache_path else None)
        L.check(rc, "exx_batch_autotune")
        return self.tunings()

    def tunings(self) -> list:
        """The tuning of every system's plan."""
        out = []
        for s in range(len(self.grids)):
            t = L.ExxTuning()
            L.check(L.lib().exx_batch_get_tuning(self._h, s, C.byref(t)), "exx_batch_get_tuning")
            out.append({"tile": t.tile, "batch_slots": t.batch_slots, "slab_threads": t.slab_threads,
                        "streams": t.streams, "slab_form": t.slab_form})
        return out

    def compute(self, psis, occs, mode: str = "energy_kpsi", outputs=None):
        """psis/occs: lists of device tensors; returns a list of (E_x, K psi) per system.

        ``outputs`` (optional) reuses [(ex, kpsi), ...] tensors, which keeps the
        captured graph valid across calls.
        """
        m = MODES[mode]
        S = len(self.grids)
        if outputs is None:
            outputs = []
            for s in range(S):
                ex = torch.empty((), dtype=torch.float64, device=self.device)
                kp = torch.empty_like(psis[s]) if m & L.MODE_KPSI else None
                outputs.append((ex, kp))
        sysarr = self._systems(psis, occs, outputs, m)
        with torch.cuda.device(self.device):
            rc = L.lib().exx_batch_compute(self._h, sysarr, m, 0, self.ws.data_ptr(), self.ws.numel(),
                                           _stream_ptr(self.device))
        L.check(rc, "exx_batch_compute")
        self._keep = (psis, occs, outputs)
        return outputs
