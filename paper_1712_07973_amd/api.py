"""Python front end of libexx.so.

PyTorch provides device memory (CUDA/HIP tensors) and the current stream;
every step of the exchange evaluation runs in the library's HIP kernels.
Arrays follow the library layout: psi is float64 ``[N, n, n, n]`` (x
fastest) on a GPU -- complex128 for a plan made with ``complex_orbitals`` --
and occ is float64 ``[N]`` on the same GPU.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

PRECISIONS = {"fp32": L.PREC_FP32, "fp64_plain": L.PREC_FP64_PLAIN, "fp64_fused": L.PREC_FP64_FUSED}
MODES = {"energy": L.MODE_ENERGY, "kpsi": L.MODE_KPSI, "energy_kpsi": L.MODE_ENERGY_KPSI}


@dataclass(frozen=True)
class Grid:
    """Cubic grid: n points per axis, spacing h (bohr), boundary 'periodic',
    'free' (isolated), 'surface' (periodic in x and y, isolated along z) or
    'wire' (isolated in x and y, periodic along z).

    R: truncation radius of the isolated directions (None: the box length n h).
    kernel: 'coulomb' (1/r), 'screened' (erfc(omega r)/r, periodic only) or 'isf'
    (the interpolating-scaling-function Green's function, free boundary only).
    """

    n: int
    h: float
    bc: str = "free"
    R: float | None = None
    kernel: str = "coulomb"
    omega: float = 0.0

    def to_c(self) -> L.ExxGrid:
        g = L.ExxGrid()
        g.nx = g.ny = g.nz = int(self.n)
        g.hx = g.hy = g.hz = float(self.h)
        g.bc = {"periodic": L.BC_PERIODIC, "free": L.BC_FREE, "surface": L.BC_SURFACE,
                "wire": L.BC_WIRE}[self.bc]
        g.kernel = {"coulomb": L.KERNEL_COULOMB, "screened": L.KERNEL_SCREENED,
                    "isf": L.KERNEL_ISF}[self.kernel]
        g.R = float(self.R) if self.R else 0.0
        g.omega = float(self.omega)
        return g

    @property
    def h3(self) -> float:
        return float(self.h) ** 3


def _stream_ptr(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _check_tensor(name: str, t: torch.Tensor, shape, device=None, dtype=torch.float64):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on a GPU (the library has no CPU path)")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """An exx_plan for one grid and precision on the current GPU.

    complex_orbitals: psi and K psi are complex128 (rho_ij = conj(psi_j) psi_i).
    """

    def __init__(self, grid: Grid, precision: str = "fp32", n_orb_max: int = 1024,
                 device: torch.device | int | None = None, complex_orbitals: bool = False):
        self.grid = grid
        self.precision = precision
        self.complex_orbitals = bool(complex_orbitals)
        self.dtype = torch.complex128 if self.complex_orbitals else torch.float64
        self.n_orb_max = int(n_orb_max)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   (device if isinstance(device, int) else device.index))
        h = C.c_void_p()
        g = grid.to_c()
        with torch.cuda.device(self.device):
            L.check(L.lib().exx_plan_create(C.byref(h), C.byref(g), PRECISIONS[precision],
                                            self.n_orb_max,
                                            L.PLAN_COMPLEX if self.complex_orbitals else 0),
                    "exx_plan_create")
        self._h = h
        self._ws: torch.Tensor | None = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.lib().exx_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def workspace_bytes(self, n_orb: int) -> int:
        out = C.c_size_t()
        L.check(L.lib().exx_workspace_bytes(self._h, int(n_orb), C.byref(out)),
                "exx_workspace_bytes")
        return int(out.value)

    def prepare(self, n_orb: int) -> None:
        with torch.cuda.device(self.device):
            L.check(L.lib().exx_plan_prepare(self._h, int(n_orb)), "exx_plan_prepare")

    def workspace(self, n_orb: int) -> torch.Tensor:
        need = self.workspace_bytes(n_orb)
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        return self._ws

    def schedule_info(self, n_orb: int):
        a, b = C.c_longlong(), C.c_longlong()
        L.check(L.lib().exx_plan_schedule_info(self._h, int(n_orb), C.byref(a), C.byref(b)),
                "exx_plan_schedule_info")
        return int(a.value), int(b.value)

    @property
    def tuning(self) -> dict:
        t = L.ExxTuning()
        L.check(L.lib().exx_plan_get_tuning(self._h, C.byref(t)), "exx_plan_get_tuning")
        forms = {v: k for k, v in L.SLAB_FORMS.items()}
        return {"tile": t.tile, "batch_slots": t.batch_slots, "slab_threads": t.slab_threads,
                "streams": t.streams, "slab_form": forms.get(t.slab_form, t.slab_form)}

    def set_tuning(self, tile: int = 0, batch_slots: int = 0, slab_threads: int = 0,
                   streams: int = 0, slab_form=0) -> None:
        """0 keeps a field; streams is 1 (serial passes) or 3 (overlapped rounds);
        slab_form is "shared" or "wave" (the y/z pass form, see exx.h)."""
        form = L.SLAB_FORMS[slab_form] if isinstance(slab_form, str) else int(slab_form)
        t = L.ExxTuning(int(tile), int(batch_slots), int(slab_threads), int(streams), form)
        L.check(L.lib().exx_plan_set_tuning(self._h, C.byref(t)), "exx_plan_set_tuning")

    def enable_profiling(self, on: bool = True) -> None:
        L.check(L.lib().exx_plan_enable_profiling(self._h, 1 if on else 0),
                "exx_plan_enable_profiling")

    def read_profile(self) -> dict:
        """{pass kind: (total ms, launches)} since the last read (waits for the events)."""
        t = L.ExxPassTimes()
        L.check(L.lib().exx_plan_read_profile(self._h, C.byref(t)), "exx_plan_read_profile")
        return {k: (t.ms[i], int(t.launches[i])) for i, k in enumerate(L.PASS_KINDS)}

    def compute(self, psi: torch.Tensor, occ: torch.Tensor, mode: str = "energy_kpsi",
                kpsi: torch.Tensor | None = None, pair_e: torch.Tensor | None = None,
                ex_out: torch.Tensor | None = None, accumulate: bool = False,
                workspace: torch.Tensor | None = None):
        """Runs exx_compute on the current stream; returns (ex_out, kpsi, pair_e)."""
        n = self.grid.n
        N = int(psi.shape[0])
        _check_tensor("psi", psi, (N, n, n, n), self.device, self.dtype)
        _check_tensor("occ", occ, (N,), self.device)
        m = MODES[mode]
        if m & L.MODE_ENERGY and ex_out is None:
            ex_out = torch.empty((), dtype=torch.float64, device=self.device)
        if m & L.MODE_KPSI and kpsi is None:
            kpsi = torch.empty_like(psi)
        keep_pe = pair_e is not None
        if m == L.MODE_ENERGY and pair_e is None and bool((occ < 0).any()):
            # the energy-only route folds sqrt(f_i f_j) into the co-densities, which
            # needs f >= 0: with a negative occupation take the pair-energy route
            pair_e = torch.empty((N, N), dtype=torch.float64, device=self.device)
        if kpsi is not None:
            _check_tensor("kpsi", kpsi, (N, n, n, n), self.device, self.dtype)
        if pair_e is not None:
            _check_tensor("pair_e", pair_e, (N, N), self.device)
        ws = workspace if workspace is not None else self.workspace(N)
        flags = L.FLAG_ACCUMULATE if accumulate else 0
        with torch.cuda.device(self.device):
            rc = L.lib().exx_compute(self._h, psi.data_ptr(), occ.data_ptr(), N, m, flags,
                                     _ptr(ex_out), _ptr(kpsi), _ptr(pair_e), ws.data_ptr(),
                                     ws.numel(), _stream_ptr(self.device))
        L.check(rc, "exx_compute")
        return ex_out, kpsi, (pair_e if keep_pe else None)

    def gradient(self, psi: torch.Tensor, occ: torch.Tensor, gbar: torch.Tensor,
                 want_occ: bool = False, workspace: torch.Tensor | None = None):
        """exx_gradient: (gbar dE_x/dpsi, gbar dE_x/df or None), gbar a device scalar."""
        n = self.grid.n
        N = int(psi.shape[0])
        _check_tensor("psi", psi, (N, n, n, n), self.device, self.dtype)
        _check_tensor("occ", occ, (N,), self.device)
        _check_tensor("gbar", gbar, (), self.device)
        grad_psi = torch.empty_like(psi)
        grad_occ = torch.empty((N,), dtype=torch.float64, device=self.device) if want_occ else None
        pe = torch.empty((N, N), dtype=torch.float64, device=self.device) if want_occ else None
        ws = workspace if workspace is not None else self.workspace(N)
        with torch.cuda.device(self.device):
            rc = L.lib().exx_gradient(self._h, psi.data_ptr(), occ.data_ptr(), N, gbar.data_ptr(),
                                      grad_psi.data_ptr(), _ptr(grad_occ), _ptr(pe), ws.data_ptr(),
                                      ws.numel(), _stream_ptr(self.device))
        L.check(rc, "exx_gradient")
        return grad_psi, grad_occ

    def compute_noalloc(self, psi: torch.Tensor, occ: torch.Tensor, mode: str = "energy_kpsi",
                        kpsi: torch.Tensor | None = None, pair_e: torch.Tensor | None = None,
                        ex_out: torch.Tensor | None = None, accumulate: bool = False):
        """exx_compute_noalloc: the library's static per-GPU workspace instead of a
        caller's; every output tensor must be passed in (nothing is allocated) and
        the schedule for this orbital count must be prepared."""
        n = self.grid.n
        N = int(psi.shape[0])
        _check_tensor("psi", psi, (N, n, n, n), self.device, self.dtype)
        _check_tensor("occ", occ, (N,), self.device)
        m = MODES[mode]
        if m & L.MODE_ENERGY and ex_out is None:
            raise ValueError("ex_out is required for energy modes (nothing is allocated)")
        if m & L.MODE_KPSI and kpsi is None:
            raise ValueError("kpsi is required for K psi modes (nothing is allocated)")
        if kpsi is not None:
            _check_tensor("kpsi", kpsi, (N, n, n, n), self.device, self.dtype)
        if pair_e is not None:
            _check_tensor("pair_e", pair_e, (N, N), self.device)
        flags = L.FLAG_ACCUMULATE if accumulate else 0
        with torch.cuda.device(self.device):
            rc = L.lib().exx_compute_noalloc(self._h, psi.data_ptr(), occ.data_ptr(), N, m, flags,
                                             _ptr(ex_out), _ptr(kpsi), _ptr(pair_e),
                                             _stream_ptr(self.device))
        L.check(rc, "exx_compute_noalloc")
        return ex_out, kpsi, pair_e

    def autotune(self, psi: torch.Tensor, occ: torch.Tensor, cache_path: str | None = None,
                 budget_ms: int = 0) -> dict:
        N = int(psi.shape[0])
        kpsi = torch.empty_like(psi)
        ws = self.workspace(N)
        # the largest candidate batch may need more workspace than the default tuning
        big = max(self.workspace_bytes(N), ws.numel())
        ws = torch.empty(big, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            rc = L.lib().exx_autotune(self._h, psi.data_ptr(), occ.data_ptr(), N, kpsi.data_ptr(),
                                      ws.data_ptr(), ws.numel(), _stream_ptr(self.device),
                                      int(budget_ms),
                                      cache_path.encode() if cache_path else None)
        L.check(rc, "exx_autotune")
        self._ws = None
        return self.tuning


_PLANS: dict = {}


def get_plan(grid: Grid, precision: str, n_orb: int, device: torch.device,
             complex_orbitals: bool = False) -> Plan:
    key = (grid, precision, device.index, bool(complex_orbitals))
    p = _PLANS.get(key)
    if p is None or p.n_orb_max < n_orb:
        p = Plan(grid, precision, max(n_orb, 64), device, complex_orbitals)
        _PLANS[key] = p
    return p


def energy_and_kpsi(psi: torch.Tensor, occ: torch.Tensor, grid: Grid, precision: str = "fp32",
                    pair_energies: bool = False):
    """E_x (0-dim float64 tensor), K psi (like psi) and optionally e_ij [N, N].

    psi may be float64 or complex128 (complex orbitals)."""
    plan = get_plan(grid, precision, psi.shape[0], psi.device, psi.is_complex())
    pe = torch.empty((psi.shape[0], psi.shape[0]), dtype=torch.float64,
                     device=psi.device) if pair_energies else None
    ex, kpsi, pe = plan.compute(psi, occ, "energy_kpsi", pair_e=pe)
    return (ex, kpsi, pe) if pair_energies else (ex, kpsi)


def exchange_energy(psi: torch.Tensor, occ: torch.Tensor, grid: Grid,
                    precision: str = "fp32") -> torch.Tensor:
    """E_x alone (Parseval route: one forward transform per pair)."""
    plan = get_plan(grid, precision, psi.shape[0], psi.device, psi.is_complex())
    ex, _, _ = plan.compute(psi, occ, "energy")
    return ex


def library_version() -> str:
    return L.lib().exx_version().decode()
