"""MI355X semi-discrete optimal transport (MAK reconstruction hot path).

Context: Laguerre cell passes (volumes, centroids, the Hessian and faces), the
damped-Newton solve (uniform or per-site target masses), the Legendre
transform of the weights on query points or a mesh, the Zel'dovich deposit
of the cells' mass on an Eulerian mesh (by Lagrangian elements, or exactly,
by clipping the moved cells against the voxels), and the power spectrum of
a mesh field.  Server: many solves of different sizes on one device.

Thin ctypes binding of libmak.so (include/mak.h): argument marshalling only.
PyTorch provides the device memory and the stream; every step of the cell
pass and of the Newton solve runs in the HIP kernels of the library.  There is
no fallback: if the library is not built, or no GPU is present, the calls
raise.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "MakError", "Context", "Server", "Request", "load_library", "laguerre_cells", "solve", "solve_from",
    "memory_estimate", "LIB_PATH", "EXPORTED_SYMBOLS",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmak.so")

EXPORTED_SYMBOLS = [
    "mak_default_options", "mak_create", "mak_destroy", "mak_last_error",
    "mak_laguerre_cells", "mak_hessian_copy", "mak_faces_copy", "mak_solve",
    "mak_solve_masses", "mak_solve_from", "mak_solve_memory_estimate", "mak_legendre",
    "mak_legendre_mesh", "mak_power_spectrum", "mak_za_deposit", "mak_za_deposit_cells",
    "mak_profile_enable", "mak_profile_read",
    "mak_profile_counters", "mak_server_create", "mak_server_submit", "mak_server_poll",
    "mak_server_wait", "mak_server_release", "mak_server_stats", "mak_server_last_error",
    "mak_server_destroy", "mak_device_bytes", "mak_legendre_noalloc",
]

STATUS = {0: "MAK_OK", 1: "MAK_EINVAL", 2: "MAK_ENOMEM", 3: "MAK_EDEGENERATE",
          4: "MAK_ENOCONV", 5: "MAK_EOVERFLOW", 6: "MAK_EHIP", 7: "MAK_ENOTFOUND"}
PRECISION = {"fp64": 0, "mixed": 1}


class MakError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))
        self.message = message


class _Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("max_newton", ctypes.c_int32),
        ("max_cg", ctypes.c_int32), ("max_halvings", ctypes.c_int32),
        ("cg_rtol", ctypes.c_double), ("grid_occupancy", ctypes.c_double),
        ("mem_budget_bytes", ctypes.c_size_t), ("verbose", ctypes.c_int32),
        ("first_stage", ctypes.c_int32), ("batch_window_us", ctypes.c_int32),
        ("cg_precond", ctypes.c_int32), ("walk_cert", ctypes.c_int32), ("topo_reuse", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class _SolveInfo(ctypes.Structure):
    _fields_ = [
        ("newton_iters", ctypes.c_int32), ("cg_iters_total", ctypes.c_int32),
        ("ls_trials", ctypes.c_int32), ("cell_passes", ctypes.c_int32),
        ("fp64_rerun_cells", ctypes.c_int64), ("overflow_cells", ctypes.c_int64),
        ("final_err", ctypes.c_double), ("seconds", ctypes.c_double),
        ("abandoned_trials", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class _CellsInfo(ctypes.Structure):
    _fields_ = [
        ("empty_cells", ctypes.c_int64), ("fp64_rerun_cells", ctypes.c_int64),
        ("overflow_cells", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("faces", ctypes.c_int64), ("max_faces", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class _KernelProfile(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
        ("units", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
    ]


COUNTER_NAMES = ["sites_scanned", "planes_tested", "vertex_tests", "cuts", "new_vertices",
                 "ball_vertices", "box_tests", "final_vertices", "faces", "cells",
                 "cycles_search", "cycles_clip", "cycles_integrals", "cycles_prefilter",
                 "cycles_cuts", "search_flops",
                 "scan_warm", "scan_near", "scan_ring2", "scan_blocks",
                 "inball_warm", "inball_near", "inball_ring2", "inball_blocks",
                 "cut_warm", "cut_near", "cut_ring2", "cut_blocks",
                 "boxtest_ring2", "boxpass_ring2", "boxtest_blocks", "boxpass_blocks",
                 "boxtest_blockcells", "boxpass_blockcells", "shell_sum",
                 "cert_recorded", "cert_sites", "cert_overflow", "cert_tried", "cert_walk_skipped",
                 "topo_tried", "topo_reused"]


class _ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("queued", ctypes.c_int64),
        ("active", ctypes.c_int32), ("peak_active", ctypes.c_int32),
        ("admitted_while_busy", ctypes.c_int64), ("used_bytes", ctypes.c_size_t),
        ("peak_used_bytes", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t),
        ("pass_batches", ctypes.c_int64), ("batched_passes", ctypes.c_int64),
        ("max_batch", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("releases", ctypes.c_int64),
    ]


class _Csr(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


def _as_dict(s) -> dict:
    return {name: getattr(s, name) for name, _ in s._fields_ if name != "reserved"}


_LIB = None


def load_library():
    """Load libmak.so (built in-tree by __graft_entry__.build())."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, D, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int32
    lib.mak_default_options.argtypes = [P]
    lib.mak_default_options.restype = None
    lib.mak_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    lib.mak_create.restype = ctypes.c_int
    lib.mak_destroy.argtypes = [P]
    lib.mak_destroy.restype = None
    lib.mak_last_error.argtypes = [P]
    lib.mak_last_error.restype = ctypes.c_char_p
    lib.mak_laguerre_cells.argtypes = [P, P, P, I64, D, P, P, P, P, P]
    lib.mak_laguerre_cells.restype = ctypes.c_int
    lib.mak_hessian_copy.argtypes = [P, P, P, P, P]
    lib.mak_hessian_copy.restype = ctypes.c_int
    lib.mak_faces_copy.argtypes = [P, P, P, P, P, P]
    lib.mak_faces_copy.restype = ctypes.c_int
    lib.mak_solve.argtypes = [P, P, I64, D, D, P, P, P, P, P]
    lib.mak_solve.restype = ctypes.c_int
    lib.mak_za_deposit.argtypes = [P, P, P, I64, D, D, I64, D, I64, ctypes.c_int32, P, P]
    lib.mak_za_deposit.restype = ctypes.c_int
    lib.mak_za_deposit_cells.argtypes = [P, P, P, I64, D, D, I64, P, P]
    lib.mak_za_deposit_cells.restype = ctypes.c_int
    lib.mak_power_spectrum.argtypes = [P, P, I64, D, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       P, P, P, P]
    lib.mak_power_spectrum.restype = ctypes.c_int
    lib.mak_legendre.argtypes = [P, P, P, I64, D, P, I64, P, P, P, P]
    lib.mak_legendre.restype = ctypes.c_int
    lib.mak_legendre_noalloc.argtypes = [P, P, P, I64, D, P, I64, P, P, P, P]
    lib.mak_legendre_noalloc.restype = ctypes.c_int
    lib.mak_legendre_mesh.argtypes = [P, P, P, I64, D, I64, D, P, P, P, P]
    lib.mak_legendre_mesh.restype = ctypes.c_int
    lib.mak_solve_masses.argtypes = [P, P, P, I64, D, D, P, P, P, P, P]
    lib.mak_solve_masses.restype = ctypes.c_int
    lib.mak_solve_from.argtypes = [P, P, I64, D, D, P, P, P, P, P]
    lib.mak_solve_from.restype = ctypes.c_int
    lib.mak_solve_memory_estimate.argtypes = [I64, I32]
    lib.mak_solve_memory_estimate.restype = ctypes.c_size_t
    lib.mak_device_bytes.argtypes = [P, P, I32]
    lib.mak_device_bytes.restype = None
    lib.mak_profile_enable.argtypes = [P, I32]
    lib.mak_profile_enable.restype = ctypes.c_int
    lib.mak_profile_read.argtypes = [P, P, I32]
    lib.mak_profile_read.restype = I32
    lib.mak_profile_counters.argtypes = [P, P]
    lib.mak_profile_counters.restype = ctypes.c_int
    lib.mak_server_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P, ctypes.c_size_t, I32]
    lib.mak_server_create.restype = ctypes.c_int
    lib.mak_server_submit.argtypes = [P, P, I64, D, D, P, P, P, ctypes.POINTER(I64)]
    lib.mak_server_submit.restype = ctypes.c_int
    lib.mak_server_poll.argtypes = [P, I64, ctypes.POINTER(I32), P, P]
    lib.mak_server_poll.restype = ctypes.c_int
    lib.mak_server_wait.argtypes = [P, I64, P, P]
    lib.mak_server_wait.restype = ctypes.c_int
    lib.mak_server_release.argtypes = [P, I64]
    lib.mak_server_release.restype = ctypes.c_int
    lib.mak_server_stats.argtypes = [P, P]
    lib.mak_server_stats.restype = ctypes.c_int
    lib.mak_server_last_error.argtypes = [P]
    lib.mak_server_last_error.restype = ctypes.c_char_p
    lib.mak_server_destroy.argtypes = [P]
    lib.mak_server_destroy.restype = None
    _LIB = lib
    return lib


def default_options() -> dict:
    lib = load_library()
    o = _Options()
    lib.mak_default_options(ctypes.byref(o))
    return _as_dict(o)


def memory_estimate(n: int, precision: str = "fp64") -> int:
    return int(load_library().mak_solve_memory_estimate(int(n), PRECISION[precision]))


def device_bytes(reset_peak: bool = False):
    """(live, peak): device bytes the library holds now and the most it held
    at once since the last reset (its own allocations, all contexts)."""
    live, peak = ctypes.c_size_t(), ctypes.c_size_t()
    load_library().mak_device_bytes(ctypes.byref(live), ctypes.byref(peak), 1 if reset_peak else 0)
    return int(live.value), int(peak.value)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the MAK library runs only on the device")
    return torch


class Context:
    """A library context on one device (owns the device workspace)."""

    def __init__(self, device: int = 0, precision: str = "fp64", **opts):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        o = _Options()
        self.lib.mak_default_options(ctypes.byref(o))
        o.precision = PRECISION[precision]
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        self.options = _as_dict(o)
        h = ctypes.c_void_p()
        torch.cuda.init()
        st = self.lib.mak_create(ctypes.byref(h), device, ctypes.byref(o))
        if st != 0:
            raise MakError(st, self.lib.mak_last_error(None).decode())
        self._h = h
        self._last_nnz = None
        self._last_faces = None
        self._last_n = None

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mak_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != 0:
            raise MakError(st, self.lib.mak_last_error(self._h).decode())

    def _stream(self):
        torch = _torch()
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, t, shape_tail=None):
        torch = _torch()
        t = torch.as_tensor(t)
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        if shape_tail is not None and tuple(t.shape[1:]) != shape_tail:
            raise ValueError(f"expected shape (N,{shape_tail}), got {tuple(t.shape)}")
        return t

    def laguerre_cells(self, points, psi, L: float):
        """Volumes (N,) and centroids (N,3) of the periodic Laguerre cells;
        the Hessian and faces of this pass are kept for hessian()/faces()."""
        torch = _torch()
        x = self._dev(points, (3,))
        n = x.shape[0]
        w = self._dev(psi)
        if w.shape != (n,):
            raise ValueError("psi must have shape (N,)")
        V = torch.empty(n, dtype=torch.float64, device=self.device)
        C = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        info = _CellsInfo()
        csr = _Csr()
        self._check(self.lib.mak_laguerre_cells(self._h, x.data_ptr(), w.data_ptr(), n, float(L),
                                                V.data_ptr(), C.data_ptr(), ctypes.byref(csr),
                                                ctypes.byref(info), self._stream()))
        self._last_n, self._last_nnz, self._last_faces = n, info.nnz, info.faces
        self._last_csr = {name: getattr(csr, name) for name, _ in csr._fields_}
        return V, C, _as_dict(info)

    def hessian_view(self) -> dict:
        """The library-owned CSR that the last mak_laguerre_cells returned:
        n_rows, nnz and the DEVICE addresses row_ptr, col, val (valid until
        the next cell pass on this context)."""
        return dict(self._last_csr)

    def hessian(self):
        """CSR (row_ptr int64, col int32, val float64) of J = dV/dpsi of the
        last cell pass (original index order)."""
        torch = _torch()
        n, nnz = self._last_n, self._last_nnz
        rp = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        self._check(self.lib.mak_hessian_copy(self._h, rp.data_ptr(), col.data_ptr(), val.data_ptr(),
                                              self._stream()))
        return rp, col[:nnz], val[:nnz]

    def faces(self):
        """Faces of the last cell pass: face_ptr (N+1), j, shift (F,3), area."""
        torch = _torch()
        n, nf = self._last_n, self._last_faces
        fp = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        fj = torch.empty(max(nf, 1), dtype=torch.int32, device=self.device)
        fs = torch.empty((max(nf, 1), 3), dtype=torch.int32, device=self.device)
        fa = torch.empty(max(nf, 1), dtype=torch.float64, device=self.device)
        self._check(self.lib.mak_faces_copy(self._h, fp.data_ptr(), fj.data_ptr(), fs.data_ptr(),
                                            fa.data_ptr(), self._stream()))
        return {"face_ptr": fp, "face_j": fj[:nf], "face_shift": fs[:nf], "face_area": fa[:nf]}

    def profile_enable(self, timing: bool = True, counting: bool = False, cells_only: bool = False):
        """Start (and clear) the kernel profile: event timing (of every main
        kernel, or with cells_only of the cell-pass kernels alone) and/or
        counted work."""
        self._check(self.lib.mak_profile_enable(
            self._h, (1 if timing else 0) | (2 if counting else 0) | (4 if cells_only else 0)))

    def profile_read(self) -> dict:
        """{kernel name: {launches, total_ms, units, flops, bytes}} since profile_enable."""
        n = self.lib.mak_profile_read(self._h, None, 0)
        if n < 0:
            raise MakError(6, self.lib.mak_last_error(self._h).decode())
        arr = (_KernelProfile * max(n, 1))()
        self.lib.mak_profile_read(self._h, arr, n)
        out = {}
        for k in range(n):
            d = _as_dict(arr[k])
            out[d.pop("name").decode()] = d
        c = (ctypes.c_double * 48)()
        self._check(self.lib.mak_profile_counters(self._h, c))
        out["_counters"] = {name: c[i] for i, name in enumerate(COUNTER_NAMES)}
        return out

    def _solve(self, fn, points, L, tol, psi0):
        torch = _torch()
        x = self._dev(points, (3,))
        n = x.shape[0]
        if psi0 is None:
            psi = torch.empty(n, dtype=torch.float64, device=self.device)
        else:
            psi = self._dev(psi0).clone()
        C = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        D = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        info = _SolveInfo()
        st = fn(self._h, x.data_ptr(), n, float(L), float(tol), psi.data_ptr(), C.data_ptr(),
                D.data_ptr(), ctypes.byref(info), self._stream())
        self._check(st)
        return psi, C, D, _as_dict(info)

    def solve(self, points, L: float, tol: float = 1e-6, masses=None):
        """Damped Newton OT solve from psi = 0: (psi, centroids, displacements, info).
        masses (optional, (N,) float64, positive, summing to L^3): the target
        volume of each cell instead of L^3 / N."""
        if masses is None:
            return self._solve(self.lib.mak_solve, points, L, tol, None)
        torch = _torch()
        x = self._dev(points, (3,))
        n = x.shape[0]
        m = self._dev(masses)
        if m.shape != (n,):
            raise ValueError("masses must have shape (N,)")
        psi = torch.empty(n, dtype=torch.float64, device=self.device)
        C = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        D = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        info = _SolveInfo()
        st = self.lib.mak_solve_masses(self._h, x.data_ptr(), m.data_ptr(), n, float(L), float(tol),
                                       psi.data_ptr(), C.data_ptr(), D.data_ptr(), ctypes.byref(info),
                                       self._stream())
        self._check(st)
        return psi, C, D, _as_dict(info)

    def solve_from(self, points, psi0, L: float, tol: float = 1e-6):
        """Resume a solve from saved weights psi0."""
        return self._solve(self.lib.mak_solve_from, points, L, tol, psi0)

    def za_deposit(self, points, psi, L: float, tau: float, n_lag: int, ng: int, scheme: str = "cic",
                   lag_offset: float = 0.5):
        """Density (ng, ng, ng) of the mass of the cells moved to growth
        amplitude tau (Zel'dovich), carried by n_lag^3 Lagrangian elements."""
        torch = _torch()
        x = self._dev(points, (3,))
        w = None if psi is None else self._dev(psi)
        sch = {"ngp": 1, "cic": 2}[scheme]
        rho = torch.empty((int(ng),) * 3, dtype=torch.float64, device=self.device)
        st = self.lib.mak_za_deposit(self._h, x.data_ptr(), None if w is None else w.data_ptr(),
                                     x.shape[0], float(L), float(tau), int(n_lag), float(lag_offset),
                                     int(ng), sch, rho.data_ptr(), self._stream())
        self._check(st)
        return rho

    def za_deposit_cells(self, points, psi, L: float, tau: float, ng: int):
        """Density (ng, ng, ng) of the cells themselves moved to growth
        amplitude tau < 1: each cell shrunk by 1 - tau towards its site and
        clipped against the voxels (the limit of za_deposit as n_lag grows)."""
        torch = _torch()
        x = self._dev(points, (3,))
        w = None if psi is None else self._dev(psi)
        rho = torch.empty((int(ng),) * 3, dtype=torch.float64, device=self.device)
        st = self.lib.mak_za_deposit_cells(self._h, x.data_ptr(), None if w is None else w.data_ptr(),
                                           x.shape[0], float(L), float(tau), int(ng), rho.data_ptr(),
                                           self._stream())
        self._check(st)
        return rho

    def power_spectrum(self, field, L: float, nbins=None, window: int = 0, contrast: bool = False):
        """Shell-averaged power spectrum of an (ng, ng, ng) mesh field:
        (k_mean, power, modes) per shell j = 1..nbins (default ng // 2)."""
        torch = _torch()
        f = self._dev(field)
        ng = f.shape[0]
        if f.shape != (ng, ng, ng):
            raise ValueError("field must have shape (ng, ng, ng)")
        nb = ng // 2 if nbins is None else int(nbins)
        k = torch.empty(nb, dtype=torch.float64, device=self.device)
        P = torch.empty(nb, dtype=torch.float64, device=self.device)
        m = torch.empty(nb, dtype=torch.int64, device=self.device)
        st = self.lib.mak_power_spectrum(self._h, f.data_ptr(), ng, float(L), nb, int(window),
                                         1 if contrast else 0, k.data_ptr(), P.data_ptr(), m.data_ptr(),
                                         self._stream())
        self._check(st)
        return k, P, m

    def _legendre_out(self, q):
        torch = _torch()
        return (torch.empty(q, dtype=torch.float64, device=self.device),
                torch.empty(q, dtype=torch.int32, device=self.device),
                torch.empty((q, 3), dtype=torch.float64, device=self.device))

    def legendre(self, points, psi, L: float, queries):
        """Legendre transform of the weights at query points (Q, 3):
        (phi (Q,), idx (Q,) int32, disp (Q, 3)), disp = x_idx + kL - q."""
        x = self._dev(points, (3,))
        w = None if psi is None else self._dev(psi)
        q = self._dev(queries, (3,))
        phi, idx, disp = self._legendre_out(q.shape[0])
        st = self.lib.mak_legendre(self._h, x.data_ptr(), None if w is None else w.data_ptr(),
                                   x.shape[0], float(L), q.data_ptr(), q.shape[0],
                                   phi.data_ptr(), idx.data_ptr(), disp.data_ptr(), self._stream())
        self._check(st)
        return phi, idx, disp

    def legendre_noalloc(self, points, psi, L: float, queries, out=None):
        """mak_legendre_noalloc: the same as legendre() with the library's
        workspace in its static device array (the library allocates no
        device memory).  out: optional (phi, idx, disp) tensors to write."""
        x = self._dev(points, (3,))
        w = None if psi is None else self._dev(psi)
        q = self._dev(queries, (3,))
        phi, idx, disp = out if out is not None else self._legendre_out(q.shape[0])
        st = self.lib.mak_legendre_noalloc(self._h, x.data_ptr(), None if w is None else w.data_ptr(),
                                           x.shape[0], float(L), q.data_ptr(), q.shape[0],
                                           phi.data_ptr(), idx.data_ptr(), disp.data_ptr(),
                                           self._stream())
        self._check(st)
        return phi, idx, disp

    def legendre_mesh(self, points, psi, L: float, ng: int, offset: float = 0.0):
        """The same on the ng^3 mesh ((a, b, c) + offset) L / ng, c fastest."""
        x = self._dev(points, (3,))
        w = None if psi is None else self._dev(psi)
        phi, idx, disp = self._legendre_out(int(ng) ** 3)
        st = self.lib.mak_legendre_mesh(self._h, x.data_ptr(), None if w is None else w.data_ptr(),
                                        x.shape[0], float(L), int(ng), float(offset), phi.data_ptr(),
                                        idx.data_ptr(), disp.data_ptr(), self._stream())
        self._check(st)
        return phi, idx, disp


class Request:
    """A submitted solve: output tensors plus its id on the server."""

    def __init__(self, server, rid, points, psi, centroids, disp):
        self.server, self.id = server, rid
        self.points, self.psi, self.centroids, self.displacements = points, psi, centroids, disp
        self.info = None
        self.times = None

    def done(self) -> bool:
        return self.server._poll(self)

    def wait(self):
        """Block until done; returns (psi, centroids, displacements, info)."""
        self.server._wait(self)
        return self.psi, self.centroids, self.displacements, self.info


class Server:
    """Continuous-batching solver: requests are admitted FIFO as worker slots
    and the memory budget allow, and run concurrently on their own streams."""

    def __init__(self, device: int = 0, precision: str = "fp64", mem_budget: int = 0,
                 max_slots: int = 4, **opts):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        o = _Options()
        self.lib.mak_default_options(ctypes.byref(o))
        o.precision = PRECISION[precision]
        for k, v in opts.items():
            setattr(o, k, v)
        h = ctypes.c_void_p()
        torch.cuda.init()
        st = self.lib.mak_server_create(ctypes.byref(h), device, ctypes.byref(o), int(mem_budget),
                                        int(max_slots))
        if st != 0:
            raise MakError(st, "server creation failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mak_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, points, L: float, tol: float = 1e-6) -> Request:
        torch = _torch()
        x = torch.as_tensor(points).to(device=self.device, dtype=torch.float64).contiguous()
        n = x.shape[0]
        psi = torch.empty(n, dtype=torch.float64, device=self.device)
        C = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        D = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()  # inputs complete before submit
        rid = ctypes.c_int64()
        st = self.lib.mak_server_submit(self._h, x.data_ptr(), n, float(L), float(tol), psi.data_ptr(),
                                        C.data_ptr(), D.data_ptr(), ctypes.byref(rid))
        if st != 0:
            raise MakError(st, self.lib.mak_server_last_error(self._h).decode())
        return Request(self, rid.value, x, psi, C, D)

    def _poll(self, r: Request) -> bool:
        done = ctypes.c_int32()
        info = _SolveInfo()
        times = (ctypes.c_double * 3)()
        st = self.lib.mak_server_poll(self._h, r.id, ctypes.byref(done), ctypes.byref(info), times)
        if done.value:
            if st != 0:
                raise MakError(st, "request failed")
            r.info, r.times = _as_dict(info), tuple(times)
        return bool(done.value)

    def _wait(self, r: Request):
        info = _SolveInfo()
        times = (ctypes.c_double * 3)()
        st = self.lib.mak_server_wait(self._h, r.id, ctypes.byref(info), times)
        if st != 0:
            raise MakError(st, self.lib.mak_server_last_error(self._h).decode())
        r.info, r.times = _as_dict(info), tuple(times)
        self.lib.mak_server_release(self._h, r.id)

    def stats(self) -> dict:
        s = _ServerStats()
        self.lib.mak_server_stats(self._h, ctypes.byref(s))
        return _as_dict(s)


def laguerre_cells(points, psi, L: float, device: int = 0, precision: str = "fp64"):
    return Context(device, precision).laguerre_cells(points, psi, L)


def solve(points, L: float, tol: float = 1e-6, device: int = 0, precision: str = "fp64", **opts):
    return Context(device, precision, **opts).solve(points, L, tol)


def solve_from(points, psi0, L: float, tol: float = 1e-6, device: int = 0, precision: str = "fp64",
               **opts):
    return Context(device, precision, **opts).solve_from(points, psi0, L, tol)
