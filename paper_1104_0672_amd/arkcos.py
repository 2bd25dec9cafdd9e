"""ctypes binding of libarkcos.so (the C ABI in include/arkcos.h).

Argument marshalling only: every step of the convolution runs in the HIP
library.  PyTorch supplies device memory and the current stream.  If the
library is missing the import-time loader raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libarkcos.so")

F32, F64 = 0, 1
ECP, HEALPIX = 0, 1
GAUSSIAN, SPLINE = 0, 1


class ArkcosError(RuntimeError):
    pass


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nside", ctypes.c_int64), ("n_theta", ctypes.c_int64),
                ("n_phi", ctypes.c_int64)]


class ProfileC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("fwhm_rad", ctypes.c_double), ("n_knots", ctypes.c_int32),
                ("theta_max_rad", ctypes.c_double), ("knot_values", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("oversample", ctypes.c_int32), ("kgen", ctypes.c_int32),
                ("fix_pole_pixels", ctypes.c_int32), ("band_tol", ctypes.c_double),
                ("mode", ctypes.c_int32), ("own_grid", ctypes.c_int32), ("kernel_eval", ctypes.c_int32),
                ("table_nodes", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("npix", ctypes.c_int64), ("nrings", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_table_pairs", ctypes.c_int64), ("spectrum_modes", ctypes.c_int64),
                ("output_modes", ctypes.c_int64), ("pair_modes", ctypes.c_int64),
                ("taps", ctypes.c_int64), ("table_entries", ctypes.c_int64),
                ("oversample", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n_knots", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("workspace_bytes", ctypes.c_size_t),
                ("plan_bytes", ctypes.c_size_t), ("pairs_by_kind", ctypes.c_int64 * 4),
                ("acc_seg_units", ctypes.c_int32), ("acc_group", ctypes.c_int32), ("acc_window", ctypes.c_int32),
                ("acc_tuned", ctypes.c_int32), ("support_radius_rad", ctypes.c_double),
                ("table_fft_rows", ctypes.c_int32), ("grad_fft_rows", ctypes.c_int32),
                ("acc_units_per_wave", ctypes.c_int32), ("reserved2", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_maps", ctypes.c_int32), ("seg_units", ctypes.c_int32), ("group", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("tuned", ctypes.c_int32), ("units_per_wave", ctypes.c_int32),
                ("n_items", ctypes.c_int64), ("npix_total", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t)]


EXPORTED = ["arkcos_default_options", "arkcos_plan", "arkcos_plan_destroy", "arkcos_plan_get_info",
            "arkcos_workspace_size", "arkcos_convolve", "arkcos_convolve_adjoint",
            "arkcos_kernel_grad",
            "arkcos_set_knots", "arkcos_set_knots_async", "arkcos_batch_plan", "arkcos_batch_get_info", "arkcos_batch_workspace_size",
            "arkcos_batch_convolve", "arkcos_batch_timing", "arkcos_batch_stage_times", "arkcos_batch_destroy",
            "arkcos_plan_timing", "arkcos_stage_times", "arkcos_status_string", "arkcos_last_error",
            "arkcos_truncation_variance", "arkcos_choose_radius", "arkcos_plan_for_error",
            "arkcos_batch_plan_shared_input", "arkcos_batch_convolve_shared",
            "arkcos_convolve_noalloc", "arkcos_noalloc_scratch_bytes"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libarkcos.so and declare its signatures.  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ArkcosError(f"{path} not found: build it with `python -m paper_1104_0672_amd.build` "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, st, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_double
    lib.arkcos_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.arkcos_default_options.restype = None
    lib.arkcos_plan.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(ProfileC), dbl, i32,
                                ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.arkcos_plan_for_error.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(ProfileC),
                                          ctypes.POINTER(ctypes.c_double), i32, dbl, i32,
                                          ctypes.POINTER(Options), ctypes.POINTER(vp),
                                          ctypes.POINTER(ctypes.c_double)]
    lib.arkcos_plan_destroy.argtypes = [vp]
    lib.arkcos_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.arkcos_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.arkcos_convolve.argtypes = [vp, vp, vp, vp, vp]
    lib.arkcos_convolve_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.arkcos_convolve_noalloc.argtypes = [vp, vp, vp, vp]
    lib.arkcos_noalloc_scratch_bytes.argtypes = []
    lib.arkcos_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.arkcos_kernel_grad.argtypes = [vp, vp, vp, vp, vp, ctypes.c_uint32, vp]
    lib.arkcos_set_knots.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.arkcos_set_knots_async.argtypes = [vp, vp, vp]
    lib.arkcos_batch_plan.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.arkcos_batch_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.arkcos_batch_convolve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp, vp]
    lib.arkcos_batch_plan_shared_input.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.arkcos_batch_convolve_shared.argtypes = [vp, vp, ctypes.POINTER(vp), vp, vp]
    lib.arkcos_batch_destroy.argtypes = [vp]
    lib.arkcos_batch_get_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    lib.arkcos_batch_timing.argtypes = [vp, i32]
    lib.arkcos_batch_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.arkcos_plan_timing.argtypes = [vp, i32]
    lib.arkcos_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    pd = ctypes.POINTER(ctypes.c_double)
    lib.arkcos_truncation_variance.argtypes = [ctypes.POINTER(ProfileC), dbl, pd, i32, pd, pd]
    lib.arkcos_choose_radius.argtypes = [ctypes.POINTER(ProfileC), pd, i32, dbl, pd]
    lib.arkcos_status_string.argtypes = [st]
    lib.arkcos_status_string.restype = ctypes.c_char_p
    lib.arkcos_last_error.argtypes = []
    lib.arkcos_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        f = getattr(lib, name)
        if name == "arkcos_noalloc_scratch_bytes":
            continue
        if f.restype is ctypes.c_int or name in ("arkcos_plan", "arkcos_plan_destroy", "arkcos_plan_for_error"):
            f.restype = st
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        lib = load_library()
        raise ArkcosError(f"{what}: {lib.arkcos_status_string(status).decode()} "
                          f"({lib.arkcos_last_error().decode()})")


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A convolution plan: geometry, kernel profile, support radius, dtype.

    Maps are 1-D torch tensors on the plan's device with npix elements
    (RING order) of the plan's dtype.  With radius=None the support radius
    is chosen from a truncation-error target instead (arkcos_plan_for_error):
    the smallest R whose error variance for the power spectrum `cl` is at
    most `target_sigma2`; it is then `info.support_radius_rad`.
    """

    def __init__(self, grid: str, radius: Optional[float], *, nside: int = 0, ntheta: int = 0, nphi: int = 0,
                 fwhm: float = 0.0, knots: Optional[Sequence[float]] = None, theta_max: float = 0.0,
                 dtype: str = "f32", oversample: int = 0, kgen: int = 0, fix_pole_pixels: bool = True,
                 band_tol: float = -1.0, mode: str = "suppressed", own_grid: str = "equal_length",
                 kernel_eval: str = "exact", table_nodes: int = 0, cl=None, target_sigma2: Optional[float] = None):
        lib = load_library()
        self._lib = lib
        self.handle = ctypes.c_void_p()
        geom = Geometry(HEALPIX if grid == "healpix" else ECP, nside, ntheta, nphi)
        self._knots = None
        if knots is not None:
            self._knots = (ctypes.c_double * len(knots))(*[float(v) for v in knots])
            prof = ProfileC(SPLINE, 0.0, len(knots), float(theta_max),
                            ctypes.cast(self._knots, ctypes.POINTER(ctypes.c_double)))
        else:
            prof = ProfileC(GAUSSIAN, float(fwhm), 0, 0.0, None)
        if mode not in ("suppressed", "default"):
            raise ArkcosError(f"mode must be 'suppressed' or 'default', not {mode!r}")
        if own_grid not in ("equal_length", "equatorial"):
            raise ArkcosError(f"own_grid must be 'equal_length' or 'equatorial', not {own_grid!r}")
        if kernel_eval not in ("exact", "table"):
            raise ArkcosError(f"kernel_eval must be 'exact' or 'table', not {kernel_eval!r}")
        opts = Options(int(oversample), int(kgen), int(bool(fix_pole_pixels)), float(band_tol),
                       1 if mode == "default" else 0, 1 if own_grid == "equatorial" else 0,
                       1 if kernel_eval == "table" else 0, int(table_nodes))
        self.dtype = torch.float32 if dtype == "f32" else torch.float64
        self.grid = grid
        if radius is None:
            if cl is None or target_sigma2 is None:
                raise ArkcosError("radius=None needs cl and target_sigma2")
            c = np.ascontiguousarray(cl, dtype=np.float64)
            _check(lib.arkcos_plan_for_error(ctypes.byref(geom), ctypes.byref(prof),
                                             c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), c.size - 1,
                                             float(target_sigma2), F32 if dtype == "f32" else F64,
                                             ctypes.byref(opts), ctypes.byref(self.handle), None),
                   "arkcos_plan_for_error")
        else:
            _check(lib.arkcos_plan(ctypes.byref(geom), ctypes.byref(prof), float(radius),
                                   F32 if dtype == "f32" else F64, ctypes.byref(opts),
                                   ctypes.byref(self.handle)), "arkcos_plan")
        self.device = torch.device("cuda", torch.cuda.current_device())
        info = PlanInfo()
        _check(lib.arkcos_plan_get_info(self.handle, ctypes.byref(info)), "arkcos_plan_get_info")
        self.info = info
        self.npix = int(info.npix)
        self.n_knots = int(info.n_knots)
        self._ws = None

    @classmethod
    def from_workload(cls, w, **kw) -> "Plan":
        g, p = w.grid, w.profile
        args = dict(nside=g.nside, ntheta=g.ntheta, nphi=g.nphi, dtype=w.dtype)
        if p.kind == "gaussian":
            args["fwhm"] = p.fwhm
        else:
            args["knots"] = list(p.knots)
            args["theta_max"] = p.theta_max
        args.update(kw)
        return cls(g.kind, w.radius, **args)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                self._lib.arkcos_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    # --------------------------------------------------------------- memory
    @property
    def workspace_bytes(self) -> int:
        return int(self.info.workspace_bytes)

    def workspace(self) -> torch.Tensor:
        """A cached workspace for calls on the current stream."""
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        return self._ws

    def _ws_ptr(self, ws: Optional[torch.Tensor]) -> ctypes.c_void_p:
        ws = self.workspace() if ws is None else ws
        if ws.numel() < self.workspace_bytes or not ws.is_cuda:
            raise ArkcosError("workspace too small")
        addr = ws.data_ptr()
        addr = (addr + 255) // 256 * 256
        if addr + self.workspace_bytes > ws.data_ptr() + ws.numel():
            raise ArkcosError("workspace too small after alignment")
        return ctypes.c_void_p(addr)

    def _map(self, t: torch.Tensor, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ArkcosError(f"{name} must be a CUDA tensor")
        if t.dtype != self.dtype or t.numel() != self.npix or not t.is_contiguous():
            raise ArkcosError(f"{name} must be a contiguous {self.dtype} tensor with {self.npix} elements")
        return t

    # ----------------------------------------------------------- operations
    def convolve(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, ws=None, stream=None):
        x = self._map(x, "x")
        y = torch.empty_like(x) if out is None else self._map(out, "out")
        _check(self._lib.arkcos_convolve(self.handle, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()), self._ws_ptr(ws),
                                         _stream_ptr(stream)), "arkcos_convolve")
        return y

    def adjoint(self, r: torch.Tensor, out: Optional[torch.Tensor] = None, ws=None, stream=None):
        r = self._map(r, "r")
        xb = torch.empty_like(r) if out is None else self._map(out, "out")
        _check(self._lib.arkcos_convolve_adjoint(self.handle, ctypes.c_void_p(r.data_ptr()),
                                                 ctypes.c_void_p(xb.data_ptr()), self._ws_ptr(ws),
                                                 _stream_ptr(stream)), "arkcos_convolve_adjoint")
        return xb

    def convolve_noalloc(self, x: torch.Tensor, out: torch.Tensor, stream=None):
        """y = C x with the library's fixed device scratch as the workspace
        (arkcos_convolve_noalloc: nothing is allocated; calls on one device
        must not overlap)."""
        x = self._map(x, "x")
        out = self._map(out, "out")
        _check(self._lib.arkcos_convolve_noalloc(self.handle, ctypes.c_void_p(x.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "arkcos_convolve_noalloc")
        return out

    def kernel_grad(self, x: torch.Tensor, r: torch.Tensor, out: Optional[torch.Tensor] = None,
                    ws=None, reuse_spectra: bool = False, stream=None):
        x = self._map(x, "x")
        r = self._map(r, "r")
        g = torch.empty(self.n_knots, dtype=torch.float64, device=x.device) if out is None else out
        _check(self._lib.arkcos_kernel_grad(self.handle, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                            self._ws_ptr(ws), 1 if reuse_spectra else 0,
                                            _stream_ptr(stream)), "arkcos_kernel_grad")
        return g

    def start_timing(self, max_calls: int):
        """Record per-stage HIP events for the next max_calls calls."""
        _check(self._lib.arkcos_plan_timing(self.handle, int(max_calls)), "arkcos_plan_timing")

    def stage_times(self):
        """(ms per stage summed over the recorded calls, number of calls)."""
        ms = (ctypes.c_double * 4)()
        calls = ctypes.c_int64()
        _check(self._lib.arkcos_stage_times(self.handle, ms, ctypes.byref(calls)), "arkcos_stage_times")
        return list(ms), int(calls.value)

    def set_knots(self, knots: Sequence[float]):
        """New knot values from the host (waits for the device)."""
        arr = (ctypes.c_double * self.n_knots)(*[float(v) for v in knots])
        _check(self._lib.arkcos_set_knots(self.handle, arr), "arkcos_set_knots")

    def set_knots_async(self, knots: torch.Tensor, stream=None):
        """New knot values from a device tensor of n_knots doubles, enqueued
        on the stream (no host synchronisation)."""
        if not isinstance(knots, torch.Tensor) or not knots.is_cuda or knots.dtype != torch.float64 \
                or knots.numel() != self.n_knots or not knots.is_contiguous():
            raise ArkcosError(f"knots must be a contiguous CUDA float64 tensor of {self.n_knots} values")
        _check(self._lib.arkcos_set_knots_async(self.handle, ctypes.c_void_p(knots.data_ptr()),
                                                _stream_ptr(stream)), "arkcos_set_knots_async")


def _profile(fwhm: float, knots, theta_max: float):
    """A ProfileC (and the knot array it points to, which must stay alive)."""
    if knots is not None:
        arr = (ctypes.c_double * len(knots))(*[float(v) for v in knots])
        ptr = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        return ProfileC(SPLINE, 0.0, len(knots), float(theta_max), ptr), arr
    return ProfileC(GAUSSIAN, float(fwhm), 0, 0.0, None), None


def truncation_variance(radius: float, cl, *, fwhm: float = 0.0, knots=None, theta_max: float = 0.0):
    """sigma^2(R) of the kernel cut at `radius` for a signal of power spectrum
    cl[0..lmax] (paper Sect. 4), and the Legendre coefficient changes dK_l.
    Host computation in libarkcos (no GPU needed)."""
    lib = load_library()
    c = np.ascontiguousarray(cl, dtype=np.float64)
    prof, keep = _profile(fwhm, knots, theta_max)
    out = ctypes.c_double()
    dk = np.empty(c.size, dtype=np.float64)
    _check(lib.arkcos_truncation_variance(ctypes.byref(prof), float(radius),
                                          c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), c.size - 1,
                                          ctypes.byref(out), dk.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "arkcos_truncation_variance")
    del keep
    return out.value, dk


def choose_radius(cl, target_sigma2: float, *, fwhm: float = 0.0, knots=None, theta_max: float = 0.0) -> float:
    """Smallest support radius whose truncation variance is at most
    target_sigma2 (paper Sect. 4).  Host computation in libarkcos."""
    lib = load_library()
    c = np.ascontiguousarray(cl, dtype=np.float64)
    prof, keep = _profile(fwhm, knots, theta_max)
    out = ctypes.c_double()
    _check(lib.arkcos_choose_radius(ctypes.byref(prof), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    c.size - 1, float(target_sigma2), ctypes.byref(out)), "arkcos_choose_radius")
    del keep
    return out.value


class Batch:
    """Many plans (same dtype) convolved together: batched ring transforms and
    one persistent accumulation launch over a shared work queue.  With
    shared_input=True the plans share one geometry and one input map
    (convolve_shared): its spectra are computed once for every kernel."""

    def __init__(self, plans: Sequence[Plan], shared_input: bool = False):
        lib = load_library()
        self._lib = lib
        self.plans = list(plans)
        self.shared_input = bool(shared_input)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        self.handle = ctypes.c_void_p()
        if self.shared_input:
            _check(lib.arkcos_batch_plan_shared_input(len(self.plans), arr, ctypes.byref(self.handle)),
                   "arkcos_batch_plan_shared_input")
        else:
            _check(lib.arkcos_batch_plan(len(self.plans), arr, ctypes.byref(self.handle)), "arkcos_batch_plan")
        info = BatchInfo()
        _check(lib.arkcos_batch_get_info(self.handle, ctypes.byref(info)), "arkcos_batch_get_info")
        self.info = info
        self._ws = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                self._lib.arkcos_batch_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def workspace_bytes(self) -> int:
        return int(self.info.workspace_bytes)

    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            dev = self.plans[0].device
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        return self._ws

    def convolve(self, xs: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]] = None,
                 adjoint: bool = False, ws=None, stream=None):
        if len(xs) != len(self.plans):
            raise ArkcosError("one input map per plan")
        xs = [p._map(x, f"x[{i}]") for i, (p, x) in enumerate(zip(self.plans, xs))]
        ys = [torch.empty_like(x) for x in xs] if outs is None else \
            [p._map(y, f"out[{i}]") for i, (p, y) in enumerate(zip(self.plans, outs))]
        wst = self.workspace() if ws is None else ws
        addr = (wst.data_ptr() + 255) // 256 * 256
        if addr + self.workspace_bytes > wst.data_ptr() + wst.numel():
            raise ArkcosError("workspace too small")
        xa = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        ya = (ctypes.c_void_p * len(ys))(*[y.data_ptr() for y in ys])
        _check(self._lib.arkcos_batch_convolve(self.handle, xa, ya, 1 if adjoint else 0, ctypes.c_void_p(addr),
                                               _stream_ptr(stream)), "arkcos_batch_convolve")
        return ys

    def convolve_shared(self, x: torch.Tensor, outs: Optional[Sequence[torch.Tensor]] = None, ws=None,
                        stream=None):
        """y[i] = C_i x for every plan i of a shared-input batch."""
        x = self.plans[0]._map(x, "x")
        ys = [torch.empty_like(x) for _ in self.plans] if outs is None else \
            [p._map(y, f"out[{i}]") for i, (p, y) in enumerate(zip(self.plans, outs))]
        wst = self.workspace() if ws is None else ws
        addr = (wst.data_ptr() + 255) // 256 * 256
        if addr + self.workspace_bytes > wst.data_ptr() + wst.numel():
            raise ArkcosError("workspace too small")
        ya = (ctypes.c_void_p * len(ys))(*[y.data_ptr() for y in ys])
        _check(self._lib.arkcos_batch_convolve_shared(self.handle, ctypes.c_void_p(x.data_ptr()), ya,
                                                      ctypes.c_void_p(addr), _stream_ptr(stream)),
               "arkcos_batch_convolve_shared")
        return ys

    def start_timing(self, max_calls: int):
        _check(self._lib.arkcos_batch_timing(self.handle, int(max_calls)), "arkcos_batch_timing")

    def stage_times(self):
        ms = (ctypes.c_double * 4)()
        calls = ctypes.c_int64()
        _check(self._lib.arkcos_batch_stage_times(self.handle, ms, ctypes.byref(calls)), "arkcos_batch_stage_times")
        return list(ms), int(calls.value)
