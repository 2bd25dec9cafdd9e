"""Oracle for the radial-kernel sphere convolution (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never links, calls or
reads anything here, and nothing here uses the HIP library.

Two references live here:

* ``direct`` / ``adjoint`` / ``knot_grad`` -- the plain definition: the FP64
  brute-force direct sum ``y_p = sum_q K(theta_pq) x_q w_q`` (paper Sect. 2,
  eq. "def"; Sect. 3.1, eq. "direct"), its explicit transpose and the exact
  knot gradient, in C with OpenMP (``direct.c``).
* ``hybrid`` -- the paper's hybrid algorithm (Sect. 4.1 and the
  artifact-suppressed variant of Sect. 4.3), step by step in FP64 with numpy
  FFTs as library primitives.  It is the oracle where the method is an
  approximation (HEALPix pairs that involve a polar ring) and must equal the
  direct sum where the method is exact (ECP grids, equatorial HEALPix pairs).
* ``truncation_variance`` -- the truncation error of the support radius of
  Sect. 4 from its definition (``truncation.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

SUPPORT_TOL = 1e-9


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64, i32, dbl, ptr = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
            lib.oracle_npix.restype = i64
            lib.oracle_npix.argtypes = [i32, i64, i64, i64]
            lib.oracle_rings.argtypes = [i32, i64, i64, i64, ptr, ptr, ptr, ptr, ptr]
            lib.oracle_kernel.argtypes = [i32, dbl, i32, dbl, ptr, dbl, ptr, ptr, i64]
            lib.oracle_basis.argtypes = [i32, dbl, ptr, dbl, ptr, ptr, i64]
            conv = [i32, i64, i64, i64, i32, dbl, i32, dbl, ptr, dbl, ptr, ptr, ptr, i64, i32]
            lib.oracle_convolve.argtypes = conv
            lib.oracle_adjoint.argtypes = conv
            lib.oracle_knot_grad.argtypes = [i32, i64, i64, i64, i32, dbl, ptr, dbl, ptr, ptr, ptr,
                                             ptr, i64, i32]
            lib.oracle_neighbour_count.argtypes = [i32, i64, i64, i64, dbl, ptr, i64, ptr, ptr]
            for f in (lib.oracle_rings, lib.oracle_kernel, lib.oracle_basis, lib.oracle_convolve,
                      lib.oracle_adjoint, lib.oracle_knot_grad, lib.oracle_neighbour_count):
                f.restype = i32
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _grid_args(grid):
    if grid.kind == "ecp":
        return (0, 0, grid.ntheta, grid.nphi)
    return (1, grid.nside, 0, 0)


def _prof_args(profile):
    if profile.kind == "gaussian":
        return (0, float(profile.fwhm), 0, 0.0, None)
    knots = np.ascontiguousarray(profile.knots, dtype=np.float64)
    return (1, 0.0, len(knots), float(profile.theta_max), knots)


# ------------------------------------------------------------------ tables

def rings(grid):
    """Ring table (theta, phi0, w, n, start) of an ECP or HEALPix grid."""
    lib = _load()
    nr = grid.nrings
    th, ph, w = (np.empty(nr) for _ in range(3))
    n, st = np.empty(nr, np.int64), np.empty(nr, np.int64)
    rc = lib.oracle_rings(*_grid_args(grid), _p(th), _p(ph), _p(w), _p(n), _p(st))
    if rc:
        raise ValueError("bad grid")
    return th, ph, w, n, st


def pixel_angles(grid):
    """(theta, phi) of every pixel, RING order."""
    th, ph0, _, n, st = rings(grid)
    theta = np.repeat(th, n)
    k = np.arange(grid.npix) - np.repeat(st, n)
    phi = np.repeat(ph0, n) + 2.0 * np.pi * k / np.repeat(n, n)
    return theta, phi


def pixel_weights(grid):
    th, _, w, n, _ = rings(grid)
    return np.repeat(w, n)


def kernel(profile, radius, t):
    """K(t) with the truncation at ``radius`` (+1e-9 rad)."""
    lib = _load()
    t = np.ascontiguousarray(t, dtype=np.float64)
    out = np.empty_like(t)
    pk, fwhm, nk, tmax, knots = _prof_args(profile)
    if lib.oracle_kernel(pk, fwhm, nk, tmax, _p(knots), float(radius), _p(t), _p(out), t.size):
        raise ValueError("bad profile")
    return out


def basis(profile, radius, t):
    """phi_k(t), shape (len(t), n_knots), for a spline profile."""
    lib = _load()
    t = np.ascontiguousarray(t, dtype=np.float64)
    knots = np.ascontiguousarray(profile.knots, dtype=np.float64)
    out = np.empty((t.size, len(knots)))
    if lib.oracle_basis(len(knots), float(profile.theta_max), _p(knots), float(radius), _p(t),
                        _p(out), t.size):
        raise ValueError("bad profile")
    return out


# ------------------------------------------------------------- direct sums

def _run(fn, grid, profile, radius, vec, idx, nthreads):
    vec = np.ascontiguousarray(vec, dtype=np.float64)
    if vec.size != grid.npix:
        raise ValueError("map size does not match the grid")
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.empty(idx.size)
        nidx = idx.size
    else:
        out = np.empty(grid.npix)
        nidx = 0
    pk, fwhm, nk, tmax, knots = _prof_args(profile)
    rc = fn(*_grid_args(grid), pk, fwhm, nk, tmax, _p(knots), float(radius), _p(vec), _p(out),
            _p(idx), nidx, int(nthreads))
    if rc:
        raise ValueError("oracle rejected its arguments")
    return out


def direct(grid, profile, radius, x, idx=None, nthreads=0):
    """y_p = sum_{theta_pq <= R} K(theta_pq) x_q w_q (all pixels, or those in idx)."""
    return _run(_load().oracle_convolve, grid, profile, radius, x, idx, nthreads)


def adjoint(grid, profile, radius, r, idx=None, nthreads=0):
    """xbar_q = w_q sum_{theta_pq <= R} K(theta_pq) r_p, the explicit transpose."""
    return _run(_load().oracle_adjoint, grid, profile, radius, r, idx, nthreads)


def knot_grad(grid, profile, radius, x, r, idx=None, nthreads=0):
    """g_k = sum_p r_p sum_q phi_k(theta_pq) x_q w_q for a spline profile."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    knots = np.ascontiguousarray(profile.knots, dtype=np.float64)
    g = np.empty(len(knots))
    nidx = 0
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        nidx = idx.size
    rc = lib.oracle_knot_grad(*_grid_args(grid), len(knots), float(profile.theta_max), _p(knots),
                              float(radius), _p(x), _p(r), _p(g), _p(idx), nidx, int(nthreads))
    if rc:
        raise ValueError("oracle rejected its arguments")
    return g


def neighbour_stats(grid, radius, idx):
    """Support size of each listed pixel, and the smallest distance
    |theta_pq - (R + 1e-9)| of any visited pair to the inclusion threshold."""
    lib = _load()
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    cnt = np.empty(idx.size, np.int64)
    gap = np.zeros(1)
    if lib.oracle_neighbour_count(*_grid_args(grid), float(radius), _p(idx), idx.size, _p(cnt), _p(gap)):
        raise ValueError("bad grid")
    return cnt, float(gap[0])


from .hybrid import hybrid, hybrid_adjoint, hybrid_knot_grad, pair_plan  # noqa: E402,F401
from .truncation import truncation_variance  # noqa: E402,F401
