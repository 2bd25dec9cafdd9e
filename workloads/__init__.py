"""Seeded synthetic inputs for the radial-kernel sphere convolution.

This module is shared by the tests, the benchmark and the smoke check.  It
holds input recipes only: grid sizes, kernel parameters, random maps, point
source positions and amplitudes, and spline knot values.  No step of the
convolution (geometry, distances, transforms, sums) lives here, so the oracle
and the HIP path both draw their inputs from it without sharing arithmetic.

The workloads stand in for the paper's synthetic Planck-like runs (Sect. 4.2,
Gaussian beams on HEALPix maps at nside 2048, and the point-source ringing test
of Sect. 4.3); the paper uses no public dataset.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ARCMIN = math.pi / (180.0 * 60.0)
FWHM_TO_SIGMA = 1.0 / math.sqrt(8.0 * math.log(2.0))


@dataclasses.dataclass(frozen=True)
class Grid:
    """An isolatitude-ring grid: ``kind`` is "ecp" or "healpix"."""

    kind: str
    nside: int = 0
    ntheta: int = 0
    nphi: int = 0

    @property
    def npix(self) -> int:
        if self.kind == "healpix":
            return 12 * self.nside * self.nside
        return self.ntheta * self.nphi

    @property
    def nrings(self) -> int:
        if self.kind == "healpix":
            return 4 * self.nside - 1
        return self.ntheta


@dataclasses.dataclass(frozen=True)
class Profile:
    """Radial kernel profile.

    ``kind`` is "gaussian" (peak-one ``exp(-t^2 / 2 sigma^2)`` with
    ``sigma = fwhm / sqrt(8 ln 2)``) or "spline" (clamped cubic spline through
    ``knots`` at equispaced angles ``k * theta_max / (n - 1)``).
    """

    kind: str
    fwhm: float = 0.0
    theta_max: float = 0.0
    knots: Optional[tuple] = None


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    grid: Grid
    profile: Profile
    radius: float          # support radius in radians
    dtype: str             # "f32" or "f64"
    seed: int


def gaussian(fwhm_arcmin: float) -> Profile:
    return Profile("gaussian", fwhm=fwhm_arcmin * ARCMIN)


# --------------------------------------------------------------------------
# Random draws
# --------------------------------------------------------------------------

def white_noise(npix: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """N(0, scale^2) map, float64, from ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(npix)


def point_sources(npix: int, count: int, seed: int, loguniform: bool):
    """Seeded point sources: pixel indices uniform in [0, npix) and amplitudes
    (1.0, or 10**U(-3, 0) when ``loguniform``).  Equal-area pixels make a
    uniform pixel index a uniform position on the sphere."""
    rng = np.random.default_rng(seed + 1_000_003)
    idx = rng.integers(0, npix, size=count)
    if loguniform:
        amp = 10.0 ** rng.uniform(-3.0, 0.0, size=count)
    else:
        amp = np.ones(count)
    return idx, amp


def mexican_hat(theta: np.ndarray, a: float) -> np.ndarray:
    u = theta * theta / (2.0 * a * a)
    return (1.0 - u) * np.exp(-u)


def mexican_hat_knots(seed: int, n_knots: int = 64, theta_max: float = 40.0 * ARCMIN,
                      a: float = 8.0 * ARCMIN, noise: float = 0.01) -> np.ndarray:
    """Knot values of the wavelet-like spline kernel: the Mexican-hat profile
    at equispaced knots plus seeded N(0, noise^2) perturbations."""
    th = np.arange(n_knots) * theta_max / (n_knots - 1)
    rng = np.random.default_rng(seed + 2_000_003)
    return mexican_hat(th, a) + noise * rng.standard_normal(n_knots)


def make_input(w: Workload) -> np.ndarray:
    """The input map of a named workload, as float64 (cast by the caller)."""
    npix = w.grid.npix
    if w.name.startswith("healpix256"):
        x = white_noise(npix, w.seed)
        idx, amp = point_sources(npix, 200, w.seed, loguniform=False)
        np.add.at(x, idx, amp)
        return x
    if w.name.startswith("healpix2048") or w.name.startswith("healpix4096"):
        x = white_noise(npix, w.seed, scale=1e-4)
        idx, amp = point_sources(npix, 2000 if w.grid.nside == 2048 else 8000, w.seed, loguniform=True)
        np.add.at(x, idx, amp)
        return x
    return white_noise(npix, w.seed)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def ecp_64x128() -> Workload:
    """ECP 64 x 128, FP64, Gaussian FWHM = 3 pixel widths (pi/64 each),
    truncated at 3 FWHM."""
    pix = math.pi / 64.0
    return Workload("ecp64x128", Grid("ecp", ntheta=64, nphi=128),
                    Profile("gaussian", fwhm=3.0 * pix), 9.0 * pix, "f64", 1)


def healpix256() -> Workload:
    """HEALPix nside 256, FP32, 30' Gaussian truncated at 90', white noise plus
    200 unit point sources."""
    return Workload("healpix256_30arcmin", Grid("healpix", nside=256), gaussian(30.0),
                    90.0 * ARCMIN, "f32", 2)


def healpix2048() -> Workload:
    """HEALPix nside 2048, FP32, 5' Gaussian truncated at 20' (Planck-HFI-like),
    1e-4 white noise plus 2000 log-uniform point sources."""
    return Workload("healpix2048_5arcmin", Grid("healpix", nside=2048), gaussian(5.0),
                    20.0 * ARCMIN, "f32", 3)


def healpix4096() -> Workload:
    """HEALPix nside 4096 (201,326,592 pixels), FP32, the same 5' Gaussian
    cut at 20' as the nside-2048 workload (a higher-resolution channel, the
    scale the paper's Sect. 5 looks ahead to), with the same input recipe."""
    return Workload("healpix4096_5arcmin", Grid("healpix", nside=4096), gaussian(5.0),
                    20.0 * ARCMIN, "f32", 6)


def healpix1024_spline(n_knots: int = 64) -> Workload:
    """HEALPix nside 1024, FP32, 64-knot spline kernel on [0, 40']."""
    knots = mexican_hat_knots(4, n_knots)
    prof = Profile("spline", theta_max=40.0 * ARCMIN, knots=tuple(float(v) for v in knots))
    return Workload("healpix1024_spline", Grid("healpix", nside=1024), prof, 40.0 * ARCMIN, "f32", 4)


def batch256(n_maps: int = 256, seed: int = 5) -> List[Workload]:
    """Many maps of uneven size: nside from {512, 1024, 2048} with weights
    0.5/0.3/0.2, FWHM uniform in [4', 30'], support radius 3 FWHM."""
    rng = np.random.default_rng(seed)
    nsides = rng.choice([512, 1024, 2048], size=n_maps, p=[0.5, 0.3, 0.2])
    fwhm = rng.uniform(4.0, 30.0, size=n_maps)
    out = []
    for k in range(n_maps):
        out.append(Workload(f"batch{k}", Grid("healpix", nside=int(nsides[k])),
                            gaussian(float(fwhm[k])), 3.0 * float(fwhm[k]) * ARCMIN,
                            "f32", seed * 100_000 + k))
    return out


def scaled_healpix(nside: int, fwhm_arcmin: float, radius_fwhm: float, dtype: str = "f32",
                   seed: int = 7) -> Workload:
    """A smaller HEALPix case with the same shape of kernel, for parity tests."""
    return Workload(f"healpix{nside}_{fwhm_arcmin:g}arcmin", Grid("healpix", nside=nside),
                    gaussian(fwhm_arcmin), radius_fwhm * fwhm_arcmin * ARCMIN, dtype, seed)


def sample_pixels(npix: int, count: int, seed: int, must_include: Sequence[int] = ()) -> np.ndarray:
    """Sorted distinct output-pixel indices for sampled parity checks."""
    rng = np.random.default_rng(seed + 3_000_017)
    idx = rng.choice(npix, size=min(count, npix), replace=False)
    idx = np.union1d(idx, np.asarray(must_include, dtype=np.int64))
    return np.sort(idx.astype(np.int64))
