"""The largest grids a plan takes: HEALPix nside 4096 in FP32 and nside
2048 in FP64, whose polar rings need Bluestein transforms of 16384 (FP32)
and 8192 (FP64) complex points held in one workgroup's LDS (paper Sect. 5
looks ahead to nside >= 4096).  Sampled output pixels, the poles' rings
among them, against the FP64 direct sum."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _frac(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _sampled_check(w, dtype, tol, count):
    from paper_1104_0672_amd import Plan
    x = W.make_input(w)
    plan = Plan.from_workload(w, dtype=dtype)
    td = torch.float32 if dtype == "f32" else torch.float64
    y = plan.convolve(torch.tensor(x, dtype=td, device="cuda")).cpu().numpy().astype(np.float64)
    npix = w.grid.npix
    # random pixels, the first and last rings' neighbourhoods, and the pixels
    # around the brightest sources (where the signal is)
    ends = list(range(0, 2000)) + list(range(npix - 2000, npix))
    idx = W.sample_pixels(npix, count, w.seed, must_include=ends)
    ref = oracle.direct(w.grid, w.profile, w.radius, x, idx=idx)
    e = _frac(y[idx], ref)
    src, amp = W.point_sources(npix, 8000 if w.grid.nside == 4096 else 2000, w.seed, loguniform=True)
    if not w.name.startswith("healpix2048") and not w.name.startswith("healpix4096"):
        src, amp = np.argsort(-np.abs(x))[:30], np.abs(x)[np.argsort(-np.abs(x))[:30]]
    near = np.unique(np.concatenate([np.arange(max(0, q - 8), min(npix, q + 9)) for q in src[np.argsort(-amp)[:30]]]))
    e_near = _frac(y[near], oracle.direct(w.grid, w.profile, w.radius, x, idx=near))
    print(f"  {w.name} {dtype}: oversample {plan.info.oversample}, fractional RMS on {idx.size} pixels {e:.2e}, "
          f"source neighbourhoods {e_near:.2e}", flush=True)
    assert e <= tol and e_near <= tol
    return plan


def test_healpix4096_fp32_sampled():
    w = W.healpix4096()
    print(f"case {w.name} FP32", flush=True)
    _sampled_check(w, "f32", 1e-4, 20000)


def test_healpix2048_fp64_sampled():
    w = W.healpix2048()
    print(f"case {w.name} FP64", flush=True)
    _sampled_check(w, "f64", 1e-9, 8000)


def test_healpix768_mixed_radix_belt_fp32():
    """nside 768 = 3 * 256: the 1537 equatorial rings have 3072 pixels, a
    1536-point complex FFT of radices 16, 16, 2 and 3 (the mixed-radix path,
    enough rings to fill its own launches); sampled against the direct sum."""
    w = W.scaled_healpix(768, fwhm_arcmin=8.0, radius_fwhm=3.0, seed=17)
    print(f"case {w.name} FP32", flush=True)
    _sampled_check(w, "f32", 1e-4, 8000)
