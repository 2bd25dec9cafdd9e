"""Support radius chosen at plan time from a truncation-error target
(paper Sect. 4): arkcos_plan_for_error picks the radius arkcos_choose_radius
returns for the caller's C_l and target variance, and the plan it builds
convolves with that radius, checked against the FP64 oracle's truncation
variance (the chosen R meets the target, a slightly smaller one does not)
and against the FP64 direct sum at that radius."""
import math

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


def test_plan_for_error_chooses_the_radius_and_convolves_with_it():
    from paper_1104_0672_amd import Plan, choose_radius
    nside = 64
    fw = 3.0 * math.sqrt(math.pi / 3) / nside  # three pixel widths
    sig = fw * W.FWHM_TO_SIGMA
    prof = W.Profile("gaussian", fwhm=fw)
    l = np.arange(3 * nside + 1)
    cl = 1.0 / (l + 10.0) ** 2
    hi, _ = oracle.truncation_variance(prof, 2.5 * sig, cl)
    lo, _ = oracle.truncation_variance(prof, 3.5 * sig, cl)
    target = math.sqrt(hi * lo)
    plan = Plan("healpix", None, nside=nside, fwhm=fw, dtype="f64", cl=cl, target_sigma2=target)
    R = plan.info.support_radius_rad
    print(f"case nside {nside}, fwhm {fw:.4e}: chosen R = {R / sig:.4f} sigma", flush=True)
    assert R == choose_radius(cl, target, fwhm=fw)
    assert 2.5 * sig < R < 3.5 * sig
    assert oracle.truncation_variance(prof, R, cl)[0] <= target * (1 + 1e-6)
    assert oracle.truncation_variance(prof, R * (1 - 1e-4), cl)[0] > target
    # the plan convolves with that radius: against the step-by-step method at
    # R (exact up to rounding), and, printed, the direct sum at R (the kernel
    # is cut where K(R) ~ 1e-2, a step that the trigonometric interpolation of
    # the cap pairs' kernel rows resolves only to ~1e-3 at this oversampling)
    grid = W.Grid("healpix", nside=nside)
    x = W.white_noise(grid.npix, 11)
    y = plan.convolve(torch.tensor(x, dtype=torch.float64, device="cuda")).cpu().numpy()
    ref_h = oracle.hybrid(grid, prof, R, x, oversample=plan.info.oversample)
    e_h = float(np.linalg.norm(y - ref_h) / np.linalg.norm(ref_h))
    ref = oracle.direct(grid, prof, R, x)
    e = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    print(f"  fractional RMS vs the FP64 step-by-step method at R {e_h:.2e}, vs the direct sum {e:.2e}",
          flush=True)
    assert e_h <= 1e-11
    # a plan at a clearly different radius differs by far more
    other = Plan("healpix", 1.5 * R, nside=nside, fwhm=fw, dtype="f64")
    y2 = other.convolve(torch.tensor(x, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert float(np.linalg.norm(y2 - ref_h) / np.linalg.norm(ref_h)) > 1e-4


def test_plan_for_error_rejects_a_target_met_without_support():
    from paper_1104_0672_amd import ArkcosError, Plan
    l = np.arange(65)
    with pytest.raises(ArkcosError, match="without any kernel support"):
        Plan("healpix", None, nside=16, fwhm=0.05, cl=1.0 / (l + 1.0) ** 2, target_sigma2=1e6)
    with pytest.raises(ArkcosError, match="target"):
        Plan("healpix", None, nside=16, fwhm=0.05, cl=np.ones(8), target_sigma2=-1.0)
