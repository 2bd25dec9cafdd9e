"""Edge and degenerate cases of the HIP path."""
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


def _run(w, x, **kw):
    from paper_1104_0672_amd import Plan
    plan = Plan.from_workload(w, **kw)
    dt = torch.float64 if w.dtype == "f64" else torch.float32
    return plan, plan.convolve(torch.tensor(x, dtype=dt, device="cuda")).cpu().numpy().astype(np.float64)


def test_nside1_and_nside2():
    for nside in (1, 2):
        w = W.Workload("tiny", W.Grid("healpix", nside=nside), W.Profile("gaussian", fwhm=0.8), 2.0, "f64", 1)
        x = W.make_input(w)
        _, y = _run(w, x, oversample=4)
        ref = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=4)
        assert np.linalg.norm(y - ref) <= 1e-11 * np.linalg.norm(ref)


def test_support_smaller_than_ring_spacing_is_identity_times_weight():
    w = W.Workload("narrow", W.Grid("healpix", nside=16), W.Profile("gaussian", fwhm=1e-3), 1e-3, "f64", 2)
    x = W.make_input(w)
    _, y = _run(w, x)
    ref = x * 4 * math.pi / w.grid.npix
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_zero_kernel_gives_zero_map():
    prof = W.Profile("spline", theta_max=0.3, knots=tuple([0.0] * 8))
    w = W.Workload("zero", W.Grid("healpix", nside=8), prof, 0.3, "f32", 3)
    x = W.make_input(w)
    _, y = _run(w, x)
    assert np.all(y == 0.0)


def test_support_covering_almost_the_whole_sphere():
    g = W.Grid("ecp", ntheta=12, nphi=24)
    w = W.Workload("wide", g, W.Profile("gaussian", fwhm=2.0), 3.0, "f64", 4)
    x = W.make_input(w)
    _, y = _run(w, x)
    ref = oracle.direct(g, w.profile, w.radius, x)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


def test_fix_pole_pixels_off_matches_reference():
    w = W.scaled_healpix(16, 200.0, 3.0, dtype="f64", seed=5)
    x = W.make_input(w)
    _, y = _run(w, x, oversample=2, fix_pole_pixels=False)
    ref = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=2, fix_poles=False)
    assert np.linalg.norm(y - ref) <= 1e-11 * np.linalg.norm(ref)


def test_unsupported_sizes_are_rejected():
    """Ring FFTs run in one workgroup's LDS up to 16384 (FP32) or 8192 (FP64)
    complex points: the polar rings' Bluestein transforms stop nside 8192 in
    FP32 and nside 4096 in FP64."""
    from paper_1104_0672_amd import ArkcosError, Plan
    with pytest.raises(ArkcosError, match="NOT_SUPPORTED"):
        Plan("healpix", 0.002, nside=8192, fwhm=0.0005, dtype="f32")
    with pytest.raises(ArkcosError, match="NOT_SUPPORTED"):
        Plan("healpix", 0.004, nside=4096, fwhm=0.001, dtype="f64")


def test_aliasing_and_argument_errors():
    from paper_1104_0672_amd import ArkcosError, Plan
    plan = Plan("healpix", 0.2, nside=8, fwhm=0.1)
    x = torch.zeros(plan.npix, device="cuda")
    with pytest.raises(ArkcosError, match="INVALID_VALUE"):
        plan.convolve(x, out=x)
    with pytest.raises(ArkcosError):
        plan.kernel_grad(x, x)  # Gaussian plan has no knots
    with pytest.raises(ArkcosError):
        plan.convolve(torch.zeros(plan.npix + 1, device="cuda"))
