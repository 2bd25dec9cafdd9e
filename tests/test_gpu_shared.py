"""One map convolved with many kernels through one set of input spectra
(the shared-input batch): the way an asymmetric beam is applied once it is
split into about ten symmetric kernels (paper Sect. 5, on ASYMFAST).  Every
component must equal its own plan's convolution bit for bit (the same
kernels read the same spectrum values in the same order) and match the
FP64 direct sum of its kernel."""
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


def _components(nside, n=10, seed=5):
    """n symmetric components: Gaussians of 1.5 to 4 pixel widths, each cut at
    3 FWHM, and one 12-knot spline (a wavelet-like kernel)."""
    pix = math.sqrt(math.pi / 3) / nside
    rng = np.random.default_rng(seed)
    out = []
    for fw in np.linspace(1.5, 4.0, n - 1) * pix:
        out.append((W.Profile("gaussian", fwhm=float(fw)), 3.0 * float(fw)))
    tmax = 5.0 * pix
    th = np.arange(12) * tmax / 11
    kn = W.mexican_hat(th, tmax / 5) + 0.01 * rng.standard_normal(12)
    out.append((W.Profile("spline", theta_max=tmax, knots=tuple(float(v) for v in kn)), tmax))
    return out


def _plan(grid, prof, radius, dtype):
    from paper_1104_0672_amd import Plan
    if prof.kind == "gaussian":
        return Plan("healpix", radius, nside=grid.nside, fwhm=prof.fwhm, dtype=dtype)
    return Plan("healpix", radius, nside=grid.nside, knots=list(prof.knots), theta_max=prof.theta_max, dtype=dtype)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-8), ("f32", 1e-4)])
def test_shared_input_components_equal_their_plans_and_the_direct_sum(dtype, tol):
    from paper_1104_0672_amd import Batch
    grid = W.Grid("healpix", nside=64)
    comps = _components(grid.nside)
    print(f"case shared input nside {grid.nside} {dtype}, {len(comps)} kernels", flush=True)
    plans = [_plan(grid, p, r, dtype) for p, r in comps]
    batch = Batch(plans, shared_input=True)
    x64 = W.white_noise(grid.npix, 17)
    idx, amp = W.point_sources(grid.npix, 50, 17, loguniform=False)
    np.add.at(x64, idx, amp)
    x = torch.tensor(x64, dtype=torch.float32 if dtype == "f32" else torch.float64, device="cuda")
    ys = batch.convolve_shared(x)
    ys2 = batch.convolve_shared(x)  # a second call reuses the workspace
    for k, ((prof, R), p, y, y2) in enumerate(zip(comps, plans, ys, ys2)):
        assert torch.equal(y, p.convolve(x)) and torch.equal(y, y2), k
        yh = y.cpu().numpy().astype(np.float64)
        if prof.kind == "gaussian":
            ref = oracle.direct(grid, prof, R, x64)
            what, bound = "FP64 direct sum", tol
        else:
            # the spline is cut with a step at theta_max, which the cap pairs'
            # trigonometric interpolation resolves only to ~1e-3 at this
            # oversampling: the reference is the FP64 step-by-step method
            ref = oracle.hybrid(grid, prof, R, x64, oversample=p.info.oversample)
            what, bound = "FP64 step-by-step method", 1e-10 if dtype == "f64" else 1e-5
        e = float(np.linalg.norm(yh - ref) / np.linalg.norm(ref))
        print(f"  component {k} ({prof.kind}): fractional RMS vs {what} {e:.2e}", flush=True)
        assert e <= bound


def test_shared_input_argument_errors():
    from paper_1104_0672_amd import ArkcosError, Batch, Plan
    a = Plan("healpix", 0.1, nside=16, fwhm=0.03)
    b = Plan("healpix", 0.1, nside=32, fwhm=0.03)
    with pytest.raises(ArkcosError, match="one geometry"):
        Batch([a, b], shared_input=True)
    c = Plan("healpix", 0.15, nside=16, fwhm=0.05)
    sb = Batch([a, c], shared_input=True)
    x = torch.zeros(a.npix, dtype=torch.float32, device="cuda")
    with pytest.raises(ArkcosError, match="arkcos_batch_convolve_shared"):
        sb.convolve([x, x])
    ob = Batch([a, c])
    with pytest.raises(ArkcosError, match="shared_input"):
        ob.convolve_shared(x)
    with pytest.raises(ArkcosError, match="overlaps"):
        sb.convolve_shared(x, outs=[x, torch.empty_like(x)])
