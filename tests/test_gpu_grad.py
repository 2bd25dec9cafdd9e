"""GPU checks of the transposed map and the kernel-profile gradient.

* FP64 plans: the knot gradient equals the gradient of the step-by-step FP64
  hybrid reference, and central differences of the GPU loss (the loss is
  quadratic in the knots, so they are exact up to rounding);
* FP32 plans: the same within FP32 accuracy;
* autograd: torch.autograd.gradcheck-style comparison of both gradients.
"""
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


def _spline_workload(nside, n_knots, dtype, seed):
    pix = math.sqrt(math.pi / 3) / nside
    tmax = 5.0 * pix
    th = np.arange(n_knots) * tmax / (n_knots - 1)
    rng = np.random.default_rng(seed)
    c = W.mexican_hat(th, tmax / 5) + 0.01 * rng.standard_normal(n_knots)
    prof = W.Profile("spline", theta_max=tmax, knots=tuple(float(v) for v in c))
    return W.Workload(f"spline{nside}", W.Grid("healpix", nside=nside), prof, tmax, dtype, seed)


def _t(a, dtype):
    return torch.tensor(a, dtype=torch.float64 if dtype == "f64" else torch.float32, device="cuda")


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
def test_knot_gradient_matches_hybrid_reference(dtype, tol):
    from paper_1104_0672_amd import Plan
    w = _spline_workload(8, 10, dtype, 3)
    print(f"case knot gradient {w.name} {dtype}", flush=True)
    plan = Plan.from_workload(w, oversample=2)
    rng = np.random.default_rng(5)
    x, t = rng.standard_normal(w.grid.npix), rng.standard_normal(w.grid.npix)
    y = plan.convolve(_t(x, dtype)).double().cpu().numpy()
    r = y - t
    g = plan.kernel_grad(_t(x, dtype), _t(r, dtype)).cpu().numpy()
    ref = oracle.hybrid_knot_grad(w.grid, w.profile, w.radius, x, r, oversample=2)
    assert np.linalg.norm(g - ref) <= tol * np.linalg.norm(ref), (g, ref)


def test_knot_gradient_central_differences_fp64():
    from paper_1104_0672_amd import Plan
    w = _spline_workload(16, 12, "f64", 4)
    print(f"case knot gradient FD {w.name}", flush=True)
    plan = Plan.from_workload(w, oversample=2)
    rng = np.random.default_rng(6)
    x, t = _t(rng.standard_normal(w.grid.npix), "f64"), _t(rng.standard_normal(w.grid.npix), "f64")
    c = np.asarray(w.profile.knots)
    r = plan.convolve(x) - t
    g = plan.kernel_grad(x, r).cpu().numpy()
    h = 1e-3
    for k in (0, 3, 7, 11):
        e = np.zeros_like(c)
        e[k] = h
        plan.set_knots(c + e)
        lp = 0.5 * float(((plan.convolve(x) - t) ** 2).sum())
        plan.set_knots(c - e)
        lm = 0.5 * float(((plan.convolve(x) - t) ** 2).sum())
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-8 * max(1.0, abs(g[k])), (k, fd, g[k])
    plan.set_knots(c)


def test_knot_gradient_reuses_forward_spectra():
    from paper_1104_0672_amd import Plan
    w = _spline_workload(8, 8, "f64", 7)
    plan = Plan.from_workload(w)
    rng = np.random.default_rng(8)
    x, r = _t(rng.standard_normal(w.grid.npix), "f64"), _t(rng.standard_normal(w.grid.npix), "f64")
    ws = torch.empty(plan.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
    plan.convolve(x, ws=ws)
    g1 = plan.kernel_grad(x, r, ws=ws, reuse_spectra=True)
    g2 = plan.kernel_grad(x, r)
    assert torch.allclose(g1, g2, rtol=1e-13, atol=0)


def test_autograd_function():
    from paper_1104_0672_amd import Plan, convolve
    w = _spline_workload(8, 8, "f64", 9)
    plan = Plan.from_workload(w)
    rng = np.random.default_rng(10)
    x = _t(rng.standard_normal(w.grid.npix), "f64").requires_grad_(True)
    knots = torch.tensor(w.profile.knots, dtype=torch.float64, device="cuda", requires_grad=True)
    target = _t(rng.standard_normal(w.grid.npix), "f64")
    for keep in (True, False):
        y = convolve(x, plan, knots, keep_spectra=keep)
        loss = 0.5 * ((y - target) ** 2).sum()
        gx, gk = torch.autograd.grad(loss, (x, knots))
        r = (y - target).detach()
        assert torch.allclose(gx, plan.adjoint(r), rtol=1e-12, atol=1e-15)
        assert torch.allclose(gk, plan.kernel_grad(x.detach(), r), rtol=1e-12, atol=1e-15)
    # directional derivative of the loss in x, by central differences
    v = _t(rng.standard_normal(w.grid.npix), "f64")
    eps = 1e-4
    with torch.no_grad():
        lp = 0.5 * ((plan.convolve(x + eps * v) - target) ** 2).sum()
        lm = 0.5 * ((plan.convolve(x - eps * v) - target) ** 2).sum()
    fd = float((lp - lm) / (2 * eps))
    assert abs(fd - float((gx * v).sum())) <= 1e-8 * abs(fd)
