"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (fractional RMS = |y - y_ref|_2 / |y_ref|_2, the paper's accuracy
measure, Sect. 4.3):
* ECP, FP64: <= 1e-12 and max |dy| <= 1e-11 max |y_ref|, against the direct
  sum (the ring FFT form is exact there, Sect. 4.3 last paragraph);
* ECP, FP32: <= 1e-6 against the direct sum;
* HEALPix, FP32: <= 1e-4 against the direct sum; against the step-by-step
  FP64 hybrid reference (same method) <= 1e-5;
* HEALPix, FP64: <= 1e-11 against the step-by-step hybrid reference (same
  oversampling), which checks the method itself, caps included.
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


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _plan(w, **kw):
    from paper_1104_0672_amd import Plan
    return Plan.from_workload(w, **kw)


def _tt(x, w):
    return torch.tensor(x, dtype=torch.float32 if w.dtype == "f32" else torch.float64, device=_dev())


def _frac(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(w, x, **kw):
    plan = _plan(w, **kw)
    y = plan.convolve(_tt(x, w))
    torch.cuda.synchronize()
    return plan, y.cpu().numpy().astype(np.float64)


def _say(msg):
    print(msg, flush=True)


def test_ecp_64x128_fp64_is_exact():
    w = W.ecp_64x128()
    _say(f"case {w.name} f64")
    x = W.make_input(w)
    _, y = _run(w, x)
    ref = oracle.direct(w.grid, w.profile, w.radius, x)
    assert _frac(y, ref) <= 1e-12
    assert np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("kgen", [0, 1, 2])
def test_ecp_fp32_all_kernel_sources(kgen):
    w = W.Workload("ecp64x128_f32", W.Grid("ecp", ntheta=64, nphi=128),
                   W.Profile("gaussian", fwhm=3 * math.pi / 64), 9 * math.pi / 64, "f32", 1)
    _say(f"case {w.name} kgen={kgen}")
    x = W.make_input(w)
    _, y = _run(w, x, kgen=kgen)
    ref = oracle.direct(w.grid, w.profile, w.radius, x)
    assert _frac(y, ref) <= 1e-6


@pytest.mark.parametrize("ntheta,nphi", [(1, 4), (3, 10), (17, 96), (40, 200)])
def test_ecp_ragged_shapes_fp64(ntheta, nphi):
    """Odd ring counts (self-mirrored middle ring), tiny rings, non-power-of-
    two ring lengths (Bluestein)."""
    g = W.Grid("ecp", ntheta=ntheta, nphi=nphi)
    prof = W.Profile("gaussian", fwhm=2.5 * math.pi / max(ntheta, 2))
    w = W.Workload("ecp_ragged", g, prof, min(3.0, 3 * prof.fwhm), "f64", 9)
    _say(f"case ecp {ntheta}x{nphi} f64")
    x = W.make_input(w)
    _, y = _run(w, x)
    ref = oracle.direct(g, prof, w.radius, x)
    assert _frac(y, ref) <= 1e-12


@pytest.mark.parametrize("nphi", [96, 120, 420, 1000, 1260, 3072])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_ecp_mixed_radix_ring_lengths(nphi, dtype, tol):
    """Rings whose half length has no prime factor above 7 take the
    mixed-radix transform (radices 2-16, 3, 5, 7; e.g. 210 = 2 3 5 7): exact
    against the direct sum on ECP grids, where the method is exact."""
    g = W.Grid("ecp", ntheta=12, nphi=nphi)
    prof = W.Profile("gaussian", fwhm=2.5 * math.pi / 12)
    w = W.Workload(f"ecp12x{nphi}", g, prof, 3 * prof.fwhm, dtype, 13)
    _say(f"case ecp 12x{nphi} {dtype}")
    x = W.make_input(w)
    _, y = _run(w, x)
    ref = oracle.direct(g, prof, w.radius, x)
    assert _frac(y, ref) <= tol


@pytest.mark.parametrize("nside,p", [(4, 2), (16, 1), (16, 2), (40, 2), (24, 4)])
def test_healpix_fp64_matches_step_by_step_method(nside, p):
    w = W.scaled_healpix(nside, fwhm_arcmin=2.5 * 60 * math.degrees(math.sqrt(math.pi / 3) / nside),
                         radius_fwhm=3.0, dtype="f64", seed=nside)
    _say(f"case {w.name} f64 p={p}")
    x = W.make_input(w)
    _, y = _run(w, x, oversample=p)
    ref = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=p)
    assert _frac(y, ref) <= 1e-11


@pytest.mark.parametrize("nside", [8, 32, 64])
def test_healpix_fp32_small(nside):
    w = W.scaled_healpix(nside, fwhm_arcmin=2.0 * 60 * math.degrees(math.sqrt(math.pi / 3) / nside),
                         radius_fwhm=3.0, seed=nside)
    _say(f"case {w.name} f32")
    x = W.make_input(w)
    plan, y = _run(w, x)
    p = plan.info.oversample
    ref_m = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=p)
    ref_d = oracle.direct(w.grid, w.profile, w.radius, x)
    assert _frac(y, ref_m) <= 1e-5
    assert _frac(y, ref_d) <= 1e-4


def test_healpix_fp32_wide_beam_oversample_one():
    """A beam of five pixels: the automatic kernel grid is the paper's
    (oversample 1), where an equatorial ring's own grid is also the fine
    grid."""
    w = W.scaled_healpix(32, fwhm_arcmin=5.0 * 60 * math.degrees(math.sqrt(math.pi / 3) / 32),
                         radius_fwhm=3.0, seed=77)
    _say(f"case {w.name} f32 wide beam")
    x = W.make_input(w)
    plan, y = _run(w, x)
    assert plan.info.oversample == 1
    ref_m = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=1)
    ref_d = oracle.direct(w.grid, w.profile, w.radius, x)
    assert _frac(y, ref_m) <= 1e-5
    assert _frac(y, ref_d) <= 1e-4


def test_healpix256_30arcmin_full_map():
    w = W.healpix256()
    _say(f"case {w.name}")
    x = W.make_input(w)
    plan, y = _run(w, x)
    ref = oracle.direct(w.grid, w.profile, w.radius, x)
    err = _frac(y, ref)
    _say(f"  oversample {plan.info.oversample}: fractional RMS vs direct sum {err:.3e}")
    assert err <= 1e-4


def test_accumulation_shapes_are_bitwise_equal():
    """Every accumulation shape (units per band, mode tiles per item, units
    per wavefront) sums each unit's pairs in the same order, so the forward
    and transposed maps are the same to the bit; the first shape's forward is
    also checked against the direct sum."""
    import os
    w = W.healpix256()
    _say(f"case accumulation shapes {w.name}")
    x = W.make_input(w)
    outs = []
    for shape in ("8,4", "8,2", "16,4", "16,4,2", "16,2,2", "24,2,3", "16,4,2,16"):
        os.environ["ARKCOS_ACC_SHAPE"] = shape
        try:
            plan = _plan(w)
        finally:
            del os.environ["ARKCOS_ACC_SHAPE"]
        info = plan.info
        want_upw = int(shape.split(",")[2]) if shape.count(",") >= 2 else 1
        _say(f"  shape {shape}: {info.acc_seg_units} units, {info.acc_group} tiles, "
             f"{info.acc_units_per_wave} per wave")
        assert info.acc_units_per_wave == want_upw and info.acc_seg_units == int(shape.split(",")[0])
        xt = _tt(x, w)
        outs.append((plan.convolve(xt).cpu(), plan.adjoint(xt).cpu()))
    for k in range(1, len(outs)):
        assert torch.equal(outs[k][0], outs[0][0]) and torch.equal(outs[k][1], outs[0][1])
    ref = oracle.direct(w.grid, w.profile, w.radius, x)
    assert _frac(outs[0][0].numpy().astype(np.float64), ref) <= 1e-4


@pytest.mark.parametrize("nside,fwhm_arcmin", [(16, 200.0), (64, 60.0), (512, 10.0)])
def test_accumulation_shapes_bitwise_equal_across_sizes(nside, fwhm_arcmin):
    """The multi-unit shapes on other sizes (ragged last bands, windows
    reaching the poles, short maps): bitwise equal to one unit per wave."""
    import os
    fw = math.radians(fwhm_arcmin / 60.0)
    w = W.Workload(f"healpix{nside}_{fwhm_arcmin:g}", W.Grid("healpix", nside=nside),
                   W.Profile("gaussian", fwhm=fw), 3.0 * fw, "f32", nside)
    _say(f"case accumulation shapes {w.name}")
    x = W.white_noise(w.grid.npix, nside)
    outs = []
    for shape in ("8,4", "16,2,2,16", "24,2,3", "16,4,2"):
        os.environ["ARKCOS_ACC_SHAPE"] = shape
        try:
            plan = _plan(w)
        finally:
            del os.environ["ARKCOS_ACC_SHAPE"]
        kinds = list(plan.info.pairs_by_kind)
        all_tab = kinds[0] + kinds[1] + kinds[3] == 0
        want = int(shape.split(",")[2]) if shape.count(",") >= 2 and all_tab else 1
        assert plan.info.acc_units_per_wave == want
        xt = _tt(x, w)
        outs.append((plan.convolve(xt).cpu(), plan.adjoint(xt).cpu()))
        _say(f"  shape {shape}: {plan.info.acc_seg_units} units, {plan.info.acc_units_per_wave} per wave")
    for k in range(1, len(outs)):
        assert torch.equal(outs[k][0], outs[0][0]) and torch.equal(outs[k][1], outs[0][1])


def test_fp64_adjoint_dot_product_and_transpose():
    for w in (W.ecp_64x128(), W.scaled_healpix(16, 200.0, 3.0, dtype="f64")):
        _say(f"case adjoint {w.name}")
        plan = _plan(w)
        rng = np.random.default_rng(21)
        x, r = rng.standard_normal(w.grid.npix), rng.standard_normal(w.grid.npix)
        cx = plan.convolve(_tt(x, w)).cpu().numpy()
        ct = plan.adjoint(_tt(r, w)).cpu().numpy()
        a, b = float(np.dot(cx, r)), float(np.dot(x, ct))
        assert abs(a - b) <= 1e-12 * np.linalg.norm(cx) * np.linalg.norm(r)
        if w.grid.kind == "ecp":
            ref = oracle.adjoint(w.grid, w.profile, w.radius, r)
        else:
            ref = oracle.hybrid_adjoint(w.grid, w.profile, w.radius, r, oversample=plan.info.oversample)
        assert _frac(ct, ref) <= 1e-11


def test_plan_graph_capture_replays():
    """A hipGraph capture of a plan's forward and transpose calls (several
    FFT classes, the accumulation and the pole fix) replays to the eager
    result, with eager work between replays."""
    w = W.healpix256()
    _say(f"case graph capture {w.name}")
    plan = _plan(w)
    x = _tt(W.make_input(w), w)
    ws = plan.workspace()
    y, z = torch.empty_like(x), torch.empty_like(x)
    plan.convolve(x, out=y, ws=ws)
    plan.adjoint(y, out=z, ws=ws)
    torch.cuda.synchronize()
    ey, ez = y.clone(), z.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.convolve(x, out=y, ws=ws)
        plan.adjoint(y, out=z, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.convolve(x, out=y, ws=ws)
        plan.adjoint(y, out=z, ws=ws)
    for rep in range(4):
        y.zero_()
        z.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ey) and torch.equal(z, ez), rep
        _ = (x * 2).sum().item()  # eager work between replays
