"""GPU parity of the plan options and of the production interfaces around
the convolution, through the C ABI, against the FP64 oracle.

* own_grid="equatorial": the artifact suppression as Sect. 4.3 states it
  (true-offset sampling only for equatorial ring pairs), at the paper's grid
  (oversample 1) and at oversample 2: FP64 against the step-by-step hybrid
  reference in the same setting (<= 1e-11), FP32 against it (<= 1e-5), and
  the error against the direct sum per region, printed;
* kernel_eval="table": the biased linear kernel table of Sect. 4.1 against
  the hybrid reference using the same table;
* kgen=1 on HEALPix: the on-the-fly Clenshaw, shifted-grid and Reinsch
  recurrences (each present in the plan) against the hybrid (FP64) and the
  direct sum (FP32);
* the knot gradient with rows of more than 48 kernel samples (64 knots,
  oversample 16) against the hybrid reference's gradient;
* knot updates on the stream (arkcos_set_knots_async) against the host call;
* autograd with one plan and two knot tensors in one graph;
* a batch's forward and transpose on different buffers captured in one graph.
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


def _frac(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _say(msg):
    print(msg, flush=True)


def _tt(x, dtype):
    return torch.tensor(x, dtype=torch.float32 if dtype == "f32" else torch.float64, device="cuda")


def _beam(nside, pixels):
    """Gaussian workload of `pixels` pixel widths FWHM, R = 3 FWHM."""
    return 60 * math.degrees(pixels * math.sqrt(math.pi / 3) / nside)


def _regions(grid, radius):
    """Pixel sets: polar caps, equatorial belt, and the belt rings within
    the support radius of a cap ring (where pairs mix the two)."""
    th, ph0, w, n, st = oracle.rings(grid)
    L = 4 * grid.nside
    belt_r = [i for i in range(len(th)) if n[i] == L]
    cap_r = [i for i in range(len(th)) if n[i] != L]
    capth = th[cap_r]
    edge_r = [i for i in belt_r if np.min(np.abs(capth - th[i])) <= radius + 1e-9]
    pix = lambda rs: np.concatenate([st[i] + np.arange(n[i]) for i in rs]) if rs else np.zeros(0, np.int64)
    return {"caps": pix(cap_r), "belt": pix(belt_r), "cap-boundary belt rings": pix(edge_r)}


@pytest.mark.parametrize("nside,p", [(16, 1), (16, 2), (40, 1), (40, 2), (64, 1)])
def test_equatorial_own_grid_fp64_matches_hybrid(nside, p):
    from paper_1104_0672_amd import Plan
    w = W.scaled_healpix(nside, fwhm_arcmin=_beam(nside, 2.5), radius_fwhm=3.0, dtype="f64", seed=nside + p)
    _say(f"case own_grid=equatorial {w.name} f64 p={p}")
    x = W.make_input(w)
    plan = Plan.from_workload(w, oversample=p, own_grid="equatorial")
    y = plan.convolve(_tt(x, "f64")).cpu().numpy()
    ref = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=p, own_grid="equatorial")
    assert _frac(y, ref) <= 1e-11
    # the transpose in the same setting
    r = np.random.default_rng(nside).standard_normal(w.grid.npix)
    yt = plan.adjoint(_tt(r, "f64")).cpu().numpy()
    ref_t = oracle.hybrid_adjoint(w.grid, w.profile, w.radius, r, oversample=p, own_grid="equatorial")
    assert _frac(yt, ref_t) <= 1e-11


@pytest.mark.parametrize("nside", [64, 256])
def test_own_grid_settings_fp32_per_region(nside):
    """Both settings of the own-grid rule, FP32 on the GPU: against the FP64
    hybrid in the same setting (<= 1e-5) and, printed per region, against
    the direct sum.  With the automatic oversampling the extension meets the
    1e-4 bound everywhere."""
    from paper_1104_0672_amd import Plan
    w = W.scaled_healpix(nside, fwhm_arcmin=_beam(nside, 2.5), radius_fwhm=3.0, seed=nside)
    x = W.make_input(w)
    ref_d = oracle.direct(w.grid, w.profile, w.radius, x)
    regions = _regions(w.grid, w.radius)
    errs = {}
    for own in ("equal_length", "equatorial"):
        for p in (1, 0):
            plan = Plan.from_workload(w, oversample=p, own_grid=own)
            pp = plan.info.oversample
            y = plan.convolve(_tt(x, "f32")).cpu().numpy().astype(np.float64)
            ref_h = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=pp, own_grid=own)
            e_h = _frac(y, ref_h)
            parts = ", ".join(f"{k} {_frac(y[v], ref_d[v]):.2e} (max {np.abs(y[v] - ref_d[v]).max() / np.abs(ref_d).max():.1e})"
                              for k, v in regions.items() if v.size)
            hparts = ", ".join(f"{k} {_frac(y[v], ref_h[v]):.2e}" for k, v in regions.items() if v.size)
            _say(f"  nside {nside} own_grid={own} p={pp}: vs hybrid {e_h:.2e} ({hparts}); vs direct sum: all "
                 f"{_frac(y, ref_d):.2e}; {parts}")
            errs[(own, p)] = (e_h, _frac(y, ref_d))
    for (own, p), (e_h, e_d) in errs.items():
        assert e_h <= 1e-5, (own, p, e_h)
        if p == 0 and own == "equal_length":
            assert e_d <= 1e-4


def test_chord_table_kernel_fp64_matches_hybrid_and_fp32_direct():
    from paper_1104_0672_amd import Plan
    w = W.scaled_healpix(24, fwhm_arcmin=_beam(24, 2.5), radius_fwhm=3.0, dtype="f64", seed=5)
    _say(f"case kernel_eval=table {w.name}")
    x = W.make_input(w)
    for nodes in (1024, 65536):
        plan = Plan.from_workload(w, oversample=2, kernel_eval="table", table_nodes=nodes)
        y = plan.convolve(_tt(x, "f64")).cpu().numpy()
        ref = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=2, kernel_eval="table", table_nodes=nodes)
        exact = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=2)
        _say(f"  nodes {nodes}: vs hybrid with the table {_frac(y, ref):.2e}, table vs exact kernel "
             f"{_frac(ref, exact):.2e}")
        assert _frac(y, ref) <= 1e-11
    w32 = W.healpix256()
    x32 = W.make_input(w32)
    plan = Plan.from_workload(w32, kernel_eval="table")
    y = plan.convolve(_tt(x32, "f32")).cpu().numpy().astype(np.float64)
    e = _frac(y, oracle.direct(w32.grid, w32.profile, w32.radius, x32))
    _say(f"  {w32.name} FP32 with the default 65536-node table: vs direct sum {e:.2e}")
    assert e <= 1e-4


@pytest.mark.parametrize("nside", [16, 40])
def test_recurrence_kernel_sources_on_healpix(nside):
    """kgen=1: K_ij(m) by the recurrences for every pair of up to 48 samples
    (centred Clenshaw, Clenshaw on the half-shifted grid of offset equatorial
    pairs, Reinsch's form for 17..48 samples); wider rows keep tables."""
    from paper_1104_0672_amd import Plan
    for dtype in ("f64", "f32"):
        w = W.scaled_healpix(nside, fwhm_arcmin=_beam(nside, 2.5), radius_fwhm=3.0, dtype=dtype, seed=nside)
        x = W.make_input(w)
        plan = Plan.from_workload(w, kgen=1, oversample=2)
        kinds = list(plan.info.pairs_by_kind)
        _say(f"case kgen=1 {w.name} {dtype}: pairs by kind (centred, shifted, table, Reinsch) {kinds}")
        assert kinds[0] > 0 and kinds[1] > 0 and kinds[3] > 0
        y = plan.convolve(_tt(x, dtype)).cpu().numpy().astype(np.float64)
        if dtype == "f64":
            assert _frac(y, oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=2)) <= 1e-11
            r = np.random.default_rng(3).standard_normal(w.grid.npix)
            yt = plan.adjoint(_tt(r, "f64")).cpu().numpy()
            assert _frac(yt, oracle.hybrid_adjoint(w.grid, w.profile, w.radius, r, oversample=2)) <= 1e-11
        else:
            e = _frac(y, oracle.direct(w.grid, w.profile, w.radius, x))
            _say(f"  FP32 vs direct sum {e:.2e}")
            assert e <= 1e-4


def _spline_workload(nside, n_knots, dtype, seed, width_pix=5.0):
    pix = math.sqrt(math.pi / 3) / nside
    tmax = width_pix * pix
    th = np.arange(n_knots) * tmax / (n_knots - 1)
    rng = np.random.default_rng(seed)
    c = W.mexican_hat(th, tmax / 5) + 0.01 * rng.standard_normal(n_knots)
    prof = W.Profile("spline", theta_max=tmax, knots=tuple(float(v) for v in c))
    return W.Workload(f"spline{nside}_{n_knots}", W.Grid("healpix", nside=nside), prof, tmax, dtype, seed)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
def test_knot_gradient_wide_rows_64_knots(dtype, tol):
    """The shape of the 64-knot spline workload at nside 32 with oversample
    16: the rows of the polar rings span the whole ring (1025 samples), so
    the gradient's wide-row items carry most of the work; all 64 knots."""
    from paper_1104_0672_amd import Plan
    w = _spline_workload(32, 64, dtype, 11)
    th = oracle.rings(w.grid)[0]
    assert th[0] < w.profile.theta_max  # the pole lies inside ring 0's support: full-ring rows
    _say(f"case knot gradient wide rows {w.name} {dtype} p=16")
    plan = Plan.from_workload(w, oversample=16)
    # the rows on the 2048-longitude grid go through the FFT forms
    _say(f"  rows by FFT: tables {plan.info.table_fft_rows}, gradient {plan.info.grad_fft_rows}")
    assert plan.info.grad_fft_rows > 0 and plan.info.table_fft_rows > 0
    rng = np.random.default_rng(12)
    x, t = rng.standard_normal(w.grid.npix), rng.standard_normal(w.grid.npix)
    y = plan.convolve(_tt(x, dtype)).double().cpu().numpy()
    r = y - t
    g = plan.kernel_grad(_tt(x, dtype), _tt(r, dtype)).cpu().numpy()
    ref = oracle.hybrid_knot_grad(w.grid, w.profile, w.radius, x, r, oversample=16)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    _say(f"  max |g - g_ref| / max |g_ref| = {err:.2e}")
    assert err <= tol


def test_knot_gradient_fft_rows_in_chunks():
    """The FFT rows' Y(d) go through the workspace a chunk of rows at a time
    (at most 256 MiB each); a tiny budget makes every chunk a few rows, so the
    chunked path (slots written by the first chunk, added to by the others)
    is compared with the one-chunk plan and with the FP64 reference."""
    import os
    from paper_1104_0672_amd import Plan
    w = _spline_workload(32, 64, "f64", 31)
    _say(f"case knot gradient in chunks {w.name} f64 p=16")
    ref_plan = Plan.from_workload(w, oversample=16)
    os.environ["ARKCOS_GRAD_CHUNK_BYTES"] = "16384"
    try:
        chunked = Plan.from_workload(w, oversample=16)
    finally:
        del os.environ["ARKCOS_GRAD_CHUNK_BYTES"]
    assert chunked.info.grad_fft_rows > 0
    assert chunked.workspace_bytes < ref_plan.workspace_bytes
    rng = np.random.default_rng(32)
    x, t = rng.standard_normal(w.grid.npix), rng.standard_normal(w.grid.npix)
    xd = _tt(x, "f64")
    r = ref_plan.convolve(xd).cpu().numpy() - t
    g1 = ref_plan.kernel_grad(xd, _tt(r, "f64")).cpu().numpy()
    g2 = chunked.kernel_grad(xd, _tt(r, "f64")).cpu().numpy()
    d = np.abs(g2 - g1).max() / np.abs(g1).max()
    ref = oracle.hybrid_knot_grad(w.grid, w.profile, w.radius, x, r, oversample=16)
    e = np.abs(g2 - ref).max() / np.abs(ref).max()
    _say(f"  chunked vs one chunk {d:.2e}, vs FP64 reference {e:.2e}")
    assert d <= 1e-12 and e <= 1e-10


@pytest.mark.parametrize("dt,tol", [("f64", 1e-10), ("f32", 2e-5)])
def test_knot_gradient_half_length_rows(dt, tol):
    """The FFT rows' cosine sums by the half-length form (one packed G/4-point
    transform, the odd samples by a scan of first differences) against the
    S-pass form of the same plan (ARKCOS_GRAD_HALF=0) and against the FP64
    reference; 2048-longitude rows, so both forms run."""
    import os
    from paper_1104_0672_amd import Plan
    w = _spline_workload(32, 64, dt, 33)
    _say(f"case knot gradient half-length rows {w.name} {dt} p=16")
    half = Plan.from_workload(w, oversample=16)
    os.environ["ARKCOS_GRAD_HALF"] = "0"
    try:
        spass = Plan.from_workload(w, oversample=16)
    finally:
        del os.environ["ARKCOS_GRAD_HALF"]
    assert half.info.grad_fft_rows > 0 and half.info.grad_fft_rows == spass.info.grad_fft_rows
    rng = np.random.default_rng(34)
    x, t = rng.standard_normal(w.grid.npix), rng.standard_normal(w.grid.npix)
    xd = _tt(x, dt)
    r = half.convolve(xd).double().cpu().numpy() - t
    g1 = half.kernel_grad(xd, _tt(r, dt)).cpu().numpy()
    g2 = spass.kernel_grad(xd, _tt(r, dt)).cpu().numpy()
    d = np.abs(g1 - g2).max() / np.abs(g2).max()
    ref = oracle.hybrid_knot_grad(w.grid, w.profile, w.radius, x, r, oversample=16)
    e1 = np.abs(g1 - ref).max() / np.abs(ref).max()
    e2 = np.abs(g2 - ref).max() / np.abs(ref).max()
    _say(f"  half vs S-pass {d:.2e}; vs FP64 reference: half {e1:.2e}, S-pass {e2:.2e}")
    assert d > 0.0  # the two forms round differently: both ran
    assert e1 <= tol and e2 <= tol and d <= tol


@pytest.mark.parametrize("nside,p", [(16, None), (32, 16)])
def test_set_knots_async_equals_host_update(nside, p):
    """Knot updates on the device and from the host give the same map, equal
    to the FP64 hybrid reference with the new knots.  At nside 32 with
    oversample 16 the wide rows' tables come from FFTs of the samples."""
    from paper_1104_0672_amd import Plan
    w = _spline_workload(nside, 12, "f64", 21)
    _say(f"case set_knots {w.name} p={p}")
    pa, pb = Plan.from_workload(w, oversample=p or 0), Plan.from_workload(w, oversample=p or 0)
    if p == 16:
        assert pa.info.table_fft_rows > 0
    c2 = np.asarray(w.profile.knots) * 1.3 + 0.05 * np.random.default_rng(22).standard_normal(12)
    x = _tt(np.random.default_rng(23).standard_normal(w.grid.npix), "f64")
    pa.set_knots(c2)
    pb.set_knots_async(torch.tensor(c2, dtype=torch.float64, device="cuda"))
    ya, yb = pa.convolve(x), pb.convolve(x)
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)
    w2 = W.Workload(w.name, w.grid, W.Profile("spline", theta_max=w.profile.theta_max, knots=tuple(c2)),
                    w.radius, "f64", w.seed)
    ref = oracle.hybrid(w2.grid, w2.profile, w2.radius, x.cpu().numpy(), oversample=pa.info.oversample)
    assert _frac(yb.cpu().numpy(), ref) <= 1e-11


def test_autograd_one_plan_two_knot_tensors():
    """One plan used with two different knot tensors in one graph: each
    backward must use its own forward's knots (the adjoint depends on them)."""
    from paper_1104_0672_amd import Plan, convolve
    w = _spline_workload(8, 8, "f64", 31)
    plan = Plan.from_workload(w)
    p = plan.info.oversample
    rng = np.random.default_rng(32)
    n = w.grid.npix
    x1, x2 = (_tt(rng.standard_normal(n), "f64").requires_grad_(True) for _ in range(2))
    t1, t2 = (_tt(rng.standard_normal(n), "f64") for _ in range(2))
    c1 = np.asarray(w.profile.knots)
    c2 = c1[::-1].copy() * 0.7
    k1 = torch.tensor(c1, dtype=torch.float64, device="cuda", requires_grad=True)
    k2 = torch.tensor(c2, dtype=torch.float64, device="cuda", requires_grad=True)
    y1 = convolve(x1, plan, k1)
    y2 = convolve(x2, plan, k2)
    loss = 0.5 * ((y1 - t1) ** 2).sum() + 0.5 * ((y2 - t2) ** 2).sum()
    gx1, gx2, gk1, gk2 = torch.autograd.grad(loss, (x1, x2, k1, k2))
    for xs, ts, ks, cc, gx, gk in ((x1, t1, k1, c1, gx1, gk1), (x2, t2, k2, c2, gx2, gk2)):
        prof = W.Profile("spline", theta_max=w.profile.theta_max, knots=tuple(cc))
        xh = xs.detach().cpu().numpy()
        yh = oracle.hybrid(w.grid, prof, w.radius, xh, oversample=p)
        r = yh - ts.cpu().numpy()
        ref_x = oracle.hybrid_adjoint(w.grid, prof, w.radius, r, oversample=p)
        ref_k = oracle.hybrid_knot_grad(w.grid, prof, w.radius, xh, r, oversample=p)
        assert _frac(gx.cpu().numpy(), ref_x) <= 1e-10
        assert np.abs(gk.cpu().numpy() - ref_k).max() <= 1e-10 * np.abs(ref_k).max()
        # and against the explicit transpose of the direct sum (method error only)
        ex = oracle.adjoint(w.grid, prof, w.radius, r)
        _say(f"  gx vs explicit transpose of the direct sum: {_frac(gx.cpu().numpy(), ex):.2e}")


def test_batch_forward_and_adjoint_captured_in_one_graph():
    from paper_1104_0672_amd import Batch, Plan
    wl = [W.scaled_healpix(ns, fwhm_arcmin=f, radius_fwhm=3.0, seed=k)
          for k, (ns, f) in enumerate(((16, 300.0), (32, 120.0), (8, 600.0)))]
    plans = [Plan.from_workload(w) for w in wl]
    batch = Batch(plans)
    xs = [_tt(W.make_input(w), "f32") for w in wl]
    ys = [torch.empty_like(x) for x in xs]
    zs = [torch.empty_like(x) for x in xs]
    ws = batch.workspace()
    ey = [p.convolve(x) for p, x in zip(plans, xs)]
    ez = [p.adjoint(y) for p, y in zip(plans, ey)]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.convolve(xs, outs=ys, ws=ws)
        batch.convolve(ys, outs=zs, adjoint=True, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.convolve(xs, outs=ys, ws=ws)
        batch.convolve(ys, outs=zs, adjoint=True, ws=ws)
    for rep in range(3):
        for t in ys + zs:
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(len(wl)):
            assert torch.equal(ys[k], ey[k]), (rep, k)
            assert torch.equal(zs[k], ez[k]), (rep, k)
        # eager batch calls on other buffers between replays must not redirect the graph
        other = [torch.zeros_like(x) for x in xs]
        batch.convolve(xs, outs=other, ws=ws)
        torch.cuda.synchronize()
        for k in range(len(wl)):
            assert torch.equal(other[k], ey[k])
