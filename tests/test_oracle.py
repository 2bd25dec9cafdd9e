"""Pins for the oracle: checks against what the paper and mathematics fix,
not against the oracle's own formulas.

* geometry: hand-written HEALPix ring tables (tests/golden), the equal-area
  property, pixel counts, total area 4 pi, north/south mirror;
* profiles: closed-form Gaussian values, the clamped spline against scipy;
* direct sum: an independent arccos brute force on tiny grids, single-pixel
  response, weighted symmetry of the operator (eq. "def"), exact rotation and
  reflection equivariance, and the Funk-Hecke eigen-relation
  K * Y_lm = b_l Y_lm with b_l = 2 pi int K P_l d(cos theta) (Sect. 2) that the
  pixel quadrature approaches at second order;
* gradients: the loss is quadratic in the knots, so central differences are
  exact up to rounding;
* the step-by-step hybrid reference: it equals the direct sum where the
  method is exact (ECP grids, equatorial HEALPix rings; Sect. 4.3) and
  converges to it with kernel oversampling elsewhere;
* its default mode (Sect. 4.1 without Sect. 4.3): the zero-padded spectrum
  and the truncated synthesis against explicit trigonometric sums, equality
  with the suppressed mode where nothing is padded or truncated (ECP), the
  truncation error vanishing as the kernel becomes band-limited, and the
  cap and equator artifacts that the suppression removes (Sect. 4.3).
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, interpolate, special

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _gauss(fwhm):
    return W.Profile("gaussian", fwhm=fwhm)


def _spline_profile(n=16, tmax=0.3, seed=0):
    th = np.arange(n) * tmax / (n - 1)
    rng = np.random.default_rng(seed)
    c = W.mexican_hat(th, tmax / 5) + 0.01 * rng.standard_normal(n)
    return W.Profile("spline", theta_max=tmax, knots=tuple(c))


# ------------------------------------------------------------------ geometry

def test_healpix_rings_match_golden_tables():
    rows = np.loadtxt(os.path.join(HERE, "golden", "healpix_rings_nside1_2.txt"))
    for nside in (1, 2):
        sel = rows[rows[:, 0] == nside]
        th, ph0, w, n, st = oracle.rings(W.Grid("healpix", nside=nside))
        assert len(th) == len(sel) == 4 * nside - 1
        np.testing.assert_allclose(np.cos(th), sel[:, 2] / sel[:, 3], atol=1e-15)
        np.testing.assert_array_equal(n, sel[:, 4].astype(int))
        np.testing.assert_allclose(ph0 / np.pi, sel[:, 5], atol=1e-15)
        np.testing.assert_array_equal(st, sel[:, 6].astype(int))


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 64, 256])
def test_healpix_equal_area_and_counts(nside):
    g = W.Grid("healpix", nside=nside)
    th, ph0, w, n, st = oracle.rings(g)
    assert n.sum() == 12 * nside * nside == g.npix
    np.testing.assert_array_equal(st, np.concatenate([[0], np.cumsum(n)[:-1]]))
    assert math.isclose(w.sum() * 0 + (w * n).sum(), 4 * math.pi, rel_tol=1e-14)
    # equal area: the spherical cap above a ring centre holds exactly the
    # pixels of the rings before it plus half of the ring itself
    np.testing.assert_allclose(2 * np.pi * (1 - np.cos(th)), w * (st + n / 2), rtol=1e-12, atol=1e-15)
    # north/south mirror
    np.testing.assert_allclose(th + th[::-1], np.pi, atol=1e-14)
    np.testing.assert_array_equal(n, n[::-1])
    np.testing.assert_allclose(ph0, ph0[::-1], atol=0)
    # polar closed form: cos(2 asin(r / (sqrt6 nside))) = 1 - r^2 / (3 nside^2)
    r = np.arange(1, nside)
    np.testing.assert_allclose(np.cos(th[: nside - 1]), 1 - r * r / (3.0 * nside * nside), atol=1e-15)
    # equatorial offsets: shifted iff (r - nside) is even
    req = np.arange(nside, 3 * nside + 1)
    expect = np.where((req - nside) % 2 == 0, np.pi / (4 * nside), 0.0)
    np.testing.assert_allclose(ph0[req - 1], expect, atol=0)


def test_ecp_weights_are_band_areas():
    g = W.Grid("ecp", ntheta=64, nphi=128)
    th, ph0, w, n, st = oracle.rings(g)
    np.testing.assert_allclose(th, (np.arange(64) + 0.5) * np.pi / 64, atol=1e-15)
    assert math.isclose((w * n).sum(), 4 * math.pi, rel_tol=1e-14)
    edges = np.arange(65) * np.pi / 64
    np.testing.assert_allclose(w * 128, 2 * np.pi * (np.cos(edges[:-1]) - np.cos(edges[1:])), rtol=1e-12)
    assert np.all(ph0 == 0) and np.all(n == 128)


# ------------------------------------------------------------------ profiles

def test_gaussian_profile_closed_forms():
    fwhm, R = 0.1, 0.3
    t = np.array([0.0, fwhm / 2, fwhm, R, R + 5e-10, R + 2e-9, 1.0])
    k = oracle.kernel(_gauss(fwhm), R, t)
    assert k[0] == 1.0
    assert math.isclose(k[1], 0.5, rel_tol=1e-14)
    assert math.isclose(k[2], 1.0 / 16.0, rel_tol=1e-13)
    assert k[3] > 0 and k[4] > 0 and k[5] == 0 and k[6] == 0


def test_spline_profile_matches_scipy_clamped_spline():
    prof = _spline_profile()
    knots = np.asarray(prof.knots)
    th = np.arange(len(knots)) * prof.theta_max / (len(knots) - 1)
    ref = interpolate.CubicSpline(th, knots, bc_type="clamped")
    t = np.linspace(0, prof.theta_max, 1001)
    np.testing.assert_allclose(oracle.kernel(prof, prof.theta_max, t), ref(t), atol=1e-13)
    # basis functions: phi_k(t_j) = delta_kj and sum_k c_k phi_k = K
    B = oracle.basis(prof, prof.theta_max, th)
    np.testing.assert_allclose(B, np.eye(len(knots)), atol=1e-13)
    Bt = oracle.basis(prof, prof.theta_max, t)
    np.testing.assert_allclose(Bt @ knots, ref(t), atol=1e-13)
    # zero outside the support
    assert np.all(oracle.kernel(prof, prof.theta_max, np.array([prof.theta_max + 1e-8, 1.0])) == 0)


# ------------------------------------------------------------- direct sums

def _healpix_angles_independent(nside):
    """Pixel centres typed again from the published HEALPix formulas, so the
    brute force below does not use the oracle's own geometry code."""
    th, ph = [], []
    for r in range(1, 4 * nside):
        if r < nside or r > 3 * nside:
            s = r if r < nside else 4 * nside - r
            z = 1 - s * s / (3.0 * nside * nside)
            if r > 3 * nside:
                z = -z
            cnt, off = 4 * s, 0.5
        else:
            z = 4.0 / 3 - 2.0 * r / (3 * nside)
            cnt, off = 4 * nside, 0.5 * ((r - nside + 1) % 2)
        for k in range(cnt):
            th.append(math.acos(z))
            ph.append((k + off) * 2 * math.pi / cnt)
    return np.array(th), np.array(ph)


def _brute_force(th, ph, w, K, x):
    """Dense arccos double loop: the definition with no neighbour search."""
    n = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    ang = np.arccos(np.clip(n @ n.T, -1, 1))
    return (K(ang) * w[None, :]) @ x


def test_direct_sum_equals_dense_brute_force_healpix():
    nside = 4
    g = W.Grid("healpix", nside=nside)
    prof, R = _gauss(0.35), 0.8
    th, ph = _healpix_angles_independent(nside)
    w = np.full(g.npix, 4 * np.pi / g.npix)
    sig = 0.35 / math.sqrt(8 * math.log(2))
    K = lambda a: np.where(a <= R, np.exp(-a * a / (2 * sig * sig)), 0.0)
    x = np.random.default_rng(3).standard_normal(g.npix)
    np.testing.assert_allclose(oracle.direct(g, prof, R, x), _brute_force(th, ph, w, K, x), atol=1e-11)


def test_direct_sum_equals_dense_brute_force_ecp_pole_discs():
    g = W.Grid("ecp", ntheta=8, nphi=16)
    prof, R = _gauss(0.6), 1.7  # discs cover the poles: full-ring windows
    i, k = np.divmod(np.arange(g.npix), 16)
    th, ph = (i + 0.5) * np.pi / 8, 2 * np.pi * k / 16
    w = (2 * np.pi / 16) * (np.cos(i * np.pi / 8) - np.cos((i + 1) * np.pi / 8))
    sig = 0.6 / math.sqrt(8 * math.log(2))
    K = lambda a: np.where(a <= R, np.exp(-a * a / (2 * sig * sig)), 0.0)
    x = np.random.default_rng(4).standard_normal(g.npix)
    np.testing.assert_allclose(oracle.direct(g, prof, R, x), _brute_force(th, ph, w, K, x), atol=1e-12)


def test_single_pixel_response():
    g = W.Grid("healpix", nside=8)
    prof, R = _gauss(0.2), 0.5
    q = 123
    x = np.zeros(g.npix)
    x[q] = 1.0
    th, ph = oracle.pixel_angles(g)
    y = oracle.direct(g, prof, R, x)
    nv = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    ang = np.arccos(np.clip(nv @ nv[q], -1, 1))
    sig = 0.2 / math.sqrt(8 * math.log(2))
    expect = np.where(ang <= R, np.exp(-ang ** 2 / (2 * sig ** 2)), 0) * 4 * np.pi / g.npix
    np.testing.assert_allclose(y, expect, atol=1e-12)
    assert np.argmax(y) == q


@pytest.mark.parametrize("grid", [W.Grid("healpix", nside=8), W.Grid("ecp", ntheta=16, nphi=32)])
def test_weighted_symmetry_and_explicit_adjoint(grid):
    prof, R = _gauss(0.3), 0.7
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(grid.npix), rng.standard_normal(grid.npix)
    w = oracle.pixel_weights(grid)
    cx, cy = oracle.direct(grid, prof, R, x), oracle.direct(grid, prof, R, y)
    lhs, rhs = np.dot(w * cx, y), np.dot(w * x, cy)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) * 10
    # explicit transpose vs <Cx, y> = <x, C^T y>
    ct = oracle.adjoint(grid, prof, R, y)
    assert abs(np.dot(cx, y) - np.dot(x, ct)) <= 1e-12 * np.linalg.norm(cx) * np.linalg.norm(y)
    np.testing.assert_allclose(ct, w * oracle.direct(grid, prof, R, y / w), rtol=1e-12, atol=1e-15)


def test_rotation_and_reflection_equivariance_healpix():
    g = W.Grid("healpix", nside=8)
    prof, R = _gauss(0.25), 0.6
    th, ph0, w, n, st = oracle.rings(g)
    x = np.random.default_rng(6).standard_normal(g.npix)
    y = oracle.direct(g, prof, R, x)
    # rotation by pi/2 about the polar axis: every ring shifts by n/4 pixels
    perm = np.concatenate([st[i] + (np.arange(n[i]) + n[i] // 4) % n[i] for i in range(len(n))])
    np.testing.assert_allclose(oracle.direct(g, prof, R, x[perm]), y[perm], atol=1e-13)
    # north/south reflection maps ring i onto ring nr-1-i pixel by pixel
    refl = np.concatenate([st[len(n) - 1 - i] + np.arange(n[i]) for i in range(len(n))])
    np.testing.assert_allclose(oracle.direct(g, prof, R, x[refl]), y[refl], atol=1e-13)


def test_shift_equivariance_ecp():
    g = W.Grid("ecp", ntheta=16, nphi=32)
    prof, R = _gauss(0.3), 0.9
    x = np.random.default_rng(7).standard_normal(g.npix)
    y = oracle.direct(g, prof, R, x)
    shift = lambda v: np.roll(v.reshape(16, 32), 1, axis=1).ravel()
    np.testing.assert_allclose(oracle.direct(g, prof, R, shift(x)), shift(y), atol=1e-14)


def _b_ell(K, R, ell):
    f = lambda t: K(t) * special.eval_legendre(ell, math.cos(t)) * math.sin(t)
    return 2 * math.pi * integrate.quad(f, 0, R, epsabs=1e-15, epsrel=1e-13, limit=200)[0]


@pytest.mark.parametrize("kind", ["healpix", "ecp"])
def test_funk_hecke_eigen_relation_converges(kind):
    """Constant maps give b_0 (the kernel integral) and real spherical
    harmonics give b_l Y_lm; the pixel quadrature error falls at second
    order, i.e. at least 3x per doubling of the resolution."""
    fwhm = math.radians(8.0)
    R = 3 * fwhm
    prof = _gauss(fwhm)
    sig = fwhm / math.sqrt(8 * math.log(2))
    K = lambda t: math.exp(-t * t / (2 * sig * sig))
    errs = []
    for res in (16, 32, 64):
        g = W.Grid("healpix", nside=res) if kind == "healpix" else W.Grid("ecp", ntheta=4 * res, nphi=8 * res)
        th, ph = oracle.pixel_angles(g)
        e = []
        for (l, m) in [(0, 0), (2, 1), (5, 3), (8, 2)]:
            Y = special.lpmv(m, l, np.cos(th)) * np.cos(m * ph)
            y = oracle.direct(g, prof, R, Y)
            b = _b_ell(K, R, l)
            e.append(np.linalg.norm(y - b * Y) / np.linalg.norm(b * Y))
        errs.append(e)
    errs = np.array(errs)
    assert np.all(errs[1] * 3 < errs[0]) and np.all(errs[2] * 3 < errs[1]), errs
    assert np.all(errs[2] < 2e-3)


def test_sampled_mode_matches_full_map():
    g = W.Grid("healpix", nside=16)
    prof, R = _gauss(0.1), 0.3
    x = np.random.default_rng(8).standard_normal(g.npix)
    idx = W.sample_pixels(g.npix, 300, 1, must_include=[0, g.npix - 1])
    np.testing.assert_array_equal(oracle.direct(g, prof, R, x, idx=idx), oracle.direct(g, prof, R, x)[idx])
    np.testing.assert_array_equal(oracle.adjoint(g, prof, R, x, idx=idx), oracle.adjoint(g, prof, R, x)[idx])


def _spline_with(prof, knots):
    return W.Profile("spline", theta_max=prof.theta_max, knots=tuple(knots))


def test_knot_gradient_equals_central_differences():
    g = W.Grid("healpix", nside=8)
    prof = _spline_profile(n=12, tmax=0.5, seed=1)
    R = prof.theta_max
    rng = np.random.default_rng(9)
    x, t = rng.standard_normal(g.npix), rng.standard_normal(g.npix)
    c = np.asarray(prof.knots)
    r = oracle.direct(g, prof, R, x) - t
    grad = oracle.knot_grad(g, prof, R, x, r)
    h = 1e-3
    loss = lambda cc: 0.5 * np.sum((oracle.direct(g, _spline_with(prof, cc), R, x) - t) ** 2)
    for k in (0, 3, 7, 11):
        e = np.zeros_like(c)
        e[k] = h
        fd = (loss(c + e) - loss(c - e)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-8 * max(1.0, abs(grad[k])), (k, fd, grad[k])


def test_knot_gradient_sampled_rows():
    g = W.Grid("healpix", nside=8)
    prof = _spline_profile(n=10, tmax=0.4, seed=2)
    rng = np.random.default_rng(10)
    x, r = rng.standard_normal(g.npix), rng.standard_normal(g.npix)
    idx = np.arange(0, g.npix, 7)
    rm = np.zeros_like(r)
    rm[idx] = r[idx]
    np.testing.assert_allclose(oracle.knot_grad(g, prof, prof.theta_max, x, r, idx=idx),
                               oracle.knot_grad(g, prof, prof.theta_max, x, rm), rtol=1e-12, atol=1e-14)


# --------------------------------------------------- support-boundary ties

def test_ecp_workload_has_exact_ties_only():
    """On the 64 x 128 ECP grid with R = 9 pi/64, pairs on one meridian nine
    rings apart and pairs through the pole with i + j = 8 sit exactly at R.
    The inclusion threshold R + 1e-9 keeps them inside on both sides: every
    pair angle stays far (> 1e-10 rad) from the threshold, while FP64 angle
    errors are ~1e-16 rad."""
    w = W.ecp_64x128()
    idx = np.arange(0, w.grid.npix, 5)
    cnt, gap = oracle.neighbour_stats(w.grid, w.radius, idx)
    assert gap > 1e-10
    assert cnt.min() > 0
    # the ties exist: a pixel sees its ninth neighbour up the meridian
    th, ph = oracle.pixel_angles(w.grid)
    q = 20 * 128 + 7
    x = np.zeros(w.grid.npix)
    x[q] = 1.0
    y = oracle.direct(w.grid, w.profile, w.radius, x)
    assert y[(20 + 9) * 128 + 7] > 0 and y[(20 + 10) * 128 + 7] == 0


@pytest.mark.parametrize("make", [W.healpix256, W.healpix2048, W.healpix1024_spline])
def test_healpix_workloads_have_no_near_ties(make):
    w = make()
    idx = W.sample_pixels(w.grid.npix, 2000, 11, must_include=[0, w.grid.npix // 2])
    cnt, gap = oracle.neighbour_stats(w.grid, w.radius, idx)
    assert gap > 1e-12, gap


# ------------------------------------------------ step-by-step hybrid method

def test_hybrid_is_exact_on_ecp():
    w = W.ecp_64x128()
    x = W.make_input(w)
    yd = oracle.direct(w.grid, w.profile, w.radius, x)
    yh = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=1)
    assert np.linalg.norm(yh - yd) / np.linalg.norm(yd) < 1e-13
    assert np.abs(yh - yd).max() < 1e-12 * np.abs(yd).max()


def test_hybrid_is_exact_on_equatorial_rings_and_converges_in_caps():
    nside = 16
    g = W.Grid("healpix", nside=nside)
    pix = math.sqrt(math.pi / 3) / nside
    prof, R = _gauss(2.5 * pix), 7.5 * pix
    x = np.random.default_rng(12).standard_normal(g.npix)
    yd = oracle.direct(g, prof, R, x)
    th, ph0, w, n, st = oracle.rings(g)
    # rings whose whole support lies in the equatorial belt
    eq = [i for i in range(len(th)) if np.all(n[np.abs(th - th[i]) <= R + 1e-6] == 4 * nside)]
    sel = np.concatenate([st[i] + np.arange(n[i]) for i in eq])
    assert len(eq) > 10
    err = []
    for p in (1, 2, 4):
        yh = oracle.hybrid(g, prof, R, x, oversample=p, fix_poles=False)
        assert np.abs(yh[sel] - yd[sel]).max() < 1e-13 * np.abs(yd).max()
        err.append(np.linalg.norm(yh - yd) / np.linalg.norm(yd))
    assert err[0] > 1e-5 and err[1] < 1e-3 * err[0] and err[2] < 1e-10, err


def test_hybrid_phase_shift_sign_is_pinned_by_single_pixel():
    """A single cap pixel must produce a response peaked on itself: a wrong
    sign of the phase shift moves it by twice the ring offset."""
    g = W.Grid("healpix", nside=16)
    th, ph0, w, n, st = oracle.rings(g)
    prof, R = _gauss(0.15), 0.4
    for q in (st[3] + 2, st[10] + 5, st[30] + 1):
        x = np.zeros(g.npix)
        x[q] = 1.0
        yh = oracle.hybrid(g, prof, R, x, oversample=4, fix_poles=False)
        yd = oracle.direct(g, prof, R, x)
        assert np.argmax(yh) == q
        assert np.abs(yh - yd).max() < 1e-8 * yd.max()


def test_hybrid_adjoint_is_transpose():
    g = W.Grid("healpix", nside=8)
    pix = math.sqrt(math.pi / 3) / 8
    prof, R = _gauss(2 * pix), 6 * pix
    rng = np.random.default_rng(13)
    x, y = rng.standard_normal(g.npix), rng.standard_normal(g.npix)
    for fix in (False, True):
        a = np.dot(oracle.hybrid(g, prof, R, x, oversample=2, fix_poles=fix), y)
        b = np.dot(x, oracle.hybrid_adjoint(g, prof, R, y, oversample=2, fix_poles=fix))
        assert abs(a - b) < 1e-12 * abs(a), (fix, a, b)


def test_hybrid_knot_gradient_equals_central_differences():
    g = W.Grid("healpix", nside=4)
    prof = _spline_profile(n=8, tmax=0.9, seed=3)
    R = prof.theta_max
    rng = np.random.default_rng(14)
    x, t = rng.standard_normal(g.npix), rng.standard_normal(g.npix)
    c = np.asarray(prof.knots)
    r = oracle.hybrid(g, prof, R, x, oversample=2) - t
    grad = oracle.hybrid_knot_grad(g, prof, R, x, r, oversample=2)
    h = 1e-3
    loss = lambda cc: 0.5 * np.sum((oracle.hybrid(g, _spline_with(prof, cc), R, x, oversample=2) - t) ** 2)
    for k in range(len(c)):
        e = np.zeros_like(c)
        e[k] = h
        fd = (loss(c + e) - loss(c - e)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-8 * max(1.0, abs(grad[k])), (k, fd, grad[k])


# ------------------------------------------- the paper's default mode (4.1)

def test_default_mode_steps_by_explicit_sums():
    """Zero-padded spectrum: A(m) = sum_k x_k exp(-i m (phi0 + 2 pi k / N))
    for m <= N/2, zero beyond; truncated synthesis: the real two-sided sum
    y_k = sum_{|m| <= N/2} B(m) exp(i m (phi0 + 2 pi k / N)), B(-m) = conj B(m)."""
    from oracle.hybrid import _extended_spectrum, _fold_inverse
    rng = np.random.default_rng(41)
    for N, phi0 in ((12, math.pi / 12), (8, 0.0), (20, math.pi / 20)):
        x = rng.standard_normal(N)
        mmax = 2 * N + 3
        got = _extended_spectrum(np.fft.rfft(x), phi0, N, mmax, mode="default")
        for m in range(mmax + 1):
            want = 0j
            if m <= N // 2:
                for k in range(N):
                    ang = m * (phi0 + 2 * math.pi * k / N)
                    want += x[k] * complex(math.cos(ang), -math.sin(ang))
            assert abs(got[m] - want) < 1e-12 * N, (N, m)
        b = rng.standard_normal(mmax + 1) + 1j * rng.standard_normal(mmax + 1)
        b[0] = b[0].real
        y = _fold_inverse(b, phi0, N, mode="default")
        for k in range(N):
            t = 0.0
            for m in range(-(N // 2), N // 2 + 1):
                bm = b[m] if m >= 0 else np.conj(b[-m])
                ang = m * (phi0 + 2 * math.pi * k / N)
                t += (bm * complex(math.cos(ang), math.sin(ang))).real
            assert abs(y[k] - t) < 1e-11 * N, (N, k)


def test_default_mode_equals_suppressed_mode_on_ecp():
    """ECP rings all have the grid's length and no offset: nothing is padded
    or truncated, so both modes are the exact direct sum."""
    w = W.ecp_64x128()
    x = W.make_input(w)
    yd = oracle.direct(w.grid, w.profile, w.radius, x)
    ya = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=1, mode="default")
    yb = oracle.hybrid(w.grid, w.profile, w.radius, x, oversample=1)
    assert np.abs(ya - yb).max() < 1e-13 * np.abs(yd).max()
    assert np.abs(ya - yd).max() < 1e-12 * np.abs(yd).max()


def test_default_mode_truncation_error_vanishes_for_band_limited_kernels():
    """On rings whose whole support lies in the equatorial belt only the
    truncation at the ring's Nyquist mode separates the default mode from the
    direct sum: the error falls by orders of magnitude as the beam widens."""
    nside = 32
    g = W.Grid("healpix", nside=nside)
    pix = math.sqrt(math.pi / 3) / nside
    th, ph0, w, n, st = oracle.rings(g)
    x = np.random.default_rng(12).standard_normal(g.npix)
    err = []
    for fw in (5.0, 6.0):
        prof, R = _gauss(fw * pix), 3 * fw * pix
        yd = oracle.direct(g, prof, R, x)
        eq = [i for i in range(len(th)) if np.all(n[np.abs(th - th[i]) <= R + 1e-6] == 4 * nside)]
        sel = np.concatenate([st[i] + np.arange(n[i]) for i in eq])
        yh = oracle.hybrid(g, prof, R, x, oversample=2, fix_poles=False, mode="default")
        err.append(np.abs(yh[sel] - yd[sel]).max() / np.abs(yd).max())
    assert err[1] < 1e-6 and err[1] < err[0] / 30, err


def test_suppression_removes_default_mode_artifacts():
    """Point sources under a 2.5-pixel beam: the default mode rings in the caps
    and on the equator (percent level), the suppressed mode with the same
    kernel grid does not (Sect. 4.3)."""
    nside = 16
    g = W.Grid("healpix", nside=nside)
    pix = math.sqrt(math.pi / 3) / nside
    th, ph0, w, n, st = oracle.rings(g)
    prof, R = _gauss(2.5 * pix), 7.5 * pix
    rng = np.random.default_rng(5)
    x = np.zeros(g.npix)
    x[rng.choice(g.npix, 40, replace=False)] = 1.0
    yd = oracle.direct(g, prof, R, x)
    for ring_sel in ([i for i in range(len(th)) if n[i] < 4 * nside], [i for i in range(len(th)) if n[i] == 4 * nside]):
        sel = np.concatenate([st[i] + np.arange(n[i]) for i in ring_sel])
        e = {}
        for mode in ("suppressed", "default"):
            yh = oracle.hybrid(g, prof, R, x, oversample=4, fix_poles=False, mode=mode)
            e[mode] = np.linalg.norm(yh[sel] - yd[sel]) / np.linalg.norm(yd[sel])
        assert e["default"] > 3e-3 and e["suppressed"] < 1e-9, e


def test_default_mode_adjoint_is_transpose():
    g = W.Grid("healpix", nside=8)
    pix = math.sqrt(math.pi / 3) / 8
    prof, R = _gauss(2 * pix), 6 * pix
    rng = np.random.default_rng(17)
    x, y = rng.standard_normal(g.npix), rng.standard_normal(g.npix)
    for fix in (False, True):
        a = np.dot(oracle.hybrid(g, prof, R, x, oversample=2, fix_poles=fix, mode="default"), y)
        b = np.dot(x, oracle.hybrid_adjoint(g, prof, R, y, oversample=2, fix_poles=fix, mode="default"))
        assert abs(a - b) < 1e-12 * abs(a), (fix, a, b)


# --------------------------- the suppression as Sect. 4.3 states it (equatorial own grid)

def test_equatorial_own_grid_is_exact_in_the_belt_and_converges_in_caps():
    """own_grid="equatorial": only pairs of equatorial rings use the true
    pixel offsets (Sect. 4.3 as stated).  Output rings of the belt keep the
    same pairs as the equal-length extension (identical values, exact where
    their support stays in the belt); polar rings pair with themselves on the
    p L grid instead, which converges to the direct sum as p grows."""
    nside = 16
    g = W.Grid("healpix", nside=nside)
    pix = math.sqrt(math.pi / 3) / nside
    prof, R = _gauss(2.5 * pix), 7.5 * pix
    x = np.random.default_rng(51).standard_normal(g.npix)
    yd = oracle.direct(g, prof, R, x)
    th, ph0, w, n, st = oracle.rings(g)
    belt = np.concatenate([st[i] + np.arange(n[i]) for i in range(len(th)) if n[i] == 4 * nside])
    caps = np.setdiff1d(np.arange(g.npix), belt)
    eq_sup = [i for i in range(len(th)) if np.all(n[np.abs(th - th[i]) <= R + 1e-6] == 4 * nside)]
    sel = np.concatenate([st[i] + np.arange(n[i]) for i in eq_sup])
    err = []
    for p in (1, 2, 4, 8):
        ye = oracle.hybrid(g, prof, R, x, oversample=p, fix_poles=False, own_grid="equatorial")
        yl = oracle.hybrid(g, prof, R, x, oversample=p, fix_poles=False, own_grid="equal_length")
        assert np.abs(ye[belt] - yl[belt]).max() <= 1e-15 * np.abs(yd).max()
        assert np.abs(ye[sel] - yd[sel]).max() < 1e-13 * np.abs(yd).max()
        if p == 1:
            # the self pair of a polar ring is the only difference, and it shows
            assert np.abs(ye[caps] - yl[caps]).max() > 1e-6 * np.abs(yd).max()
        err.append(np.linalg.norm(ye[caps] - yd[caps]) / np.linalg.norm(yd[caps]))
    assert err[0] > 1e-5 and err[1] < 1e-2 * err[0] and err[3] < 1e-10, err
    # the transpose and the pairing agree with the plan's listing
    plan = oracle.pair_plan(g, R, 2, own_grid="equatorial")
    for i, pairs in enumerate(plan):
        for (j, G, s) in pairs:
            assert (G == n[i]) == (n[i] == n[j] == 4 * nside)
    rng = np.random.default_rng(52)
    a, b = rng.standard_normal(g.npix), rng.standard_normal(g.npix)
    lhs = np.dot(oracle.hybrid(g, prof, R, a, oversample=2, own_grid="equatorial"), b)
    rhs = np.dot(a, oracle.hybrid_adjoint(g, prof, R, b, oversample=2, own_grid="equatorial"))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ------------------------------------ the biased linear kernel table (Sect. 4.1)

def test_chord_table_kernel_nodes_linearity_and_error_bound():
    """The table of Sect. 4.1 holds K at nodes uniform in the squared chord
    u = 2 (1 - cos t); between nodes it is linear in u.  Its error is at most
    du^2 / 8 max |d^2 K / du^2| (linear interpolation), checked on a Gaussian
    whose u-derivatives follow from K = exp(-t^2 / 2 s^2), t = 2 asin(sqrt(u) / 2)."""
    from oracle.hybrid import chord_table_kernel
    fwhm = 0.02
    s = fwhm / math.sqrt(8 * math.log(2))
    R = 3 * fwhm
    prof = _gauss(fwhm)
    nodes = 257
    f = chord_table_kernel(prof, R, nodes)
    umax = 4 * math.sin(0.5 * (R + 1e-9)) ** 2
    du = umax / (nodes - 1)
    uk = np.arange(nodes - 1) * du
    tk = 2 * np.arcsin(0.5 * np.sqrt(uk))
    assert np.abs(f(tk) - np.exp(-tk ** 2 / (2 * s * s))).max() < 1e-14
    # midpoints in u: the average of the neighbouring nodes
    um = (np.arange(nodes - 1) + 0.5) * du
    tm = 2 * np.arcsin(0.5 * np.sqrt(um))
    kn = np.exp(-(2 * np.arcsin(0.5 * np.sqrt(np.arange(nodes) * du))) ** 2 / (2 * s * s))
    kn[-1] = math.exp(-(R + 1e-9) ** 2 / (2 * s * s))
    assert np.abs(f(tm) - 0.5 * (kn[:-1] + kn[1:])).max() < 1e-14
    # error bound from the second derivative in u (finite differences of the
    # closed form on a fine grid)
    uf = np.linspace(0, umax, 200001)
    kf = np.exp(-(2 * np.arcsin(0.5 * np.sqrt(uf))) ** 2 / (2 * s * s))
    d2 = np.abs(np.diff(kf, 2)).max() / (uf[1] - uf[0]) ** 2
    tf = 2 * np.arcsin(0.5 * np.sqrt(uf))
    err = np.abs(f(tf) - kf).max()
    assert err <= 1.01 * du * du / 8 * d2 and err > 0.05 * du * du / 8 * d2
    assert f(np.array([R + 1e-6]))[0] == 0.0


def test_hybrid_with_chord_table_converges_at_second_order():
    g = W.Grid("healpix", nside=8)
    pix = math.sqrt(math.pi / 3) / 8
    prof, R = _gauss(2.5 * pix), 7.5 * pix
    x = np.random.default_rng(53).standard_normal(g.npix)
    ye = oracle.hybrid(g, prof, R, x, oversample=2)
    errs = []
    nodes = (256, 1024, 4096)
    for n in nodes:
        yt = oracle.hybrid(g, prof, R, x, oversample=2, kernel_eval="table", table_nodes=n)
        errs.append(np.linalg.norm(yt - ye) / np.linalg.norm(ye))
    # error ~ nodes^-2: a factor 16 per factor 4 in nodes (12 .. 20 allowed)
    for a, b in zip(errs, errs[1:]):
        assert 12.0 < a / b < 20.0, errs
