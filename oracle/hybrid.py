"""The paper's hybrid Fourier/direct-space algorithm, step by step, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Library FFTs (numpy)
serve as steps; nothing is blocked, fused or reordered.

Steps, in the paper's order (Sect. 4.1 and the artifact suppression of
Sect. 4.3):

(a) real FFT of every input ring, ``A_j(m) = sum_k x_jk exp(-2 pi i m k / N_j)``;
    the phase shift of eq. "fftrot" turns it into the spectrum of the ring in
    absolute longitude, ``A_j(m) exp(-i m phi0_j)``; the artifact-suppressed
    mode duplicates (periodically extends) it past the ring's own Nyquist
    frequency instead of zero-padding it.
(b) for every output ring i and input ring j in the support, the kernel row
    ``g(nu) = w_j K(theta(i, j, nu))`` sampled on a longitude grid centred on
    the output ring (the paper's kernel grid, 4 nside points per ring), and its
    FFT ``K_ij(m)``.  Equatorial ring pairs with equal ring lengths do not use
    the phase shift: the kernel is sampled at the true pixel offsets, i.e. at
    longitudes shifted by ``phi0_i - phi0_j`` (Sect. 4.3), which makes them
    exact; the same holds for any two rings of equal length N (a polar ring
    with itself or its mirror).  In absolute longitude this is the grid
    ``2 pi (d + s/2) / N`` with s = 1 when the rings are offset by an odd
    multiple of pi / N.
(c) ``B_i(m) = sum_j K_ij(m) A~_j(m)`` (the theta-direction summation).
(d) reverse phase shift, fold the super-Nyquist modes onto the ring's own
    modes (Sect. 4.3), inverse real FFT of length N_i.
(e) optionally, the first and last ring (8 pixels on HEALPix) recomputed by
    the direct sum (Sect. 4.2).

``mode="default"`` is the paper's plain mode of Sect. 4.1, without the
artifact suppression of Sect. 4.3: every pair uses the ``p L`` kernel grid
(no pair is sampled at its true pixel offsets), step (a) zero-pads each
ring's spectrum beyond its own Nyquist mode instead of repeating it, and
step (d) keeps only the output ring's modes |m| <= N_i / 2 instead of folding
the higher ones onto them.

Readings taken where the paper is silent:

* Kernel grids: pairs of equal-length rings sample the kernel at their true
  pixel offsets on a grid of their own length (exact); other pairs sample it
  on ``p L`` longitudes (``p = 1`` is the paper's grid) and keep modes up to
  ``p L / 2``.
* The Nyquist mode of each pair's grid is split symmetrically (half weight),
  so every pair contributes the real trigonometric interpolant of its kernel
  row, evaluated at the true pixel offsets.
* The 1 / (grid length) normalisation of the kernel FFT is applied per pair.
* Default mode: the zero-padded spectrum keeps the ring's DFT at 0 <= m <= N/2
  (the Nyquist coefficient included once, as the paper's rectangular array
  holds it), and the truncated synthesis is the two-sided real sum over
  |m| <= N_i / 2 (both +N_i/2 and -N_i/2 kept).
* ``own_grid="equatorial"`` restricts the true-offset sampling to pairs of
  equatorial rings, as Sect. 4.3 states it; ``"equal_length"`` (the default)
  extends it to a polar ring with itself and with its mirror.
* ``kernel_eval="table"`` replaces K in step (b) by the paper's biased table
  of Sect. 4.1 (eq. "kernel_angle"): the distance parametrised by the squared
  chord u = 2 (1 - cos theta), a table of K(2 asin(sqrt(u) / 2)) at nodes
  uniform in u on [0, u(R)] (the last node at R itself), interpolated
  linearly in u.
"""
from __future__ import annotations

import numpy as np

from . import SUPPORT_TOL, direct, kernel, rings, basis


def _ring_distance(th_i, th_j, nu):
    """Angle between (th_i, 0) and (th_j, nu), from 3-D unit vectors."""
    ax, az = np.sin(th_i), np.cos(th_i)
    bx, by, bz = np.sin(th_j) * np.cos(nu), np.sin(th_j) * np.sin(nu), np.cos(th_j)
    cx = -az * by
    cy = az * bx - ax * bz
    cz = ax * by
    return np.arctan2(np.sqrt(cx * cx + cy * cy + cz * cz), ax * bx + az * bz)


def _grid_length(grid):
    return 4 * grid.nside if grid.kind == "healpix" else grid.nphi


def chord_table_kernel(profile, radius, nodes):
    """K evaluated through the biased linear table of Sect. 4.1: returns a
    function of the angle t that interpolates, linearly in u = 4 sin^2(t/2),
    the values K(2 asin(sqrt(u_k) / 2)) at u_k = k u(R) / (nodes - 1)."""
    rt = radius + SUPPORT_TOL
    umax = 4.0 * np.sin(0.5 * rt) ** 2
    du = umax / (nodes - 1)
    uk = np.arange(nodes) * du
    tk = 2.0 * np.arcsin(np.minimum(0.5 * np.sqrt(uk), 1.0))
    tk[-1] = rt
    tab = kernel(profile, radius, tk)

    def f(t):
        t = np.asarray(t, dtype=np.float64)
        u = 4.0 * np.sin(0.5 * t) ** 2
        x = u / du
        k = np.clip(np.floor(x).astype(np.int64), 0, nodes - 2)
        v = tab[k] + (x - k) * (tab[k + 1] - tab[k])
        return np.where(u > umax, 0.0, v)
    return f


def pair_plan(grid, radius, oversample, mode="suppressed", own_grid="equal_length"):
    """For each output ring i: list of (j, G, s) -- input ring, number of
    kernel-grid longitudes and half-shift flag of the grid.

    Rings of equal length (a HEALPix ring with itself or its mirror, any two
    equatorial rings, any ECP pair) are sampled at their true pixel offsets on
    a grid of their own length (the equatorial modification of Sect. 4.3,
    applied to every equal-length pair); the rest use oversample * L
    longitudes (L = 4 nside: the paper's kernel grid when oversample = 1).
    With own_grid="equatorial" only pairs of rings of L pixels (the
    equatorial ones) are sampled on their own grid.  In the default mode
    every pair uses the oversample * L grid."""
    if own_grid not in ("equal_length", "equatorial"):
        raise ValueError(own_grid)
    th, ph0, w, n, st = rings(grid)
    L = _grid_length(grid)
    out = []
    for i in range(len(th)):
        lst = []
        for j in range(len(th)):
            if abs(th[j] - th[i]) > radius + 1e-6:
                continue
            e = (ph0[i] - ph0[j]) * n[i] / np.pi
            aligned = mode == "suppressed" and n[i] == n[j] and abs(e - round(e)) < 1e-9
            if own_grid == "equatorial":
                aligned = aligned and n[i] == L
            if aligned:
                lst.append((j, int(n[i]), int(round(e)) % 2))
            else:
                lst.append((j, int(oversample) * L, 0))
        out.append(lst)
    return out


def _extended_spectrum(a, phi0, nring, mmax, mode="suppressed"):
    """Physical-longitude spectrum A_j(m mod N_j) exp(-i m phi0), m = 0..mmax;
    in the default mode A_j(m) exp(-i m phi0) up to m = N_j / 2 and zero
    beyond."""
    m = np.arange(mmax + 1)
    if mode == "default":
        base = np.where(m <= nring // 2, a[np.minimum(m, nring // 2)], 0.0)
        return base * np.exp(-1j * m * phi0)
    r = m % nring
    lower = r <= nring // 2
    base = np.where(lower, a[np.minimum(r, nring // 2)], np.conj(a[np.minimum(nring - r, nring // 2)]))
    return base * np.exp(-1j * m * phi0)


def _kernel_row_spectrum(profile, radius, th_i, th_j, w_j, nn, s, values=None):
    """K_ij(m), m = 0..nn/2, for the kernel sampled on nn longitudes, with the
    1/nn normalisation and the half-weight Nyquist mode.  ``values``
    optionally replaces K by another radial function (used for the knot
    basis); if it returns one column per function (shape (nn, K)), every
    column is transformed and K_ij(m) has shape (nn/2 + 1, K)."""
    nu = 2.0 * np.pi * (np.arange(nn) + 0.5 * s) / nn
    t = _ring_distance(th_i, th_j, nu)
    g = w_j * (kernel(profile, radius, t) if values is None else values(t))
    m = np.arange(nn // 2 + 1)
    ph = np.exp(-1j * np.pi * m * s / nn)
    kf = np.fft.fft(g, axis=0)[: nn // 2 + 1] * (ph if g.ndim == 1 else ph[:, None])
    kf = kf.real / nn
    kf[nn // 2] *= 0.5
    return kf


def _fold_inverse(bm, phi0, nring, mode="suppressed"):
    """Reverse phase shift, alias every mode onto m mod N, inverse real FFT;
    the default mode first drops the modes above N / 2 (truncation)."""
    if mode == "default":
        bm = bm[: nring // 2 + 1]
    m = np.arange(bm.size)
    bp = bm * np.exp(1j * m * phi0)
    half = nring // 2
    g = np.zeros(half + 1, complex)
    r = m % nring
    pos = r <= half
    np.add.at(g, r[pos], bp[pos])
    rn = (nring - r) % nring
    neg = (m > 0) & (rn <= half)
    np.add.at(g, rn[neg], np.conj(bp[neg]))
    return np.fft.irfft(g, nring) * nring


def _hybrid_core(grid, profile, radius, x, oversample, values=None, mode="suppressed", own_grid="equal_length"):
    if mode not in ("suppressed", "default"):
        raise ValueError(mode)
    th, ph0, w, n, st = rings(grid)
    L = _grid_length(grid)
    x = np.asarray(x, dtype=np.float64)
    spec = [np.fft.rfft(x[st[j]: st[j] + n[j]]) for j in range(len(th))]      # step (a)
    plan = pair_plan(grid, radius, oversample, mode, own_grid)
    y = None
    for i, pairs in enumerate(plan):
        mmax = max(nn // 2 for (_, nn, _) in pairs)
        b = None
        for (j, nn, s) in pairs:
            kf = _kernel_row_spectrum(profile, radius, th[i], th[j], w[j], nn, s, values)  # (b)
            a = _extended_spectrum(spec[j], ph0[j], n[j], kf.shape[0] - 1, mode)
            if b is None:
                b = np.zeros((mmax + 1,) + kf.shape[1:], complex)
            b[: kf.shape[0]] += kf * (a if kf.ndim == 1 else a[:, None])                  # (c)
        if y is None:
            y = np.empty((grid.npix,) + b.shape[1:])
        if b.ndim == 1:
            y[st[i]: st[i] + n[i]] = _fold_inverse(b, ph0[i], n[i], mode)                  # (d)
        else:
            for k in range(b.shape[1]):
                y[st[i]: st[i] + n[i], k] = _fold_inverse(b[:, k], ph0[i], n[i], mode)
    return y


def _pole_pixels(grid):
    if grid.kind != "healpix":
        return np.zeros(0, np.int64)
    npix = grid.npix
    return np.array([0, 1, 2, 3, npix - 4, npix - 3, npix - 2, npix - 1], np.int64)


def hybrid(grid, profile, radius, x, oversample=2, fix_poles=True, mode="suppressed", own_grid="equal_length",
           kernel_eval="exact", table_nodes=65536):
    """The method's output map (FP64).  ``fix_poles`` recomputes the first and
    last HEALPix ring by the direct sum (step (e)); ``mode`` is "suppressed"
    (Sect. 4.3) or "default" (Sect. 4.1 alone); ``own_grid`` and
    ``kernel_eval`` as in the module docstring (the pole fix always uses the
    exact kernel)."""
    values = None
    if kernel_eval == "table":
        values = chord_table_kernel(profile, radius, table_nodes)
    elif kernel_eval != "exact":
        raise ValueError(kernel_eval)
    y = _hybrid_core(grid, profile, radius, x, oversample, values=values, mode=mode, own_grid=own_grid)
    idx = _pole_pixels(grid)
    if fix_poles and idx.size:
        y[idx] = direct(grid, profile, radius, x, idx=idx)
    return y


def hybrid_adjoint(grid, profile, radius, r, oversample=2, fix_poles=True, mode="suppressed",
                   own_grid="equal_length"):
    """Transpose of ``hybrid`` as a linear map of x.  Ring pairs use symmetric
    kernel grids, so the transpose of the ring pipeline is
    ``w * pipeline(r / w)``; the direct-sum rows of step (e) transpose into
    direct-sum columns."""
    th, ph0, w, n, st = rings(grid)
    wpix = np.repeat(w, n)
    r = np.asarray(r, dtype=np.float64).copy()
    idx = _pole_pixels(grid)
    rfix = np.zeros(grid.npix)
    if fix_poles and idx.size:
        rfix[idx] = r[idx]
        r[idx] = 0.0
    out = wpix * _hybrid_core(grid, profile, radius, r / wpix, oversample, mode=mode, own_grid=own_grid)
    if fix_poles and idx.size:
        from . import adjoint
        out += adjoint(grid, profile, radius, rfix)
    return out


def hybrid_knot_grad(grid, profile, radius, x, r, oversample=2, fix_poles=True, mode="suppressed",
                     own_grid="equal_length"):
    """Gradient of 1/2 |hybrid(x) - t|^2 with respect to the spline knots,
    given r = hybrid(x) - t: the method is linear in the kernel, so
    g_k = <r, hybrid_k(x)> with hybrid_k the method run with kernel phi_k.
    All hybrid_k(x) are computed in one pass over the ring pairs (each pair's
    basis rows phi_k(theta) evaluated once, one column per knot; the basis is
    zero beyond the support, so only samples inside it are evaluated)."""
    nk = len(profile.knots)
    idx = _pole_pixels(grid)
    r = np.asarray(r, dtype=np.float64)

    def rows(t):
        out = np.zeros((t.size, nk))
        inside = t <= radius + 1e-6
        if inside.any():
            out[inside] = basis(profile, radius, t[inside])
        return out
    yk = _hybrid_core(grid, profile, radius, x, oversample, values=rows, mode=mode, own_grid=own_grid)
    rr = r.copy()
    if fix_poles and idx.size:
        rr[idx] = 0.0
    g = rr @ yk
    if fix_poles and idx.size:
        from . import knot_grad
        rr = np.zeros_like(r)
        rr[idx] = r[idx]
        g += knot_grad(grid, profile, radius, x, rr)
    return g
