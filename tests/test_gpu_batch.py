"""GPU checks of the batched form: every map of a batch of uneven maps (each
with its own beam) equals its own plan's result bit for bit, forward and
transpose; a hipGraph capture replays to the same result; the batch agrees
with the FP64 oracle through its plans."""
import math
import os

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


def _small_batch(seed=31, n=7):
    rng = np.random.default_rng(seed)
    ws = []
    for k in range(n):
        nside = int(rng.choice([8, 16, 32, 64]))
        pix = 60 * math.degrees(math.sqrt(math.pi / 3) / nside)
        fwhm = float(rng.uniform(1.2, 3.0)) * pix
        ws.append(W.scaled_healpix(nside, fwhm, 3.0, seed=seed + k))
    return ws


def test_batch_equals_per_plan_results():
    from paper_1104_0672_amd import Batch, Plan
    wl = _small_batch()
    print("case batch of", [w.grid.nside for w in wl], flush=True)
    plans = [Plan.from_workload(w) for w in wl]
    batch = Batch(plans)
    assert batch.info.n_maps == len(wl) and batch.info.tuned in (1, 2)
    xs = [torch.tensor(W.make_input(w), dtype=torch.float32, device="cuda") for w in wl]
    for adjoint in (False, True):
        ys = batch.convolve(xs, adjoint=adjoint)
        for p, x, y in zip(plans, xs, ys):
            ref = p.adjoint(x) if adjoint else p.convolve(x)
            assert torch.equal(y, ref)
    # and against the FP64 direct sum
    ys = batch.convolve(xs)
    for w, y in zip(wl, ys):
        ref = oracle.direct(w.grid, w.profile, w.radius, W.make_input(w))
        assert np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-4


def test_batch_mixed_kernel_sources_equal_per_plan_results():
    """Plans whose K_ij(m) come from tables (automatic and kgen=2) and from the
    recurrence (kgen=1) in one batch: the batch takes its general path, and
    every map still equals its own plan's result bit for bit."""
    from paper_1104_0672_amd import Batch, Plan
    wl = _small_batch(seed=61, n=6)
    print("case mixed-source batch of", [w.grid.nside for w in wl], flush=True)
    plans = [Plan.from_workload(w, kgen=k % 3) for k, w in enumerate(wl)]
    batch = Batch(plans)
    xs = [torch.tensor(W.make_input(w), dtype=torch.float32, device="cuda") for w in wl]
    for adjoint in (False, True):
        ys = batch.convolve(xs, adjoint=adjoint)
        for p, x, y in zip(plans, xs, ys):
            ref = p.adjoint(x) if adjoint else p.convolve(x)
            assert torch.equal(y, ref)


def test_batch_many_rings_equals_per_plan_results():
    """Seven nside-512 maps: the batch holds more than 8192 rings of each of
    the 1024- and 2048-point FFT lengths, so it runs them through the
    compile-time ring kernels that a single plan of this size does not use.
    Those kernels keep the FFT passes in registers and round differently
    from the LDS kernels, so every map equals its own plan's result to a few
    FP32 ulps rather than bit for bit."""
    from paper_1104_0672_amd import Batch, Plan
    w0 = W.scaled_healpix(512, 2.5 * 60 * math.degrees(math.sqrt(math.pi / 3) / 512), 3.0, seed=71)
    plan = Plan.from_workload(w0)
    batch = Batch([plan] * 7)
    print("case seven nside-512 maps", flush=True)
    xs = []
    for k in range(7):
        g = torch.Generator(device="cuda")
        g.manual_seed(100 + k)
        xs.append(torch.randn(w0.grid.npix, generator=g, device="cuda", dtype=torch.float32))
    for adjoint in (False, True):
        ys = batch.convolve(xs, adjoint=adjoint)
        for x, y in zip(xs, ys):
            ref = plan.adjoint(x) if adjoint else plan.convolve(x)
            err = float((y - ref).abs().max()) / float(ref.abs().max())
            assert err <= 1e-6, err


def test_batch_graph_capture_replays():
    from paper_1104_0672_amd import Batch, Plan
    wl = _small_batch(seed=41, n=5)
    plans = [Plan.from_workload(w) for w in wl]
    batch = Batch(plans)
    xs = [torch.tensor(W.make_input(w), dtype=torch.float32, device="cuda") for w in wl]
    ys = [torch.empty_like(x) for x in xs]
    ws = batch.workspace()
    eager = [y.clone() for y in batch.convolve(xs, outs=ys, ws=ws)]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.convolve(xs, outs=ys, ws=ws)  # warm, same pointers
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.convolve(xs, outs=ys, ws=ws)
    for rep in range(4):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for y, e in zip(ys, eager):
            assert torch.equal(y, e), rep
        _ = (xs[0] * 2).sum().item()  # eager work between replays


def test_batch_autotune_cache(tmp_path):
    from paper_1104_0672_amd import Batch, Plan
    wl = _small_batch(seed=51, n=3)
    plans = [Plan.from_workload(w) for w in wl]
    os.environ["ARKCOS_AUTOTUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        b1 = Batch(plans)
        b2 = Batch(plans)
    finally:
        del os.environ["ARKCOS_AUTOTUNE_CACHE"]
    assert b1.info.tuned == 1 and b2.info.tuned == 2
    assert (b1.info.seg_units, b1.info.group, b1.info.grid) == (b2.info.seg_units, b2.info.group, b2.info.grid)
