"""arkcos_convolve_noalloc, the forward convolution whose workspace is the
library's fixed device scratch array (for callers that cannot allocate),
called through the C ABI and compared with arkcos_convolve on the same plan
and input: the same kernels in the same order, so the maps must be equal
bit for bit.  Two calls in a row, the second on a smaller plan; and a plan
whose workspace exceeds the scratch is rejected without any work."""
import ctypes

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    from paper_1104_0672_amd.arkcos import load_library
    lib = load_library()
    lib.arkcos_convolve_noalloc.argtypes = [ctypes.c_void_p] * 4
    lib.arkcos_convolve_noalloc.restype = ctypes.c_int
    lib.arkcos_noalloc_scratch_bytes.argtypes = []
    lib.arkcos_noalloc_scratch_bytes.restype = ctypes.c_size_t
    return lib


def _noalloc(lib, plan, x, y):
    s = torch.cuda.current_stream()
    return lib.arkcos_convolve_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       ctypes.c_void_p(s.cuda_stream))


def test_noalloc_equals_convolve_on_two_calls_second_smaller():
    from paper_1104_0672_amd import Plan
    lib = _lib()
    cap = lib.arkcos_noalloc_scratch_bytes()
    cases = [(W.scaled_healpix(128, fwhm_arcmin=60.0, radius_fwhm=3.0), "f32"),
             (W.scaled_healpix(32, fwhm_arcmin=240.0, radius_fwhm=3.0), "f64")]
    for w, dt in cases:
        plan = Plan.from_workload(w, dtype=dt)
        print(f"case noalloc {w.name} {dt}: workspace {plan.workspace_bytes} of {cap} bytes", flush=True)
        assert plan.workspace_bytes <= cap
        td = torch.float32 if dt == "f32" else torch.float64
        x = torch.tensor(W.make_input(w), dtype=td, device="cuda")
        ref = plan.convolve(x)
        y = torch.full_like(x, float("nan"))
        assert _noalloc(lib, plan, x, y) == 0
        torch.cuda.synchronize()
        assert torch.equal(y, ref)


def test_noalloc_rejects_a_workspace_beyond_the_scratch():
    from paper_1104_0672_amd import Plan
    lib = _lib()
    cap = lib.arkcos_noalloc_scratch_bytes()
    w = W.scaled_healpix(1024, fwhm_arcmin=10.0, radius_fwhm=3.0)
    plan = Plan.from_workload(w)
    print(f"case noalloc reject {w.name}: workspace {plan.workspace_bytes} of {cap} bytes", flush=True)
    assert plan.workspace_bytes > cap
    x = torch.zeros(plan.npix, dtype=torch.float32, device="cuda")
    y = torch.full_like(x, 7.0)
    assert _noalloc(lib, plan, x, y) == 2  # ARKCOS_ERR_NOT_SUPPORTED
    assert b"exceeds the fixed scratch" in lib.arkcos_last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
