"""CPU-side checks of the C ABI: the library loads, exports every function
include/arkcos.h declares, and rejects bad arguments on the host before any
device work (no GPU call is needed for these)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "arkcos.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(arkcos_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1104_0672_amd import arkcos as ak
    path = ak.LIB_PATH
    if not os.path.exists(path):
        from paper_1104_0672_amd import build
        build.build()
    return ak.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("arkcos_plan", "arkcos_convolve", "arkcos_convolve_adjoint", "arkcos_kernel_grad",
                 "arkcos_batch_plan", "arkcos_batch_convolve", "arkcos_workspace_size"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1104_0672_amd import arkcos as ak
    out = subprocess.run(["nm", "-D", "--defined-only", ak.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (arkcos_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(_declared()) == set(ak.EXPORTED)


def _plan_status(lib, geom, prof, radius=0.1, dtype=0, opts=None):
    from paper_1104_0672_amd import arkcos as ak
    h = ctypes.c_void_p()
    st = lib.arkcos_plan(ctypes.byref(geom), ctypes.byref(prof), radius, dtype,
                         ctypes.byref(opts) if opts is not None else None, ctypes.byref(h))
    return st, lib.arkcos_last_error().decode(), h


def test_host_argument_checks(lib):
    from paper_1104_0672_amd import arkcos as ak
    good_g = ak.Geometry(1, 8, 0, 0)
    good_p = ak.ProfileC(0, 0.05, 0, 0.0, None)
    cases = [
        (ak.Geometry(1, 0, 0, 0), good_p, 0.1, 0, None, "nside"),
        (ak.Geometry(0, 0, 8, 7), good_p, 0.1, 0, None, "ECP"),
        (ak.Geometry(2, 8, 0, 0), good_p, 0.1, 0, None, "kind"),
        (good_g, ak.ProfileC(0, -1.0, 0, 0.0, None), 0.1, 0, None, "FWHM"),
        (good_g, ak.ProfileC(1, 0.0, 2, 0.1, None), 0.1, 0, None, "spline"),
        (good_g, good_p, 0.0, 0, None, "radius"),
        (good_g, good_p, 4.0, 0, None, "radius"),
        (good_g, good_p, 0.1, 7, None, "dtype"),
        (good_g, good_p, 0.1, 0, ak.Options(3, 0, 1, -1.0), "oversample"),
        (good_g, good_p, 0.1, 0, ak.Options(2, 5, 1, -1.0), "kgen"),
        (good_g, good_p, 0.1, 0, ak.Options(2, 0, 1, -1.0, 2, 0), "mode"),
        (good_g, good_p, 0.1, 0, ak.Options(2, 0, 1, -1.0, 0, 2), "own_grid"),
        (good_g, good_p, 0.1, 0, ak.Options(2, 0, 1, -1.0, 0, 0, 3), "kernel_eval"),
        (good_g, good_p, 0.1, 0, ak.Options(2, 0, 1, -1.0, 0, 0, 1, 1), "table_nodes"),
        (good_g, good_p, 0.1, 0, ak.Options(2, 0, 1, -1.0, 0, 0, 0, 0, (0, 0, 1, 0)), "reserved"),
    ]
    for g, p, r, dt, o, word in cases:
        st, msg, h = _plan_status(lib, g, p, r, dt, o)
        assert st == 1, (word, st, msg)
        assert word.lower() in msg.lower()
        assert not h.value
    assert lib.arkcos_convolve(None, None, None, None, None) == 1
    assert lib.arkcos_plan_destroy(None) == 1
    assert lib.arkcos_status_string(0) == b"ARKCOS_OK"


def test_default_options(lib):
    from paper_1104_0672_amd import arkcos as ak
    o = ak.Options(9, 9, 9, 9.0, 9, 9, 9, 9, (9, 9, 9, 9))
    lib.arkcos_default_options(ctypes.byref(o))
    assert (o.oversample, o.kgen, o.fix_pole_pixels, o.band_tol, o.mode, o.own_grid, o.kernel_eval,
            o.table_nodes, tuple(o.reserved)) == (0, 0, 1, -1.0, 0, 0, 0, 0, (0, 0, 0, 0))


def test_device_code_is_built_for_gfx950_only(lib):
    """Every object of the library that carries device code carries it for
    gfx950 and for no other target: a kernel in a source compiled without the
    target would have no code object on the MI355X."""
    build = os.path.join(ROOT, "paper_1104_0672_amd", "_build")
    objs = sorted(f for f in os.listdir(build) if f.endswith(".o"))
    assert objs
    with_device = 0
    for f in objs:
        path = os.path.join(build, f)
        sections = subprocess.run(["readelf", "-S", path], capture_output=True, text=True).stdout
        if ".hip_fatbin" not in sections:
            continue
        dump = os.path.join(build, f + ".fatbin.tmp")
        subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", path, dump], check=True)
        data = open(dump, "rb").read()
        os.remove(dump)
        targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", data))
        if targets:
            with_device += 1
            assert targets == {b"gfx950"}, (f, targets)
    assert with_device >= 6  # the .hip sources


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program built against include/arkcos.h prints them)."""
    from paper_1104_0672_amd import arkcos as ak
    pairs = [(ak.Geometry, "arkcos_geometry_t"), (ak.ProfileC, "arkcos_profile_t"),
             (ak.Options, "arkcos_options_t"), (ak.PlanInfo, "arkcos_plan_info_t"),
             (ak.BatchInfo, "arkcos_batch_info_t")]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "arkcos.h"', "int main(void) {"]
    expect = []
    for cls, cname in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for name, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {name}));')
            expect.append(getattr(cls, name).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    # (the header takes hipStream_t from the HIP runtime header)
    cpp = subprocess.run(["/opt/rocm/bin/hipconfig", "--cpp_config"], capture_output=True, text=True).stdout.split()
    subprocess.run(["gcc", "-std=c11", *cpp, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect
