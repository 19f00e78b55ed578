"""CPU checks of the boundary: libsn.so loads and exports every symbol that
include/sn.h declares, and the Python binding binds the same set.  No
compute call is made here (there is no GPU)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sn_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2401_14906_amd as sn

    if not os.path.exists(sn.LIB_PATH):
        from paper_2401_14906_amd import _build

        _build.build()
    return sn.load_library()


def test_header_declares_the_api():
    fns = declared_functions()
    for name in ("sn_extract", "sn_smooth", "sn_batch_submit", "sn_serve_start",
                 "sn_serve_submit", "sn_serve_poll", "sn_serve_wait", "sn_serve_stop"):
        assert name in fns


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, f"libsn.so lacks {missing}"


def test_binding_covers_every_declared_symbol(lib):
    import paper_2401_14906_amd as sn

    bound = {name for name, _, _ in sn._API}
    assert bound == set(declared_functions())


def test_error_strings_without_gpu(lib):
    assert lib.sn_strerror(0) == b"ok"
    assert lib.sn_strerror(-2) == b"out of device memory"
    assert lib.sn_version().startswith(b"libsn gfx950")


def test_null_arguments_are_rejected_without_gpu(lib):
    import paper_2401_14906_amd as sn

    # argument validation happens before any device call
    assert lib.sn_extract(None, None, None, None) == sn.SN_EINVAL
    assert lib.sn_smooth(None, None, None, None) == sn.SN_EINVAL
    assert lib.sn_mesh_view_get(None, None) == sn.SN_EINVAL
    assert lib.sn_serve_stop(None) == sn.SN_EINVAL
    assert lib.sn_triangulate(None, None, 0, None, None, None) == sn.SN_EINVAL
    assert b"NULL" in lib.sn_last_error() or lib.sn_last_error() != b""


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that the C compiler gives the header's struct of the same name."""
    import subprocess

    import paper_2401_14906_amd as sn

    structs = [sn.sn_volume, sn.sn_smooth_params, sn.sn_mesh_view, sn.sn_serve_config,
               sn.sn_serve_stats, sn.sn_kernel_stat]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sn.h"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, f"{name}.{f}"


def test_volume_checks_without_gpu(lib):
    """Volume validation (run by sn_noalloc_scratch_bytes, which needs no
    device): labels must be aligned to their dtype; sizes follow the dims."""
    import paper_2401_14906_amd as sn

    def vol(ptr, dtype, dims=(37, 20, 9)):
        v = sn.sn_volume()
        v.labels = ptr
        v.dtype = dtype
        v.dims[0], v.dims[1], v.dims[2] = dims
        v.spacing[0] = v.spacing[1] = v.spacing[2] = 1.0
        v.prim = sn.SN_QUADS
        return v

    base = 1 << 20  # never dereferenced: no compute call is made
    for dtype in (1, 2, 4):
        assert lib.sn_noalloc_scratch_bytes(ctypes.byref(vol(base + dtype, dtype))) > 0
        if dtype > 1:
            assert lib.sn_noalloc_scratch_bytes(ctypes.byref(vol(base + 1, dtype))) == -1
    assert lib.sn_noalloc_scratch_bytes(ctypes.byref(vol(base + 2, 4))) == -1
    assert b"aligned" in lib.sn_last_error()
