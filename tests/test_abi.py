"""CPU checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made here; on a machine without a GPU, context creation
must fail cleanly with ENMF_EDEVICE instead of crashing.
"""

import ctypes
import os
import re

import pytest

from paper_2605_19325_amd import enmf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "enmf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(enmf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("enmf_svd_init", "enmf_rotate", "enmf_iterate", "enmf_objective_kkt",
                 "enmf_xv", "enmf_xtu", "enmf_gram", "enmf_convert", "enmf_create",
                 "enmf_serve_start", "enmf_enmc_init", "enmf_enmc_grad", "enmf_enmc_iterate",
                 "enmf_sparse_create", "enmf_sparse_destroy", "enmf_rotate_general"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = enmf.load_library()
    raw = ctypes.CDLL(enmf.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name
    # the binding declares the same set
    assert sorted(n for n, _, _ in enmf.SIGNATURES) == declared_functions()
    assert lib.enmf_version() >= 100


def test_status_strings():
    lib = enmf.load_library()
    assert lib.enmf_status_string(0) == b"ok"
    assert lib.enmf_status_string(1) == b"invalid argument"
    assert lib.enmf_status_string(99) == b"unknown status"


STRUCTS = [("enmf_matrix", enmf.Matrix), ("enmf_svd_opts", enmf.SvdOpts),
           ("enmf_rotate_opts", enmf.RotateOpts), ("enmf_iter_opts", enmf.IterOpts),
           ("enmf_iter_report", enmf.IterReport), ("enmf_kkt", enmf.Kkt),
           ("enmf_serve_opts", enmf.ServeOpts), ("enmf_request", enmf.Request),
           ("enmf_mask", enmf.MaskArg), ("enmf_grot_opts", enmf.GrotOpts)]


def test_struct_layouts_match_header(tmp_path):
    """Size and every field offset of the ctypes mirrors equal what a C
    compiler makes of include/enmf.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "enmf.h"', "int main(void) {"]
    for cname, py in STRUCTS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n"):
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in STRUCTS:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = enmf.load_library()
    h = ctypes.c_void_p()
    st = lib.enmf_create(ctypes.byref(h), 0, None)
    assert st == 3 and not h.value          # ENMF_EDEVICE, no context
    assert lib.enmf_last_error(None) == b"null context"
