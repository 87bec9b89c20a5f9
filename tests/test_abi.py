"""The C-ABI library loads and exports every function include/amg.h declares.

No compute call is made here (these run without a GPU): only the pure-host
entry points (status strings, default parameters) are called.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg.h")


def _lib_path():
    from paper_0707_4018_amd import binding
    p = binding.lib_path()
    if not os.path.exists(p):
        from paper_0707_4018_amd import build
        build.build()
    return p


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(amg_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("amg_gauge_create", "amg_apply", "amg_setup", "amg_setup_adaptive", "amg_solve",
              "amg_cgnr_solve", "amg_vcycle", "amg_status_str"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_entry_points():
    from paper_0707_4018_amd import binding
    lib = binding.load_library(_lib_path())
    assert lib.amg_status_str(0) == b"ok"
    assert lib.amg_status_str(6).startswith(b"linearly dependent")
    p = binding._Params()
    lib.amg_default_params(ctypes.byref(p))
    assert p.nlevels == 2 and p.nvec[0] == 8 and p.block[0][0] == 4
    assert p.nu_pre == 2 and p.nu_post == 2 and abs(p.omega - 0.8) < 1e-15


def test_null_arguments_rejected_without_gpu_work():
    from paper_0707_4018_amd import binding
    lib = binding.load_library(_lib_path())
    out = ctypes.c_void_p()
    assert lib.amg_gauge_create(None, None, 0.0, None, ctypes.byref(out)) == 1
    assert lib.amg_solve(None, None, None, 1, 1e-10, 10, None, None) == 1
    lat = binding._Lattice()
    lat.nd = 3
    assert lib.amg_gauge_create(ctypes.byref(lat), ctypes.c_void_p(16), 0.0, None, ctypes.byref(out)) == 1
    assert b"nd" in lib.amg_last_error()


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_0707_4018_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
