"""The C ABI library loads and exports every entry point include/ebic.h
declares; argument checks that happen before any device work.  No GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebic.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(ebic_[a-z_]+)\s*\((?!\s*\*)", src))
    # typedef'd callback types are not functions
    names -= set(re.findall(r"\(\s*\*\s*(ebic_[a-z_]+)\s*\)", src))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("ebic_create", "ebic_evaluate", "ebic_evaluate_device", "ebic_evolve",
                 "ebic_destroy", "ebic_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1801_03039_amd as e
    lib = ctypes.CDLL(e.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_mask_words():
    import paper_1801_03039_amd as e
    assert [e.mask_words(n) for n in (0, 1, 63, 64, 65, 128, 20000)] == [0, 1, 1, 1, 2, 2, 313]


def test_create_argument_errors_before_device_work():
    import numpy as np
    import paper_1801_03039_amd as e
    from paper_1801_03039_amd import binding as b
    h = ctypes.c_void_p()
    a = np.zeros((4, 3), dtype=np.float32)
    ptr = a.ctypes.data_as(ctypes.c_void_p)
    assert b._create(None, 4, 3, 3, 0, 0, ctypes.byref(h)) == b.EBIC_E_ARG
    assert b._create(ptr, 0, 3, 3, 0, 0, ctypes.byref(h)) == b.EBIC_E_ARG
    assert b._create(ptr, 4, 0, 3, 0, 0, ctypes.byref(h)) == b.EBIC_E_ARG
    assert b._create(ptr, 4, 3, 2, 0, 0, ctypes.byref(h)) == b.EBIC_E_ARG   # ld < n_cols
    assert b"leading dimension" in b._last_error(None)
    assert b._create(ptr, 4, 3, 3, 1, 0, ctypes.byref(h)) == b.EBIC_E_ARG   # col-major, ld < n_rows
    assert b"leading dimension" in b._last_error(None)
    assert b._create(ptr, 4, 3, 3, 7, 0, ctypes.byref(h)) == b.EBIC_E_ARG   # layout
    assert b"layout" in b._last_error(None)
    assert b._create(ptr, 4, 3, 3, 0, 0, None) == b.EBIC_E_ARG
    assert b"out is null" in b._last_error(None)
    assert b._evaluate(None, None, None, 1, None, None, None, None) == b.EBIC_E_ARG
    prm = e.make_params(1)
    assert b._evaluate_device(None, None, None, 1, 0, ctypes.byref(prm), None, None, None,
                              None) == b.EBIC_E_ARG
    assert b._destroy(None) == b.EBIC_OK
    assert b._set_path(None, 0) == b.EBIC_E_ARG


def test_one_hip_runtime_per_process():
    # The package must bind libebic to the HIP runtime torch already loaded
    # (same SONAME), never bring in a second one.
    import subprocess
    import sys
    code = ("import paper_1801_03039_amd as e\n"
            "e.Context  # loads libebic.so\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
            "print(len(libs), libs)\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("1 "), out.stdout
