"""The C-ABI library loads and exports every symbol include/rss.h declares (CPU only;
no compute calls: only argument-validation paths that return before any device work)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1609_08130_amd import rss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rss.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rss_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rss.load_library()
    names = _declared()
    assert set(names) == set(rss.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rss.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rss_[a-z_0-9]+)", out))
    assert set(names) <= exported


def test_params_layout_matches_c_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "rss.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu\\n", sizeof(rss_params), offsetof(rss_params, tol), '
                   'offsetof(rss_params, root_lo), offsetof(rss_params, root_side), '
                   'offsetof(rss_params, precision)); return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P = rss.Params
    assert vals == [ctypes.sizeof(P), P.tol.offset, P.root_lo.offset, P.root_side.offset, P.precision.offset]


def test_params_default_and_argument_errors():
    lib = rss.load_library()
    p = rss.Params()
    lib.rss_params_default(ctypes.byref(p))
    assert p.struct_size == ctypes.sizeof(rss.Params)
    assert (p.dim, p.diag, p.tol, p.leaf_size, p.n_proxy, p.proxy_radius) == (2, 1.0, 1e-6, 64, 16, 1.25)
    h = ctypes.c_void_p(123)
    fake = ctypes.c_void_p(1)   # never dereferenced: validation fails first
    bad = []
    for field, val in [("tol", -1.0), ("tol", float("nan")), ("leaf_size", 0), ("leaf_size", 1000),
                       ("n_proxy", 0), ("proxy_radius", 0.5), ("proxy_radius", 3.0), ("dim", 3)]:
        q = rss.Params()
        lib.rss_params_default(ctypes.byref(q))
        setattr(q, field, val)
        st = lib.rss_factor_create(fake, 100, ctypes.byref(q), None, ctypes.byref(h))
        bad.append((field, st))
        assert h.value is None
        assert lib.rss_last_error().decode() != ""
    assert all(st in (1, 5) for _, st in bad)
    q = rss.Params()
    lib.rss_params_default(ctypes.byref(q))
    assert lib.rss_factor_create(fake, 0, ctypes.byref(q), None, ctypes.byref(h)) == 1
    q.struct_size = 7
    assert lib.rss_factor_create(fake, 10, ctypes.byref(q), None, ctypes.byref(h)) == 1
    assert lib.rss_factor_destroy(None) == 0
    assert lib.rss_solve(None, None, None, 1, 1, 0, None) == 1


def test_binding_has_no_cpu_fallback():
    src = open(os.path.join(ROOT, "paper_1609_08130_amd", "rss.py")).read()
    assert "oracle" not in src
    assert "numpy.linalg" not in src and "np.linalg" not in src
